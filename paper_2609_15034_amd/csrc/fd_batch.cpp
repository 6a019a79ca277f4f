// Batched decode: many columns of mixed codecs and offset widths in one stream
// submission (optionally one HIP graph), with an autotuner for tile sizes.
//
// A batch is split into groups of one codec and offset width.  Each group runs
// as one persistent kernel over a device table of per-column parameters; its
// tiles are numbered consecutively over its columns and taken from one
// counter, so every workgroup works through the group's columns in order and
// small columns cost no launch of their own.  The tile cursors come either from
// a decoupled look-back per column (mode 0) or from three phases per group
// (mode 1): the group's tile totals in global tile order, one scan over them,
// then the expand pass, each column's cursors taken relative to its first
// tile.  Each column keeps its own error word; a last one-workgroup kernel
// turns the error words into per-column statuses.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "fastdecode.h"
#include "fd_internal.h"

using namespace fd;

namespace {

constexpr int kMaxGroups = 6;          // (codec, offset width) pairs
constexpr size_t kBOffStatus = 128;    // the status word
constexpr size_t kBOffCounters = 256;  // a counter block (tile queues) per group
constexpr size_t kBHdr = kBOffCounters + kMaxGroups * kCounterBlockBytes;
static_assert(kBHdr % 256 == 0, "the column states start 256-byte aligned");
constexpr int32_t kMaxCols = 65536;

// Candidate tile sizes of the autotuner: fractions (percent) of the largest
// tile (smaller tiles: more tiles for the small columns and more parallel
// look-back, larger: fewer tiles and less overhead per byte).
constexpr int kScales[] = {100, 50, 25};
constexpr int kNumScales = 3;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Group {
    int codec = 0, index_bits = 0;
    std::vector<int32_t> cols;   // column indices (caller order)
    int64_t total = 0;           // tiles
    int64_t max_samples = 0;     // the largest coarse index sample count of its columns
    int grid = 0;
    size_t off_sum = 0;          // mode 1: tile totals, then cursors (total + 1 words)
    size_t off_gsum = 0;         // mode 1: block sums of their scan
};

struct BatchPlan {
    int mode = 0;                         // 0: look-back per column, 1: three phases per group
    std::vector<int64_t> tcodes, n_tiles; // per column
    std::vector<int> g_shift;             // per column
    std::vector<size_t> off_state;        // per column: tile aggregates, then block states
    std::vector<size_t> off_coarse;       // per column: its coarse string index
    std::vector<Group> groups;
    size_t states_end = 0;                // [0, states_end) is zeroed per call
    size_t off_errs = 0, off_table = 0, table_bytes = 0, bytes = 0;
};

int group_of(int codec, int index_bits) {
    return (codec == FD_FSST8 ? 0 : codec == FD_ONPAIR16 ? 2 : 4) + (index_bits == 64 ? 1 : 0);
}

// Host-visible checks of one column (those of the single-column entry points).
bool column_ok(const fd_column& c) {
    if (!c.dict) return false;
    const fd_codec codec = c.dict->codec;
    if (codec != FD_FSST8 && codec != FD_ONPAIR16 && codec != FD_ONPAIR12) return false;
    if (c.index_bits != 32 && c.index_bits != 64) return false;
    if (c.n_strings < 0 || c.n_codes < 0 || c.out_capacity < 0) return false;
    if (c.n_strings > (int64_t)1 << 40 || c.n_codes > (int64_t)1 << 40) return false;
    if (!c.code_offsets || !c.out_offsets) return false;
    if (c.n_codes > 0 && !c.codes) return false;
    if (c.out_capacity > 0 && !c.out_bytes) return false;
    if (codec == FD_ONPAIR16 && c.codes && ((uintptr_t)c.codes & 1)) return false;
    if (c.index_bits == 32 &&
        (c.n_codes > INT32_MAX || ((uintptr_t)c.code_offsets & 3) || ((uintptr_t)c.out_offsets & 3)))
        return false;
    if (c.index_bits == 64 && (((uintptr_t)c.code_offsets & 7) || ((uintptr_t)c.out_offsets & 7))) return false;
    return true;
}

// Plan of a batch for one tile-size choice: `tc_fixed` > 0 sets every
// column's codes per tile, else `scale` percent of the largest tile (rounded
// to whole chunks).
bool make_plan(const fd_column* cols, int32_t n, int64_t tc_fixed, int scale, int grid_req, int mode,
               BatchPlan* pl, int grid_pct = 100) {
    pl->mode = mode;
    pl->tcodes.assign(n, 0);
    pl->n_tiles.assign(n, 0);
    pl->g_shift.assign(n, 0);
    pl->off_state.assign(n, 0);
    pl->off_coarse.assign(n, 0);
    pl->groups.assign(kMaxGroups, Group());
    size_t off = kBHdr;
    for (int32_t c = 0; c < n; c++) {
        const fd_column& col = cols[c];
        const fd_codec codec = col.dict->codec;
        int64_t T = tc_fixed;
        if (T == 0) {
            const int64_t q = codes_per_chunk((int)codec);
            T = std::max<int64_t>(q, tile_codes_max(codec) * scale / 100 / q * q);
        }
        T = tile_codes_for(codec, T);
        if (T < 0) return false;
        const int64_t tiles = tiles_of(col.n_codes, T);
        if (tiles > (int64_t)UINT32_MAX / 4) return false;
        const int64_t tiles_pad = (tiles + kBlk - 1) / kBlk * kBlk;
        pl->tcodes[c] = T;
        pl->n_tiles[c] = tiles;
        pl->g_shift[c] = coarse_shift(col.n_codes, col.n_strings, T);
        pl->off_state[c] = off;
        if (mode == 0) off += (size_t)tiles_pad * 8 + (size_t)(tiles_pad / kBlk) * 8;
        pl->off_coarse[c] = off;
        off += (size_t)tiles * 8;
        Group& g = pl->groups[group_of((int)codec, col.index_bits)];
        g.codec = (int)codec;
        g.index_bits = col.index_bits;
        g.cols.push_back(c);
        g.total += tiles;
        g.max_samples = std::max(g.max_samples, (col.n_strings + ((int64_t)1 << pl->g_shift[c]) - 1) >> pl->g_shift[c]);
    }
    // inside a group, columns of one dictionary run back to back: a workgroup
    // then keeps its LDS table, and the dictionary stays warm in L2
    // (statuses stay per column, so the order is not visible)
    for (Group& g : pl->groups)
        std::stable_sort(g.cols.begin(), g.cols.end(),
                         [&](int32_t a, int32_t b) { return (uintptr_t)cols[a].dict < (uintptr_t)cols[b].dict; });
    if (mode == 1) {
        for (Group& g : pl->groups) {
            if (g.cols.empty()) continue;
            g.off_sum = off;
            off += (size_t)(g.total + 1) * 8;
            g.off_gsum = off;
            off += (size_t)((g.total + 1 + 1023) / 1024 + 1) * 8;
        }
    }
    pl->states_end = off;
    pl->off_errs = align_up(off, 256);
    pl->off_table = align_up(pl->off_errs + (size_t)n * 8, 256);
    // the table: every group's DecodeParams (group order), then every group's first-tile array
    size_t tb = (size_t)n * sizeof(DecodeParams);
    for (const Group& g : pl->groups) tb += (g.cols.size() + (g.cols.empty() ? 0 : 1)) * sizeof(int64_t);
    pl->table_bytes = tb;
    pl->bytes = align_up(pl->off_table + tb, 256);
    for (Group& g : pl->groups) {
        if (g.cols.empty()) continue;
        int grid = grid_req ? grid_req
                            : (int)((int64_t)resident_grid_batch(g.codec, g.index_bits,
                                                                 mode == 1 ? kModeExpand : kModeLookback) *
                                    grid_pct / 100);
        if ((int64_t)grid > g.total) grid = (int)g.total;
        g.grid = grid < 1 ? 1 : grid;
    }
    return true;
}

// Fill the host image of the device table.
void fill_table(const fd_column* cols, int32_t n, const BatchPlan& pl, uint8_t* ws, uint8_t* host) {
    DecodeParams* dp = (DecodeParams*)host;
    int64_t* ft = (int64_t*)(host + (size_t)n * sizeof(DecodeParams));
    int k = 0;
    for (int gi = 0; gi < kMaxGroups; gi++) {
        const Group& g = pl.groups[gi];
        if (g.cols.empty()) continue;
        int64_t first = 0;
        for (int32_t c : g.cols) {
            const fd_column& col = cols[c];
            DecodeParams p;
            memset(&p, 0, sizeof(p));
            p.codes = (const uint8_t*)col.codes;
            p.n_codes = col.n_codes;
            p.code_off = col.code_offsets;
            p.n_strings = col.n_strings;
            p.dict_bytes = col.dict->bytes;
            p.dict_lens = col.dict->lens;
            p.n_sym = col.dict->n;
            p.fsst_tab = col.dict->fsst_tab;
            p.fsst_len = col.dict->fsst_len;
            p.tok16 = col.dict->tok16;
            p.tok_len = col.dict->tok_len;
            p.out_off = col.out_offsets;
            p.out = col.out_bytes;
            p.out_cap = col.out_capacity;
            p.n_tiles = pl.n_tiles[c];
            p.tile_codes = pl.tcodes[c];
            p.g_shift = pl.g_shift[c];
            p.off_pref = offsets_prefetch_count(col.dict->codec, col.n_codes, col.n_strings, pl.tcodes[c],
                                                pl.g_shift[c]);
            p.coarse = (int64_t*)(ws + pl.off_coarse[c]);
            p.err = (unsigned long long*)(ws + pl.off_errs) + c;
            p.counters = nullptr;
            if (pl.mode == 1) {
                // the group's scanned totals from this column's first tile on
                p.tagg = (unsigned long long*)(ws + g.off_sum) + first;
                p.bstate = nullptr;
            } else {
                p.tagg = (unsigned long long*)(ws + pl.off_state[c]);
                const int64_t tiles_pad = (pl.n_tiles[c] + kBlk - 1) / kBlk * kBlk;
                p.bstate = p.tagg + tiles_pad;
            }
            dp[k++] = p;
            *ft++ = first;
            first += pl.n_tiles[c];
        }
        *ft++ = first;
    }
}

// Streams for the groups of a batch beyond the first, per (device, calling
// stream): each group's kernels run on a stream of their own, forked from and
// joined back into the caller's stream, so that a group's workgroups start as
// soon as the previous group's last ones leave the CUs, instead of after its
// whole launch.  At most kMaxAux calling streams get a set; batches on others
// run their groups one after another on the calling stream.
struct AuxSet {
    hipStream_t s[kMaxGroups - 1] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxGroups - 1] = {};
};
constexpr size_t kMaxAux = 64;
std::map<std::pair<int, hipStream_t>, AuxSet> g_aux;

AuxSet* aux_for(int dev, hipStream_t st) {
    const auto key = std::make_pair(dev, st);
    auto it = g_aux.find(key);
    if (it != g_aux.end()) return &it->second;
    if (g_aux.size() >= kMaxAux) return nullptr;
    AuxSet a;
    bool ok = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kMaxGroups - 1 && ok; i++) {
        ok = hipStreamCreateWithFlags(&a.s[i], hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&a.join[i], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        if (a.fork) (void)hipEventDestroy(a.fork);
        for (int i = 0; i < kMaxGroups - 1; i++) {
            if (a.s[i]) (void)hipStreamDestroy(a.s[i]);
            if (a.join[i]) (void)hipEventDestroy(a.join[i]);
        }
        return nullptr;
    }
    return &(g_aux[key] = a);
}

// Enqueue a planned batch whose table image is in pinned memory `host`;
// `copied` (optional) is recorded once the image has been copied.
hipError_t enqueue(const fd_column* cols, int32_t n, const BatchPlan& pl, uint8_t* ws, const uint8_t* host,
                   int32_t* status, hipStream_t st, int dev, hipEvent_t copied = nullptr) {
    hipError_t e = hipMemcpyAsync(ws + pl.off_table, host, pl.table_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    if (copied && (e = hipEventRecord(copied, st)) != hipSuccess) return e;
    unsigned long long* errs = (unsigned long long*)(ws + pl.off_errs);
    e = launch_batch_reset((unsigned long long*)ws, (int64_t)(pl.states_end / 8), errs, n, st);
    if (e != hipSuccess) return e;
    const DecodeParams* dp = (const DecodeParams*)(ws + pl.off_table);
    const int64_t* ft = (const int64_t*)(ws + pl.off_table + (size_t)n * sizeof(DecodeParams));
    // the groups' places in the table, and their launch order: the most
    // tiles first (the smaller groups then fill the larger one's tail)
    int first_col[kMaxGroups], first_ft[kMaxGroups], order[kMaxGroups], ng = 0;
    for (int gi = 0, k = 0, f = 0; gi < kMaxGroups; gi++) {
        const Group& g = pl.groups[gi];
        first_col[gi] = k;
        first_ft[gi] = f;
        if (g.cols.empty()) continue;
        k += (int)g.cols.size();
        f += (int)g.cols.size() + 1;
        order[ng++] = gi;
    }
    std::stable_sort(order, order + ng, [&](int a, int b) { return pl.groups[a].total > pl.groups[b].total; });
    AuxSet* aux = ng > 1 ? aux_for(dev, st) : nullptr;
    if (aux && (e = hipEventRecord(aux->fork, st)) != hipSuccess) return e;
    for (int o = 0; o < ng; o++) {
        const int gi = order[o];
        const Group& g = pl.groups[gi];
        hipStream_t gs = (aux && o > 0) ? aux->s[o - 1] : st;
        if (gs != st && (e = hipStreamWaitEvent(gs, aux->fork, 0)) != hipSuccess) return e;
        unsigned* ctr = (unsigned*)(ws + kBOffCounters + kCounterBlockBytes * gi);
        const int32_t nc = (int32_t)g.cols.size();
        const DecodeParams* gdp = dp + first_col[gi];
        const int64_t* gft = ft + first_ft[gi];
        e = launch_coarse_batch(g.index_bits, gdp, nc, g.max_samples, gs);
        if (e != hipSuccess) return e;
        if (pl.mode == 1) {
            unsigned long long* sum = (unsigned long long*)(ws + g.off_sum);
            e = launch_tile_totals_batch(g.codec, g.index_bits, gdp, gft, nc, g.total, sum, dev_cus(), gs);
            if (e != hipSuccess) return e;
            e = launch_scan_multi(sum, g.total + 1, (unsigned long long*)(ws + g.off_gsum), gs);
            if (e != hipSuccess) return e;
            e = launch_decode_batch(g.codec, g.index_bits, kModeExpand, gdp, gft, nc, g.total, ctr, g.grid, gs);
        } else {
            e = launch_decode_batch(g.codec, g.index_bits, kModeLookback, gdp, gft, nc, g.total, ctr, g.grid, gs);
        }
        if (e != hipSuccess) return e;
        if (gs != st && (e = hipEventRecord(aux->join[o - 1], gs)) != hipSuccess) return e;
    }
    for (int o = 1; aux && o < ng; o++)
        if ((e = hipStreamWaitEvent(st, aux->join[o - 1], 0)) != hipSuccess) return e;
    (void)cols;
    return launch_batch_status(errs, n, status, (int32_t*)(ws + kBOffStatus), st);
}

// ---- pinned staging for the table image: a ring per device, each buffer
// reused once the copy that read it is done (not the whole batch), so that
// the host prepares the next batch while earlier ones run ----
constexpr int kRing = 8;
struct Staging {
    uint8_t* buf = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

// ---- caches: autotuned choice per batch shape, graphs per exact batch ----
// A graph is reused only for a batch equal to the one it was recorded for in
// every field the recording depends on: each column's dictionary (by its
// unique id, never its address), codec, buffers and sizes, the workspace,
// status pointer, tiling, mode, grid and device.  The hash only narrows the
// search; the full key is compared.
struct GraphKey {
    std::vector<uint64_t> words;
    uint64_t hash = 0;
    bool operator==(const GraphKey& o) const { return hash == o.hash && words == o.words; }
};

struct GraphEntry {
    GraphKey key;
    int device = 0;
    hipGraphExec_t exec = nullptr;
    uint8_t* pinned = nullptr;
};

std::mutex g_bmu;
Staging g_stage[64][kRing];
int g_stage_next[64];
// the autotuner's choice for a batch shape
struct Choice {
    int mode = 0, scale = 100, grid_pct = 100;
    bool from_file = false;
};
std::unordered_map<uint64_t, Choice> g_tuned;               // shape (and device) -> choice
bool g_tuned_file_read = false;                             // the persisted choices, read once
std::list<GraphEntry> g_graphs;                             // most recent first
hipStream_t g_capture[64];                                  // per device: the stream graphs are recorded on
constexpr size_t kMaxGraphs = 16;
int g_hash_bits = 64;                                       // testing: fewer bits force collisions

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

int log2_bucket(int64_t x) { return x <= 0 ? 0 : 64 - __builtin_clzll((uint64_t)x); }

uint64_t shape_key(const fd_column* cols, int32_t n, int dev) {
    uint64_t h = mix(0x5eed, (uint64_t)n);
    h = mix(h, (uint64_t)dev);
    for (int32_t c = 0; c < n; c++) {
        h = mix(h, (uint64_t)cols[c].dict->codec);
        h = mix(h, (uint64_t)cols[c].index_bits);
        h = mix(h, (uint64_t)log2_bucket(cols[c].n_strings));
        h = mix(h, (uint64_t)log2_bucket(cols[c].n_codes));
    }
    return h;
}

GraphKey exact_key(const fd_column* cols, int32_t n, const void* ws, size_t ws_bytes, const int32_t* status,
                   int64_t tc_fixed, int scale, int grid, int dev) {
    GraphKey k;
    std::vector<uint64_t>& w = k.words;
    w.reserve(8 + (size_t)n * 10);
    w.push_back((uint64_t)n);
    w.push_back((uint64_t)dev);
    w.push_back((uint64_t)(uintptr_t)ws);
    w.push_back((uint64_t)ws_bytes);
    w.push_back((uint64_t)(uintptr_t)status);
    w.push_back((uint64_t)tc_fixed);
    w.push_back((uint64_t)scale);
    w.push_back((uint64_t)(int64_t)grid);
    for (int32_t c = 0; c < n; c++) {
        const fd_column& col = cols[c];
        w.push_back(col.dict->id);
        w.push_back((uint64_t)col.dict->codec);
        w.push_back((uint64_t)(uintptr_t)col.codes);
        w.push_back((uint64_t)col.n_codes);
        w.push_back((uint64_t)(uintptr_t)col.code_offsets);
        w.push_back((uint64_t)(int64_t)col.index_bits);
        w.push_back((uint64_t)col.n_strings);
        w.push_back((uint64_t)(uintptr_t)col.out_offsets);
        w.push_back((uint64_t)(uintptr_t)col.out_bytes);
        w.push_back((uint64_t)col.out_capacity);
    }
    uint64_t h = 0x9a9a;
    for (uint64_t x : w) h = mix(h, x);
    k.hash = g_hash_bits >= 64 ? h : (g_hash_bits <= 0 ? 0 : (h & ((1ull << g_hash_bits) - 1)));
    return k;
}

void destroy_graph(GraphEntry& ge) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.pinned) (void)hipHostFree(ge.pinned);
    ge.exec = nullptr;
    ge.pinned = nullptr;
}

// Plan and enqueue one batch decode (no graph), staging the table in pinned memory.
fd_status run_once(const fd_column* cols, int32_t n, const BatchPlan& pl, uint8_t* ws, int32_t* status,
                   hipStream_t st, int dev) {
    Staging& sg = g_stage[dev][g_stage_next[dev]];
    g_stage_next[dev] = (g_stage_next[dev] + 1) % kRing;
    if (sg.pending) {
        if (hipEventSynchronize(sg.done) != hipSuccess) return FD_EHIP;
        sg.pending = false;
    }
    if (sg.cap < pl.table_bytes) {
        if (sg.buf) (void)hipHostFree(sg.buf);
        sg.buf = nullptr;
        sg.cap = 0;
        const size_t cap = std::max<size_t>(pl.table_bytes, 64 * 1024);
        if (hipHostMalloc((void**)&sg.buf, cap, hipHostMallocDefault) != hipSuccess) return FD_ENOMEM;
        sg.cap = cap;
    }
    if (!sg.done && hipEventCreateWithFlags(&sg.done, hipEventDisableTiming) != hipSuccess) return FD_EHIP;
    fill_table(cols, n, pl, ws, sg.buf);
    if (enqueue(cols, n, pl, ws, sg.buf, status, st, dev, sg.done) != hipSuccess) return FD_EHIP;
    sg.pending = true;
    return FD_OK;
}

// Autotune.  Candidates: mode (look-back or three phases) x tile size (100,
// 50, 25% of the largest) x resident workgroups (all, or three quarters: the
// look-back's waits on other tiles can favour fewer workgroups per CU).  A
// residency model prunes them before any is timed (the paper's performance
// model: a launch keeps R = CUs x workgroups-per-CU tiles in flight, set by
// the kernel's registers and LDS): a smaller tile size is tried only while
// the larger one leaves some group with fewer than 2 R tiles (too few to
// fill the device twice over), and fewer workgroups only for the look-back
// and only on groups of at least 2 R tiles.  Each survivor runs once to warm
// up and twice timed; the fastest is kept.
fd_status autotune(const fd_column* cols, int32_t n, uint8_t* ws, size_t ws_bytes, hipStream_t st, int dev,
                   Choice* best_out, int* n_timed) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return FD_EHIP;
    float best = 1e30f;
    Choice best_c;
    fd_status rc = FD_OK;
    *n_timed = 0;
    for (int mode = 0; mode < 2 && rc == FD_OK; mode++) {
        bool larger_fills = false;          // the previous (larger) tile size gave every group >= 2 R tiles
        for (int si = 0; si < kNumScales && rc == FD_OK; si++) {
            const int scale = kScales[si];
            BatchPlan pl;
            if (!make_plan(cols, n, 0, scale, 0, mode, &pl) || pl.bytes > ws_bytes) continue;
            if (si > 0 && larger_fills) break;
            bool fills = true, big = false;
            for (const Group& g : pl.groups) {
                if (g.cols.empty()) continue;
                const int64_t R = resident_grid_batch(g.codec, g.index_bits, mode == 1 ? kModeExpand : kModeLookback);
                fills = fills && g.total >= 2 * R;
                big = big || g.total >= 2 * R;
            }
            larger_fills = fills;
            for (int gp : {100, 75}) {
                if (gp != 100 && (mode != 0 || !big)) continue;
                BatchPlan pg;
                if (!make_plan(cols, n, 0, scale, 0, mode, &pg, gp)) continue;
                float ms_sum = 0.f;
                for (int rep = 0; rep < 3 && rc == FD_OK; rep++) {
                    if (hipEventRecord(a, st) != hipSuccess) { rc = FD_EHIP; break; }
                    rc = run_once(cols, n, pg, ws, nullptr, st, dev);
                    if (rc != FD_OK) break;
                    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
                        rc = FD_EHIP;
                        break;
                    }
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) { rc = FD_EHIP; break; }
                    if (rep > 0) ms_sum += ms;
                }
                *n_timed += 1;
                if (rc == FD_OK && ms_sum < best) {
                    best = ms_sum;
                    best_c.mode = mode;
                    best_c.scale = scale;
                    best_c.grid_pct = gp;
                }
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *best_out = best_c;
    return rc;
}

// The persisted choices: with FD_AUTOTUNE_CACHE naming a file, the choices
// found by timing are appended to it, one line each
//   fastdecode-autotune 1 <key, 16 hex digits> <mode> <tile %> <workgroup %>
// and read back by later processes; the key hashes the batch shape and the
// device's architecture name and CU count (not its ordinal).
uint64_t device_key(int dev) {
    static uint64_t keys[64];
    if (!keys[dev]) {
        hipDeviceProp_t prop;
        uint64_t h = 0xd1ce;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            for (const char* c = prop.gcnArchName; *c; c++) h = mix(h, (uint64_t)(unsigned char)*c);
            h = mix(h, (uint64_t)prop.multiProcessorCount);
        }
        keys[dev] = h | 1;
    }
    return keys[dev];
}

uint64_t persist_key(const fd_column* cols, int32_t n, int dev) {
    return mix(shape_key(cols, n, 0), device_key(dev));
}

void read_tuned_file() {
    g_tuned_file_read = true;
    const char* path = getenv("FD_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char tag[32];
    int ver = 0, mode = 0, scale = 0, gp = 0;
    unsigned long long key = 0;
    while (fscanf(f, "%31s %d %llx %d %d %d", tag, &ver, &key, &mode, &scale, &gp) == 6) {
        if (strcmp(tag, "fastdecode-autotune") != 0 || ver != 1) continue;
        const bool ok_scale = std::find(std::begin(kScales), std::end(kScales), scale) != std::end(kScales);
        if ((mode != 0 && mode != 1) || !ok_scale || (gp != 100 && gp != 75)) continue;
        Choice c;
        c.mode = mode;
        c.scale = scale;
        c.grid_pct = gp;
        c.from_file = true;
        g_tuned[(uint64_t)key] = c;
    }
    fclose(f);
}

void write_tuned(uint64_t key, const Choice& c) {
    const char* path = getenv("FD_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "fastdecode-autotune 1 %016llx %d %d %d\n", (unsigned long long)key, c.mode, c.scale, c.grid_pct);
    fclose(f);
}

// The choice for a batch: cached (in memory, or from the file), else timed.
// `source`: 0 timed now, 1 from this process's cache, 2 read from the file.
fd_status choose(const fd_column* cols, int32_t n, uint8_t* ws, size_t ws_bytes, hipStream_t st, int dev, Choice* c,
                 int* source, int* n_timed) {
    if (!g_tuned_file_read) read_tuned_file();
    const uint64_t key = persist_key(cols, n, dev);
    *n_timed = 0;
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
        *c = it->second;
        *source = c->from_file ? 2 : 1;
        return FD_OK;
    }
    const fd_status rc = autotune(cols, n, ws, ws_bytes, st, dev, c, n_timed);
    if (rc != FD_OK) return rc;
    g_tuned[key] = *c;
    write_tuned(key, *c);
    *source = 0;
    return FD_OK;
}

fd_status read_status(uint8_t* ws, hipStream_t st) {
    if (hipStreamSynchronize(st) != hipSuccess) return FD_EHIP;
    int32_t hs = 0;
    if (hipMemcpy(&hs, ws + kBOffStatus, sizeof(hs), hipMemcpyDeviceToHost) != hipSuccess) return FD_EHIP;
    return (fd_status)hs;
}

}  // namespace

namespace fd {

void batch_forget_dict(uint64_t dict_id, int device) {
    std::lock_guard<std::mutex> lk(g_bmu);
    bool synced = false;
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        bool uses = false;
        const std::vector<uint64_t>& w = it->key.words;
        for (size_t i = 8; i < w.size(); i += 10)       // per column: the dictionary id first
            if (w[i] == dict_id) { uses = true; break; }
        if (uses) {
            if (!synced) {
                // a replay of it may still run: wait before freeing what it reads
                int cur = 0;
                (void)hipGetDevice(&cur);
                if (cur != device) (void)hipSetDevice(device);
                (void)hipDeviceSynchronize();
                if (cur != device) (void)hipSetDevice(cur);
                synced = true;
            }
            destroy_graph(*it);
            it = g_graphs.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace fd

extern "C" {

fd_status fd_debug_graph_hash_bits(int32_t bits) {
    if (bits < 0 || bits > 64) return FD_EINVAL;
    std::lock_guard<std::mutex> lk(g_bmu);
    g_hash_bits = bits;
    return FD_OK;
}

int32_t fd_debug_graph_count(void) {
    std::lock_guard<std::mutex> lk(g_bmu);
    return (int32_t)g_graphs.size();
}

fd_status fd_batch_autotune(const fd_column* cols, int32_t n_cols, void* workspace, size_t workspace_bytes,
                            void* hip_stream, fd_batch_choice* out) {
    try {
        if (!out || n_cols <= 0 || n_cols > kMaxCols || !cols) return FD_EINVAL;
        if (!workspace || ((uintptr_t)workspace & 255)) return FD_EINVAL;
        for (int32_t c = 0; c < n_cols; c++)
            if (!column_ok(cols[c])) return FD_EINVAL;
        size_t need = 0;
        if (fd_batch_workspace_size(cols, n_cols, nullptr, &need) != FD_OK || workspace_bytes < need) return FD_EINVAL;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FD_EHIP;
        std::lock_guard<std::mutex> lk(g_bmu);
        Choice c;
        int source = 0, n_timed = 0;
        const fd_status rc = choose(cols, n_cols, (uint8_t*)workspace, workspace_bytes, (hipStream_t)hip_stream, dev,
                                    &c, &source, &n_timed);
        if (rc != FD_OK) return rc;
        if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return FD_EHIP;
        out->mode = c.mode;
        out->tile_scale_pct = c.scale;
        out->grid_pct = c.grid_pct;
        out->source = source;
        out->candidates_timed = n_timed;
        return FD_OK;
    } catch (...) {
        return FD_ENOMEM;
    }
}

fd_status fd_debug_autotune_forget(void) {
    std::lock_guard<std::mutex> lk(g_bmu);
    g_tuned.clear();
    g_tuned_file_read = false;
    return FD_OK;
}

fd_status fd_batch_workspace_size(const fd_column* cols, int32_t n_cols, const fd_tuning* tuning, size_t* bytes) {
    if (!bytes || n_cols < 0 || n_cols > kMaxCols || (n_cols > 0 && !cols)) return FD_EINVAL;
    for (int32_t c = 0; c < n_cols; c++)
        if (!column_ok(cols[c])) return FD_EINVAL;
    if (tuning && ((tuning->mode != 0 && tuning->mode != 1) || tuning->tile_codes < 0 || tuning->grid < 0))
        return FD_EINVAL;
    size_t need = kBHdr;
    for (int i = 0; i < (tuning ? 1 : 2 * kNumScales); i++) {
        BatchPlan pl;
        const int mode = tuning ? tuning->mode : i / kNumScales;
        if (!make_plan(cols, n_cols, tuning ? tuning->tile_codes : 0, tuning ? 100 : kScales[i % kNumScales], 1,
                       mode, &pl))
            return FD_EINVAL;
        need = std::max(need, pl.bytes);
    }
    *bytes = need;
    return FD_OK;
}

fd_status batch_decode(const fd_column* cols, int32_t n_cols, const fd_tuning* tuning, void* workspace,
                       size_t workspace_bytes, int32_t* status, unsigned flags, void* hip_stream) {
    try {
        if (n_cols < 0 || n_cols > kMaxCols || (n_cols > 0 && !cols)) return FD_EINVAL;
        if (!workspace || ((uintptr_t)workspace & 255)) return FD_EINVAL;
        if ((flags & FD_ASYNC) && !status) return FD_EINVAL;
        if (flags & ~(FD_ASYNC | FD_GRAPH)) return FD_EINVAL;
        if (tuning && ((tuning->mode != 0 && tuning->mode != 1) || tuning->tile_codes < 0 || tuning->grid < 0))
            return FD_EINVAL;
        for (int32_t c = 0; c < n_cols; c++)
            if (!column_ok(cols[c])) return FD_EINVAL;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FD_EHIP;
        hipStream_t st = (hipStream_t)hip_stream;
        uint8_t* ws = (uint8_t*)workspace;
        if (n_cols == 0) {
            if (status && hipMemsetAsync(status, 0, sizeof(int32_t), st) != hipSuccess) return FD_EHIP;
            if (!(flags & FD_ASYNC) && hipStreamSynchronize(st) != hipSuccess) return FD_EHIP;
            return FD_OK;
        }

        std::lock_guard<std::mutex> lk(g_bmu);
        // the tile-size choice
        int64_t sb_fixed = tuning ? tuning->tile_codes : 0;
        int grid = tuning ? tuning->grid : 0;
        int scale = 100, mode = tuning ? tuning->mode : 0, grid_pct = 100;
        if (!tuning) {
            Choice c;
            int source = 0, n_timed = 0;
            const fd_status rc = choose(cols, n_cols, ws, workspace_bytes, st, dev, &c, &source, &n_timed);
            if (rc != FD_OK) return rc;
            mode = c.mode;
            scale = c.scale;
            grid_pct = c.grid_pct;
        }
        BatchPlan pl;
        if (!make_plan(cols, n_cols, sb_fixed, scale, grid, mode, &pl, grid_pct)) return FD_EINVAL;
        if (workspace_bytes < pl.bytes) return FD_EINVAL;

        if (flags & FD_GRAPH) {
            GraphKey key =
                exact_key(cols, n_cols, workspace, workspace_bytes, status, sb_fixed, mode * 1000 + scale,
                          grid ? grid : -grid_pct, dev);
            GraphEntry* ge = nullptr;
            for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it) {
                if (it->key == key) {
                    g_graphs.splice(g_graphs.begin(), g_graphs, it);
                    ge = &g_graphs.front();
                    break;
                }
            }
            if (!ge) {
                GraphEntry ne;
                ne.key = std::move(key);
                ne.device = dev;
                if (hipHostMalloc((void**)&ne.pinned, pl.table_bytes, hipHostMallocDefault) != hipSuccess)
                    return FD_ENOMEM;
                fill_table(cols, n_cols, pl, ws, ne.pinned);
                // recorded on the device's capture stream (kept: its group
                // streams are cached per calling stream)
                hipStream_t& cs = g_capture[dev];
                hipGraph_t graph = nullptr;
                bool ok = cs || hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
                ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    const bool enq = enqueue(cols, n_cols, pl, ws, ne.pinned, status, cs, dev) == hipSuccess;
                    ok = hipStreamEndCapture(cs, &graph) == hipSuccess && enq;
                }
                ok = ok && hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0) == hipSuccess;
                if (graph) (void)hipGraphDestroy(graph);
                if (!ok) {
                    destroy_graph(ne);
                    return FD_EHIP;
                }
                g_graphs.push_front(std::move(ne));
                ge = &g_graphs.front();
                while (g_graphs.size() > kMaxGraphs) {
                    // a graph launched earlier may still run: wait before freeing what it reads
                    (void)hipDeviceSynchronize();
                    destroy_graph(g_graphs.back());
                    g_graphs.pop_back();
                }
            }
            if (hipGraphLaunch(ge->exec, st) != hipSuccess) return FD_EHIP;
        } else {
            const fd_status rc = run_once(cols, n_cols, pl, ws, status, st, dev);
            if (rc != FD_OK) return rc;
        }
        if (flags & FD_ASYNC) return FD_OK;
        return read_status(ws, st);
    } catch (...) {
        return FD_ENOMEM;
    }
}

}  // extern "C"
