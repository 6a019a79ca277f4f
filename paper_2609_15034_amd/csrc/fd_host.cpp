// Host runtime behind the C ABI: argument validation, workspace layout,
// launch planning, device-resident dictionaries and status reporting.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>

#include "fastdecode.h"
#include "fd_internal.h"

using namespace fd;

namespace fd {

int64_t codes_per_pass(fd_codec c) {
    const int codec = (int)c;
    return (int64_t)kWG * chunks_per_lane(codec) * codes_per_chunk(codec);
}

int64_t tile_codes_max(fd_codec c) { return c == FD_FSST8 ? kTileMaxFsst : kTileMaxOnpair; }

int64_t tile_codes_for(fd_codec c, int64_t requested) {
    const int64_t mx = tile_codes_max(c), q = codes_per_chunk((int)c);
    if (requested == 0) return mx;
    if (requested < q || requested > mx || requested % q) return -1;
    return requested;
}

int64_t tiles_of(int64_t n_codes, int64_t tile_codes) {
    const int64_t t = (n_codes + tile_codes - 1) / tile_codes;
    return t < 1 ? 1 : t;
}

int offsets_prefetch_count(fd_codec c, int64_t n_codes, int64_t n_strings, int64_t tile_codes, int g_shift) {
    const int cap = c == FD_FSST8 ? kWG : 4 * kWG;
    const double spt = n_codes > 0 ? (double)tile_codes * (double)n_strings / (double)n_codes : (double)cap;
    const double want = 1.25 * spt + (double)((int64_t)1 << g_shift) + 2.0;
    int k = want >= (double)cap ? cap : (int)want;
    k = (k + 63) / 64 * 64;
    return k < 64 ? 64 : (k > cap ? cap : k);
}

int coarse_shift(int64_t n_codes, int64_t n_strings, int64_t tile_codes) {
    const double spt = n_codes > 0 ? (double)tile_codes * (double)n_strings / (double)n_codes : 4096.0;
    int sh = kCoarseShiftMin;
    while (sh < kCoarseShiftMax && (double)((int64_t)2 << sh) <= spt / 2.0) sh++;
    return sh;
}

namespace {
struct DevInfo {
    int cus = 0;
    int occ[5][2][3] = {};  // [codec id 1..4][index64][mode]
    int bocc[4][2][2] = {}; // batch kernels: [codec id 1..3][index64][expand]
};
std::mutex g_mu;
DevInfo g_dev[64];

DevInfo& dev_info(int* dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (dev_out) *dev_out = dev;
    DevInfo& d = g_dev[dev];
    if (!d.cus) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 1;
        d.cus = v;
    }
    return d;
}
}  // namespace

int dev_cus() {
    std::lock_guard<std::mutex> lk(g_mu);
    return dev_info(nullptr).cus;
}

int resident_grid(int codec, int index_bits, int mode) {
    std::lock_guard<std::mutex> lk(g_mu);
    DevInfo& d = dev_info(nullptr);
    int& o = d.occ[codec][index_bits == 64][mode];
    if (!o) o = decode_occupancy(codec, index_bits, mode);
    return d.cus * o;
}

int resident_grid_batch(int codec, int index_bits, int mode) {
    std::lock_guard<std::mutex> lk(g_mu);
    DevInfo& d = dev_info(nullptr);
    int& o = d.bocc[codec][index_bits == 64][mode == kModeExpand];
    if (!o) o = batch_occupancy(codec, index_bits, mode);
    return d.cus * o;
}

}  // namespace fd

namespace {

// workspace header: the error word, status words, then the counter block
constexpr size_t kOffErr = 0;
constexpr size_t kOffStatus = 16;
constexpr size_t kOffBadFlag = 20;
constexpr size_t kOffCounters = 256;
constexpr size_t kHdr = kOffCounters + kCounterBlockBytes;
static_assert(kHdr % 256 == 0, "the tile words start 256-byte aligned");
constexpr size_t kTok16Bytes = 65536 * 16;
constexpr size_t kTokLenBytes = 65536;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Plan {
    int64_t T;          // codes per tile
    int64_t n_tiles;
    int64_t n_blocks;
    int g_shift;        // coarse string index stride (log2)
    size_t off_tiles;   // n_tiles + 1 tile words
    size_t off_blocks;  // look-back block states
    size_t off_coarse;  // coarse string index, one word per tile
    size_t off_scan;    // three-phase mode: block sums of the cursor scan
    size_t off_dict;    // OnPair: prepared dictionary for the one-shot entry point
    size_t bytes;
};

bool plan_for(fd_codec codec, int64_t n_codes, int64_t n_strings, const fd_tuning* tu, Plan* pl) {
    if (n_codes < 0 || n_strings < 0) return false;
    if (codec != FD_FSST8 && codec != FD_ONPAIR16 && codec != FD_ONPAIR12) return false;
    const int64_t T = tile_codes_for(codec, tu ? tu->tile_codes : 0);
    if (T < 0) return false;
    pl->T = T;
    pl->n_tiles = tiles_of(n_codes, T);
    if (pl->n_tiles > (int64_t)UINT32_MAX / 2) return false;   // tile ids are 32-bit
    pl->n_blocks = (pl->n_tiles + kBlk - 1) / kBlk;
    pl->g_shift = coarse_shift(n_codes, n_strings, T);
    pl->off_tiles = kHdr;
    // n_tiles + 1 tile words (the three-phase scan leaves the decoded total in
    // the last), the block states and the coarse index, contiguous: one
    // zeroing covers them
    pl->off_blocks = pl->off_tiles + (size_t)(pl->n_tiles + 1) * 8;
    pl->off_coarse = pl->off_blocks + (size_t)pl->n_blocks * 8;
    pl->off_scan = pl->off_coarse + (size_t)pl->n_tiles * 8;
    pl->off_dict = align_up(pl->off_scan + (size_t)((pl->n_tiles + 1 + 1023) / 1024 + 1) * 8, 256);
    pl->bytes = pl->off_dict + (codec == FD_ONPAIR16 ? align_up(kTok16Bytes + kTokLenBytes, 256) : 0);
    return true;
}

fd_status hip_fail() { return FD_EHIP; }

// Selective decode: the workspace holds the decode plan of the compacted
// column (its tile words and block states after the header), the per-1,024-row
// code counts, the compacted code offsets and the compacted codes.
struct TakePlan {
    Plan dec;              // tiling of the compacted column (n_rows strings)
    fd_codec codec2;       // codec of the compacted codes (12-bit codes are widened to 16)
    int64_t nblk;
    size_t off_bsum, off_noff, off_src, off_codes, bytes;
};

bool take_plan_for(fd_codec codec, int64_t n_codes, int64_t n_strings, int64_t n_rows, int64_t max_codes,
                   const fd_tuning* tu, TakePlan* tp) {
    if (n_codes < 0 || n_strings < 0 || n_rows < 0 || max_codes < 0) return false;
    if (n_rows > (int64_t)1 << 40 || max_codes > (int64_t)1 << 40) return false;
    if (codec != FD_FSST8 && codec != FD_ONPAIR16 && codec != FD_ONPAIR12) return false;
    if (tu && tu->mode != 0 && tu->mode != 1) return false;
    tp->codec2 = codec == FD_ONPAIR12 ? FD_ONPAIR16 : codec;
    // tiles over the compacted buffer of max_codes codes (the tiles past the
    // selection's codes are skipped on the device); the coarse index stride
    // from the column's mean codes per string (the rows are a sample of it)
    if (!plan_for(tp->codec2, max_codes, n_rows, tu, &tp->dec)) return false;
    const double mean = n_strings ? (double)n_codes / (double)n_strings : 1.0;
    tp->dec.g_shift = coarse_shift((int64_t)(mean * (double)n_rows) + 1, n_rows, tp->dec.T);
    tp->nblk = n_rows > 0 ? (n_rows + 1023) / 1024 : 1;
    tp->off_bsum = tp->dec.off_dict;                                   // no dictionary repack here
    tp->off_noff = align_up(tp->off_bsum + (size_t)(tp->nblk + 1) * 8, 256);
    tp->off_src = align_up(tp->off_noff + (size_t)(n_rows + 1) * 8, 256);
    tp->off_codes = align_up(tp->off_src + (size_t)n_rows * 8, 256);
    const size_t w = tp->codec2 == FD_FSST8 ? 1 : 2;
    tp->bytes = align_up(tp->off_codes + (size_t)max_codes * w + 64, 256);
    return true;
}

struct Args {
    fd_codec codec;
    const void* codes;
    int64_t n_codes;
    const void* code_off;
    int index_bits;
    int64_t n_strings;
    // raw dictionary (one-shot) or prepared handle
    const uint8_t* dict_bytes;
    const uint8_t* dict_lens;
    int32_t n_dict;
    const fd_dict* dict;
    void* out_off;
    uint8_t* out;
    int64_t out_cap;
    void* ws;
    size_t ws_bytes;
    int32_t* status;
    unsigned flags;
    const fd_tuning* tuning;
    hipStream_t stream;
    // persisted output positions: 0 none, 1 build them (no output), 2 decode with them
    int sidecar_op;
    int64_t* sidecar;
    int64_t sidecar_n;
};

constexpr int kSidecarBuild = 1;
constexpr int kSidecarDecode = 2;

fd_status run_decode(const Args& a) {
    // ---------------- host-side validation ----------------
    if (a.index_bits != 32 && a.index_bits != 64) return FD_EINVAL;
    if (a.n_strings < 0 || a.n_codes < 0 || a.out_cap < 0) return FD_EINVAL;
    if (a.n_strings > (int64_t)1 << 40 || a.n_codes > (int64_t)1 << 40) return FD_EINVAL;
    const bool build = a.sidecar_op == kSidecarBuild;        // no decoded output
    if (!a.code_off || (!build && !a.out_off) || !a.ws) return FD_EINVAL;
    if (a.n_codes > 0 && !a.codes) return FD_EINVAL;
    if (a.out_cap > 0 && !a.out) return FD_EINVAL;
    if ((a.flags & FD_ASYNC) && !a.status) return FD_EINVAL;
    if (a.codec == FD_ONPAIR16 && a.codes && ((uintptr_t)a.codes & 1)) return FD_EINVAL;
    if (a.index_bits == 32 && (a.n_codes > INT32_MAX || ((uintptr_t)a.code_off & 3) || ((uintptr_t)a.out_off & 3)))
        return FD_EINVAL;
    if (a.index_bits == 64 && (((uintptr_t)a.code_off & 7) || ((uintptr_t)a.out_off & 7))) return FD_EINVAL;
    if ((uintptr_t)a.ws & 255) return FD_EINVAL;
    const int mode_sel = a.tuning ? a.tuning->mode : 0;
    if (mode_sel != 0 && mode_sel != 1) return FD_EINVAL;
    if (a.sidecar_op && (mode_sel != 0 || !a.dict || !a.sidecar || ((uintptr_t)a.sidecar & 7))) return FD_EINVAL;
    if (a.tuning && a.tuning->grid < 0) return FD_EINVAL;
    if (!a.dict) {
        if (a.n_dict < 0) return FD_EINVAL;
        if (a.codec == FD_FSST8 && a.n_dict > 255) return FD_EINVAL;
        if (a.codec == FD_ONPAIR16 && a.n_dict > 65536) return FD_EINVAL;
        if (a.codec == FD_ONPAIR12) return FD_EINVAL;   // 12-bit codes decode with a prepared dictionary only
        if (a.n_dict > 0 && (!a.dict_lens || !a.dict_bytes)) return FD_EINVAL;
    }
    Plan pl;
    if (!plan_for(a.codec, a.n_codes, a.n_strings, a.tuning, &pl)) return FD_EINVAL;
    // a prepared dictionary needs no room for the one-shot repack
    if (a.ws_bytes < (a.dict ? pl.off_dict : pl.bytes)) return FD_EINVAL;
    if (a.sidecar_op && a.sidecar_n != pl.n_tiles + 1) return FD_EINVAL;   // another tiling's sidecar
    // without a tuning: the three phases when the column's tiles fill the
    // resident workgroups four times over (their expand pass takes tiles from
    // the split queues; measured crossover: FSST-8 between 32 and 64 MiB
    // decoded, OnPair-16 between 64 and 128 MiB), the single pass (fewer
    // launches, the codes read once) below that
    int mode = mode_sel;
    if (!a.tuning && !a.sidecar_op &&
        pl.n_tiles >= kAutoTilesPerWorkgroup * (int64_t)resident_grid((int)a.codec, a.index_bits, kModeExpand))
        mode = 1;

    uint8_t* ws = (uint8_t*)a.ws;
    DecodeParams p;
    memset(&p, 0, sizeof(p));
    p.codes = (const uint8_t*)a.codes;
    p.n_codes = a.n_codes;
    p.code_off = a.code_off;
    p.n_strings = a.n_strings;
    p.out_off = a.out_off;
    p.out = a.out;
    p.out_cap = a.out_cap;
    p.n_tiles = pl.n_tiles;
    p.tile_codes = pl.T;
    p.g_shift = pl.g_shift;
    p.off_pref = offsets_prefetch_count(a.codec, a.n_codes, a.n_strings, pl.T, pl.g_shift);
    p.coarse = (int64_t*)(ws + pl.off_coarse);
    p.err = (unsigned long long*)(ws + kOffErr);
    p.counters = (unsigned*)(ws + kOffCounters);
    p.tagg = (unsigned long long*)(ws + pl.off_tiles);
    p.bstate = (unsigned long long*)(ws + pl.off_blocks);
    p.status = a.status;
    p.status2 = (int32_t*)(ws + kOffStatus);

    hipStream_t st = a.stream;
    // tile words, block states and the coarse index are contiguous: one zeroing covers them
    const int64_t nz = (int64_t)((pl.off_scan - pl.off_tiles) / 8);
    if (timed(FD_PROF_RESET, st, [&] { return launch_reset(p.err, p.counters, (unsigned long long*)(ws + pl.off_tiles), nz, st); }) !=
        hipSuccess)
        return hip_fail();
    if (a.sidecar_op == kSidecarBuild) {
        // the totals pass writes the entries of the tiles with codes; the rest and the last start at zero
        p.tagg = (unsigned long long*)a.sidecar;
        if (timed(FD_PROF_RESET, st, [&] { return launch_reset(p.err, p.counters, p.tagg, pl.n_tiles + 1, st); }) !=
            hipSuccess)
            return hip_fail();
    } else if (a.sidecar_op == kSidecarDecode) {
        p.tagg = (unsigned long long*)a.sidecar;     // read only (entries t and t + 1 per tile)
    }

    if (a.codec == FD_FSST8) {
        if (a.dict) {
            p.dict_bytes = a.dict->bytes;
            p.dict_lens = a.dict->lens;
            p.n_sym = a.dict->n;
            p.fsst_tab = a.dict->fsst_tab;
            p.fsst_len = a.dict->fsst_len;
        } else {
            p.dict_bytes = a.dict_bytes;
            p.dict_lens = a.dict_lens;
            p.n_sym = a.n_dict;
        }
    } else {
        p.n_sym = a.dict ? a.dict->n : a.n_dict;    // codes at or past it are not tokens
        if (a.dict) {
            p.tok16 = a.dict->tok16;
            p.tok_len = a.dict->tok_len;
        } else {
            uint4* t16 = (uint4*)(ws + pl.off_dict);
            uint8_t* tl = ws + pl.off_dict + kTok16Bytes;
            if (timed(FD_PROF_PREPARE, st, [&] {
                    return launch_onpair_prepare(a.dict_bytes, a.dict_lens, a.n_dict, t16, tl, p.err, nullptr, st);
                }) != hipSuccess)
                return hip_fail();
            p.tok16 = t16;
            p.tok_len = tl;
        }
    }

    const int codec = (int)a.codec;
    int grid_req = a.tuning ? a.tuning->grid : 0;
    if (timed(FD_PROF_COARSE, st, [&] { return launch_coarse_one(a.index_bits, p, st); }) != hipSuccess)
        return hip_fail();
    if (a.sidecar_op == kSidecarBuild) {
        int g1 = grid_req ? grid_req : resident_grid(codec, a.index_bits, kModeTotals);
        if ((int64_t)g1 > pl.n_tiles) g1 = (int)pl.n_tiles;
        if (timed(FD_PROF_TOTALS, st, [&] { return launch_decode(codec, a.index_bits, kModeTotals, p, g1, st); }) !=
            hipSuccess)
            return hip_fail();
        if (timed(FD_PROF_SCAN, st,
                  [&] { return launch_scan_totals(p.tagg, pl.n_tiles + 1, p.err, a.status, p.status2, st); }) !=
            hipSuccess)
            return hip_fail();
    } else if (a.sidecar_op == kSidecarDecode) {
        int g2 = grid_req ? grid_req : resident_grid(codec, a.index_bits, kModeExpand);
        if ((int64_t)g2 > pl.n_tiles) g2 = (int)pl.n_tiles;
        if (timed(FD_PROF_DECODE, st, [&] { return launch_decode(codec, a.index_bits, kModeExpand, p, g2, st); }) !=
            hipSuccess)
            return hip_fail();
    } else if (mode == 0) {
        int grid = grid_req ? grid_req : resident_grid(codec, a.index_bits, kModeLookback);
        if ((int64_t)grid > pl.n_tiles) grid = (int)pl.n_tiles;
        if (timed(FD_PROF_DECODE, st,
                  [&] { return launch_decode(codec, a.index_bits, kModeLookback, p, grid, st); }) != hipSuccess)
            return hip_fail();
    } else {
        // tile totals streamed, scanned into cursors, then the expand phase
        // (which validates and checks every tile's total against its cursors)
        if (timed(FD_PROF_TOTALS, st, [&] { return launch_tile_totals(codec, a.index_bits, p, dev_cus(), st); }) !=
            hipSuccess)
            return hip_fail();
        if (timed(FD_PROF_SCAN, st, [&] {
                return launch_scan_multi(p.tagg, pl.n_tiles + 1, (unsigned long long*)(ws + pl.off_scan), st);
            }) != hipSuccess)
            return hip_fail();
        // 12-bit codes whose output capacity allows at most 3.5 bytes per code
        // of the tiles (FSST-12's short tokens): the 16 KiB staging window holds
        // a tile's output, and four workgroups fit a CU instead of three
        const int ce = (codec == kOnpair12 && (double)a.out_cap <= 3.5 * (double)pl.n_tiles * (double)p.tile_codes)
                           ? kOnpair12s
                           : codec;
        int g2 = grid_req ? grid_req : resident_grid(ce, a.index_bits, kModeExpand);
        if ((int64_t)g2 > pl.n_tiles) g2 = (int)pl.n_tiles;
        if (timed(FD_PROF_DECODE, st, [&] { return launch_decode(ce, a.index_bits, kModeExpand, p, g2, st); }) !=
            hipSuccess)
            return hip_fail();
    }

    if (a.flags & FD_ASYNC) return FD_OK;
    if (hipStreamSynchronize(st) != hipSuccess) return hip_fail();
    int32_t hs = 0;
    if (hipMemcpy(&hs, p.status2, sizeof(hs), hipMemcpyDeviceToHost) != hipSuccess) return hip_fail();
    return (fd_status)hs;
}

std::atomic<uint64_t> g_dict_ids{0};     // dictionary handle ids

// ---- the no-allocation entry point: its scratch is a file-scope device
// array (each GPU the library runs on holds its own copy until the process
// ends), found once per device by hipGetSymbolAddress ----
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64];

// The device address of this device's scratch array (nullptr on failure).
void* static_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char* fd_status_str(int status) {
    switch (status) {
        case FD_OK: return "FD_OK";
        case FD_EINVAL: return "FD_EINVAL";
        case FD_EBADCODE: return "FD_EBADCODE";
        case FD_EESCAPE: return "FD_EESCAPE";
        case FD_ECAPACITY: return "FD_ECAPACITY";
        case FD_EOVERFLOW: return "FD_EOVERFLOW";
        case FD_EBADDICT: return "FD_EBADDICT";
        case FD_EOFFSETS: return "FD_EOFFSETS";
        case FD_EHIP: return "FD_EHIP";
        case FD_ENOMEM: return "FD_ENOMEM";
        case FD_ESIDECAR: return "FD_ESIDECAR";
        case FD_ETIMEOUT: return "FD_ETIMEOUT";
        case FD_ECANCELED: return "FD_ECANCELED";
        case FD_EBUSY: return "FD_EBUSY";
        default: return "FD_UNKNOWN";
    }
}

const char* fd_version(void) { return "fastdecode 0.1 gfx950"; }

fd_status fd_workspace_size_ex(fd_codec codec, int64_t n_codes, int64_t n_strings, const fd_tuning* tuning,
                               size_t* bytes) {
    if (!bytes) return FD_EINVAL;
    // a margin of 4 standard deviations gives the most tiles: enough for every path
    Plan pl;
    if (!plan_for(codec, n_codes, n_strings, tuning, &pl)) return FD_EINVAL;
    *bytes = pl.bytes;
    return FD_OK;
}

fd_status fd_workspace_size(fd_codec codec, int64_t n_codes, int64_t n_strings, size_t* bytes) {
    return fd_workspace_size_ex(codec, n_codes, n_strings, nullptr, bytes);
}

fd_status fd_decoded_bound(fd_codec codec, int64_t n_codes, int64_t* bytes) {
    if (!bytes || n_codes < 0) return FD_EINVAL;
    if (codec == FD_FSST8) *bytes = n_codes * 8;
    else if (codec == FD_ONPAIR16 || codec == FD_ONPAIR12) *bytes = n_codes * 16;
    else return FD_EINVAL;
    return FD_OK;
}

fd_status fsst_decode(const uint8_t* codes, int64_t n_codes, const void* code_offsets, int index_bits,
                      int64_t n_strings, const uint8_t* dict_bytes, const uint8_t* dict_lens, int32_t n_symbols,
                      void* out_offsets, uint8_t* out_bytes, int64_t out_capacity, void* workspace,
                      size_t workspace_bytes, int32_t* status, unsigned flags, void* hip_stream) {
    Args a;
    memset(&a, 0, sizeof(a));
    a.codec = FD_FSST8;
    a.codes = codes; a.n_codes = n_codes; a.code_off = code_offsets; a.index_bits = index_bits;
    a.n_strings = n_strings; a.dict_bytes = dict_bytes; a.dict_lens = dict_lens; a.n_dict = n_symbols;
    a.out_off = out_offsets; a.out = out_bytes; a.out_cap = out_capacity; a.ws = workspace;
    a.ws_bytes = workspace_bytes; a.status = status; a.flags = flags; a.stream = (hipStream_t)hip_stream;
    return run_decode(a);
}

fd_status onpair_decode(const uint16_t* codes, int64_t n_codes, const void* code_offsets, int index_bits,
                        int64_t n_strings, const uint8_t* dict_bytes, const uint8_t* dict_lens, int32_t n_tokens,
                        void* out_offsets, uint8_t* out_bytes, int64_t out_capacity, void* workspace,
                        size_t workspace_bytes, int32_t* status, unsigned flags, void* hip_stream) {
    Args a;
    memset(&a, 0, sizeof(a));
    a.codec = FD_ONPAIR16;
    a.codes = codes; a.n_codes = n_codes; a.code_off = code_offsets; a.index_bits = index_bits;
    a.n_strings = n_strings; a.dict_bytes = dict_bytes; a.dict_lens = dict_lens; a.n_dict = n_tokens;
    a.out_off = out_offsets; a.out = out_bytes; a.out_cap = out_capacity; a.ws = workspace;
    a.ws_bytes = workspace_bytes; a.status = status; a.flags = flags; a.stream = (hipStream_t)hip_stream;
    return run_decode(a);
}

fd_status fd_decode_ex(const fd_dict* dict, const void* codes, int64_t n_codes, const void* code_offsets,
                       int index_bits, int64_t n_strings, void* out_offsets, uint8_t* out_bytes, int64_t out_capacity,
                       void* workspace, size_t workspace_bytes, int32_t* status, unsigned flags,
                       const fd_tuning* tuning, void* hip_stream) {
    if (!dict) return FD_EINVAL;
    Args a;
    memset(&a, 0, sizeof(a));
    a.codec = dict->codec;
    a.dict = dict;
    a.codes = codes; a.n_codes = n_codes; a.code_off = code_offsets; a.index_bits = index_bits;
    a.n_strings = n_strings; a.out_off = out_offsets; a.out = out_bytes; a.out_cap = out_capacity;
    a.ws = workspace; a.ws_bytes = workspace_bytes; a.status = status; a.flags = flags; a.tuning = tuning;
    a.stream = (hipStream_t)hip_stream;
    return run_decode(a);
}

fd_status fd_sidecar_layout(fd_codec codec, int64_t n_codes, int64_t n_strings, const fd_tuning* tuning,
                            int32_t* tile_codes, int64_t* n_entries) {
    if (!tile_codes || !n_entries) return FD_EINVAL;
    if (tuning && tuning->mode != 0) return FD_EINVAL;
    Plan pl;
    if (!plan_for(codec, n_codes, n_strings, tuning, &pl)) return FD_EINVAL;
    *tile_codes = (int32_t)pl.T;
    *n_entries = pl.n_tiles + 1;
    return FD_OK;
}

fd_status fd_sidecar_build(const fd_dict* dict, const void* codes, int64_t n_codes, const void* code_offsets,
                           int index_bits, int64_t n_strings, int64_t* sidecar, int64_t n_entries, void* workspace,
                           size_t workspace_bytes, int32_t* status, unsigned flags, const fd_tuning* tuning,
                           void* hip_stream) {
    if (!dict) return FD_EINVAL;
    Args a;
    memset(&a, 0, sizeof(a));
    a.codec = dict->codec;
    a.dict = dict;
    a.codes = codes; a.n_codes = n_codes; a.code_off = code_offsets; a.index_bits = index_bits;
    a.n_strings = n_strings; a.ws = workspace; a.ws_bytes = workspace_bytes; a.status = status; a.flags = flags;
    a.tuning = tuning; a.stream = (hipStream_t)hip_stream;
    a.sidecar_op = kSidecarBuild; a.sidecar = sidecar; a.sidecar_n = n_entries;
    return run_decode(a);
}

fd_status fd_decode_sidecar(const fd_dict* dict, const void* codes, int64_t n_codes, const void* code_offsets,
                            int index_bits, int64_t n_strings, const int64_t* sidecar, int64_t n_entries,
                            void* out_offsets, uint8_t* out_bytes, int64_t out_capacity, void* workspace,
                            size_t workspace_bytes, int32_t* status, unsigned flags, const fd_tuning* tuning,
                            void* hip_stream) {
    if (!dict) return FD_EINVAL;
    Args a;
    memset(&a, 0, sizeof(a));
    a.codec = dict->codec;
    a.dict = dict;
    a.codes = codes; a.n_codes = n_codes; a.code_off = code_offsets; a.index_bits = index_bits;
    a.n_strings = n_strings; a.out_off = out_offsets; a.out = out_bytes; a.out_cap = out_capacity;
    a.ws = workspace; a.ws_bytes = workspace_bytes; a.status = status; a.flags = flags; a.tuning = tuning;
    a.stream = (hipStream_t)hip_stream;
    a.sidecar_op = kSidecarDecode; a.sidecar = (int64_t*)sidecar; a.sidecar_n = n_entries;
    return run_decode(a);
}

fd_status fd_take_workspace_size(fd_codec codec, int64_t n_codes, int64_t n_strings, int64_t n_rows, int64_t max_codes,
                                 const fd_tuning* tuning, size_t* bytes) {
    if (!bytes) return FD_EINVAL;
    TakePlan tp;
    if (!take_plan_for(codec, n_codes, n_strings, n_rows, max_codes, tuning, &tp)) return FD_EINVAL;
    *bytes = tp.bytes;
    return FD_OK;
}

fd_status fd_decode_take(const fd_dict* dict, const void* codes, int64_t n_codes, const void* code_offsets,
                         int index_bits, int64_t n_strings, const int64_t* rows, int64_t n_rows, int64_t max_codes,
                         void* out_offsets, uint8_t* out_bytes, int64_t out_capacity, void* workspace,
                         size_t workspace_bytes, int32_t* status, unsigned flags, const fd_tuning* tuning,
                         void* hip_stream) {
    // ---------------- host-side validation ----------------
    if (!dict || !code_offsets || !out_offsets || !workspace) return FD_EINVAL;
    if (index_bits != 32 && index_bits != 64) return FD_EINVAL;
    if (n_strings < 0 || n_codes < 0 || out_capacity < 0 || n_rows < 0 || max_codes < 0) return FD_EINVAL;
    if (n_strings > (int64_t)1 << 40 || n_codes > (int64_t)1 << 40) return FD_EINVAL;
    if (n_codes > 0 && !codes) return FD_EINVAL;
    if (n_rows > 0 && (!rows || ((uintptr_t)rows & 7))) return FD_EINVAL;
    if (out_capacity > 0 && !out_bytes) return FD_EINVAL;
    if ((flags & FD_ASYNC) && !status) return FD_EINVAL;
    if (flags & ~(unsigned)FD_ASYNC) return FD_EINVAL;
    if (dict->codec == FD_ONPAIR16 && codes && ((uintptr_t)codes & 1)) return FD_EINVAL;
    const size_t ia = index_bits / 8;
    if (((uintptr_t)code_offsets & (ia - 1)) || ((uintptr_t)out_offsets & (ia - 1))) return FD_EINVAL;
    if (index_bits == 32 && (n_codes > INT32_MAX || max_codes > INT32_MAX)) return FD_EINVAL;
    if ((uintptr_t)workspace & 255) return FD_EINVAL;
    if (tuning && tuning->grid < 0) return FD_EINVAL;
    TakePlan tp;
    if (!take_plan_for(dict->codec, n_codes, n_strings, n_rows, max_codes, tuning, &tp)) return FD_EINVAL;
    if (workspace_bytes < tp.bytes) return FD_EINVAL;

    uint8_t* ws = (uint8_t*)workspace;
    hipStream_t st = (hipStream_t)hip_stream;
    unsigned long long* err = (unsigned long long*)(ws + kOffErr);
    unsigned* counters = (unsigned*)(ws + kOffCounters);
    unsigned long long* tagg = (unsigned long long*)(ws + tp.dec.off_tiles);
    // tile words, block states and the coarse index of the compacted column
    if (timed(FD_PROF_RESET, st, [&] {
            return launch_reset(err, counters, tagg, (int64_t)((tp.dec.off_scan - tp.dec.off_tiles) / 8), st);
        }) != hipSuccess)
        return hip_fail();
    // compaction: the selected strings' codes, whole, one after another
    uint8_t* ccodes = ws + tp.off_codes;
    void* coff = ws + tp.off_noff;
    // copy workgroups of about 16,384 FSST-8 codes or 4,096 OnPair codes at the
    // column's mean codes per string (measured: fewer, larger workgroups pay
    // on the long FSST-8 strings and cost on the short OnPair ones)
    const double mean = n_strings ? (double)n_codes / (double)n_strings : 1.0;
    const double per_wg = dict->codec == FD_FSST8 ? 16384.0 : 4096.0;
    int rows_per_wg = 16;
    while (rows_per_wg < 1024 && (double)(2 * rows_per_wg) * mean <= per_wg) rows_per_wg *= 2;
    if (timed(FD_PROF_PREPARE, st, [&] {
            return launch_take_compact((int)dict->codec, index_bits, rows, n_rows, code_offsets, n_strings, n_codes,
                                       (const uint8_t*)codes, (unsigned long long*)(ws + tp.off_bsum), max_codes,
                                       coff, (int64_t*)(ws + tp.off_src), ccodes, rows_per_wg, err, st);
        }) != hipSuccess)
        return hip_fail();
    // the compacted column through the decode kernels
    DecodeParams p;
    memset(&p, 0, sizeof(p));
    p.codes = ccodes;
    p.n_codes = max_codes;
    p.code_off = coff;
    p.n_strings = n_rows;
    p.out_off = out_offsets;
    p.out = out_bytes;
    p.out_cap = out_capacity;
    p.n_tiles = tp.dec.n_tiles;
    p.tile_codes = tp.dec.T;
    p.g_shift = tp.dec.g_shift;
    {
        const double mean = n_strings ? (double)n_codes / (double)n_strings : 1.0;
        p.off_pref = offsets_prefetch_count(tp.codec2, (int64_t)(mean * (double)n_rows) + 1, n_rows, tp.dec.T,
                                            tp.dec.g_shift);
    }
    p.coarse = (int64_t*)(ws + tp.dec.off_coarse);
    p.err = err;
    p.counters = counters;
    p.tagg = tagg;
    p.bstate = (unsigned long long*)(ws + tp.dec.off_blocks);
    p.status = status;
    p.status2 = (int32_t*)(ws + kOffStatus);
    if (dict->codec == FD_FSST8) {
        p.dict_bytes = dict->bytes;
        p.dict_lens = dict->lens;
        p.n_sym = dict->n;
        p.fsst_tab = dict->fsst_tab;
        p.fsst_len = dict->fsst_len;
    } else {
        p.n_sym = dict->n;                 // codes at or past it are not tokens
        p.tok16 = dict->tok16;
        p.tok_len = dict->tok_len;
    }
    const int codec2 = (int)tp.codec2;
    if (timed(FD_PROF_COARSE, st, [&] { return launch_coarse_one(index_bits, p, st); }) != hipSuccess) return hip_fail();
    // the mode: as asked, else the three phases when the selection is expected
    // (at the column's mean codes per string) to fill the resident workgroups
    // four times over with tiles, the single pass (fewer launches) below that
    int mode = tuning ? tuning->mode : -1;
    if (mode < 0) {
        const double mean = n_strings ? (double)n_codes / (double)n_strings : 1.0;
        const double tiles = mean * (double)n_rows / (double)tp.dec.T;
        mode = tiles >= (double)kAutoTilesPerWorkgroup * (double)resident_grid(codec2, index_bits, kModeExpand) ? 1
                                                                                                            : 0;
    }
    if (mode == 1) {
        if (timed(FD_PROF_TOTALS, st, [&] { return launch_tile_totals(codec2, index_bits, p, dev_cus(), st); }) !=
            hipSuccess)
            return hip_fail();
        if (timed(FD_PROF_SCAN, st, [&] {
                return launch_scan_multi(p.tagg, tp.dec.n_tiles + 1, (unsigned long long*)(ws + tp.dec.off_scan), st);
            }) != hipSuccess)
            return hip_fail();
    }
    const int kmode = mode == 1 ? kModeExpand : kModeLookback;
    int grid = (tuning && tuning->grid) ? tuning->grid : resident_grid(codec2, index_bits, kmode);
    if ((int64_t)grid > tp.dec.n_tiles) grid = (int)tp.dec.n_tiles;
    if (timed(FD_PROF_DECODE, st, [&] { return launch_decode(codec2, index_bits, kmode, p, grid, st); }) != hipSuccess)
        return hip_fail();
    if (flags & FD_ASYNC) return FD_OK;
    if (hipStreamSynchronize(st) != hipSuccess) return hip_fail();
    int32_t hs = 0;
    if (hipMemcpy(&hs, p.status2, sizeof(hs), hipMemcpyDeviceToHost) != hipSuccess) return hip_fail();
    return (fd_status)hs;
}

fd_status fd_decode_noalloc(const fd_dict* dict, const void* codes, int64_t n_codes, const void* code_offsets,
                            int index_bits, int64_t n_strings, void* out_offsets, uint8_t* out_bytes,
                            int64_t out_capacity, int32_t* status, unsigned flags, const fd_tuning* tuning,
                            void* hip_stream) {
    if (!dict) return FD_EINVAL;
    // the size check comes first: a column whose tiles do not fit the static
    // scratch is rejected before the device is touched
    Plan pl;
    if (!plan_for(dict->codec, n_codes, n_strings, tuning, &pl)) return FD_EINVAL;
    if (pl.off_dict > kStaticScratchBytes) return FD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FD_EHIP;
    void* ws = static_scratch(dev);
    if (!ws) return FD_EHIP;
    Args a;
    memset(&a, 0, sizeof(a));
    a.codec = dict->codec;
    a.dict = dict;
    a.codes = codes; a.n_codes = n_codes; a.code_off = code_offsets; a.index_bits = index_bits;
    a.n_strings = n_strings; a.out_off = out_offsets; a.out = out_bytes; a.out_cap = out_capacity;
    a.ws = ws; a.ws_bytes = kStaticScratchBytes; a.status = status; a.flags = flags; a.tuning = tuning;
    a.stream = (hipStream_t)hip_stream;
    return run_decode(a);
}

fd_status fd_decode(const fd_dict* dict, const void* codes, int64_t n_codes, const void* code_offsets, int index_bits,
                    int64_t n_strings, void* out_offsets, uint8_t* out_bytes, int64_t out_capacity, void* workspace,
                    size_t workspace_bytes, int32_t* status, unsigned flags, void* hip_stream) {
    return fd_decode_ex(dict, codes, n_codes, code_offsets, index_bits, n_strings, out_offsets, out_bytes,
                        out_capacity, workspace, workspace_bytes, status, flags, nullptr, hip_stream);
}

fd_status fd_dict_create(fd_codec codec, const uint8_t* dict_bytes, const uint8_t* dict_lens, int32_t n_tokens,
                         void* hip_stream, fd_dict** out) {
    if (!out) return FD_EINVAL;
    *out = nullptr;
    if (codec != FD_FSST8 && codec != FD_ONPAIR16 && codec != FD_ONPAIR12) return FD_EINVAL;
    if (n_tokens < 0 || (codec == FD_FSST8 && n_tokens > 255) || (codec == FD_ONPAIR16 && n_tokens > 65536) ||
        (codec == FD_ONPAIR12 && n_tokens > 4096))
        return FD_EINVAL;
    if (n_tokens > 0 && (!dict_bytes || !dict_lens)) return FD_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    fd_dict* d = new (std::nothrow) fd_dict;
    if (!d) return FD_ENOMEM;
    memset(d, 0, sizeof(*d));
    d->codec = codec;
    d->n = n_tokens;
    d->id = g_dict_ids.fetch_add(1) + 1;
    if (hipGetDevice(&d->device) != hipSuccess) { delete d; return FD_EHIP; }
    // scratch: err word + bad flag
    const size_t hdr = 256;
    size_t bytes;
    if (codec == FD_FSST8) bytes = hdr + 256 + 255 * 8 + 8 + 256 * 8 + 256;
    else bytes = hdr + kTok16Bytes + kTokLenBytes;
    if (hipMalloc(&d->mem, bytes) != hipSuccess) { delete d; return FD_ENOMEM; }
    uint8_t* m = (uint8_t*)d->mem;
    unsigned long long* err = (unsigned long long*)m;
    int* bad = (int*)(m + 8);
    if (hipMemsetAsync(m, 0, hdr, st) != hipSuccess) goto fail;
    if (codec == FD_FSST8) {
        uint8_t* lens = m + hdr;
        uint8_t* syms = m + hdr + 256;
        if (hipMemsetAsync(lens, 0, 256 + 255 * 8, st) != hipSuccess) goto fail;
        if (n_tokens > 0) {
            // the packed size is only known on the device: copy lengths first
            uint8_t hl[256];
            if (hipMemcpyAsync(hl, dict_lens, (size_t)n_tokens, hipMemcpyDeviceToHost, st) != hipSuccess) goto fail;
            if (hipStreamSynchronize(st) != hipSuccess) goto fail;
            size_t sum = 0;
            for (int i = 0; i < n_tokens; i++) {
                if (hl[i] == 0 || hl[i] > 8) { (void)hipFree(d->mem); delete d; return FD_EBADDICT; }
                sum += hl[i];
            }
            if (hipMemcpyAsync(lens, dict_lens, (size_t)n_tokens, hipMemcpyDeviceToDevice, st) != hipSuccess) goto fail;
            if (sum && hipMemcpyAsync(syms, dict_bytes, sum, hipMemcpyDeviceToDevice, st) != hipSuccess) goto fail;
        }
        // the decode table in the layout the kernels keep in LDS, built once here
        {
            uint8_t hl[256] = {0}, hs[256 * 8] = {0};
            if (n_tokens > 0) {
                if (hipMemcpyAsync(hl, dict_lens, (size_t)n_tokens, hipMemcpyDeviceToHost, st) != hipSuccess) goto fail;
                if (hipStreamSynchronize(st) != hipSuccess) goto fail;
                size_t sum = 0;
                for (int i = 0; i < n_tokens; i++) sum += hl[i];
                if (sum && hipMemcpyAsync(hs, dict_bytes, sum, hipMemcpyDeviceToHost, st) != hipSuccess) goto fail;
                if (hipStreamSynchronize(st) != hipSuccess) goto fail;
            }
            unsigned long long* tab = (unsigned long long*)(m + hdr + 256 + 255 * 8 + 8);
            uint8_t* tl = (uint8_t*)(tab + 256);
            // host images, uploaded before this function returns (it synchronizes below)
            unsigned long long htab[256] = {0};
            uint8_t htl[256];
            size_t at = 0;
            for (int c = 0; c < 256; c++) {
                if (c < n_tokens) {
                    for (int j = 0; j < hl[c]; j++) htab[c] |= (unsigned long long)hs[at + j] << (8 * j);
                    at += hl[c];
                    htl[c] = hl[c];
                } else {
                    htl[c] = 0x80;
                }
                if (c == 255) htl[c] = 0;
            }
            if (hipMemcpyAsync(tab, htab, sizeof(htab), hipMemcpyHostToDevice, st) != hipSuccess) goto fail;
            if (hipMemcpyAsync(tl, htl, sizeof(htl), hipMemcpyHostToDevice, st) != hipSuccess) goto fail;
            if (hipStreamSynchronize(st) != hipSuccess) goto fail;
            d->fsst_tab = tab;
            d->fsst_len = tl;
        }
        d->lens = lens;
        d->bytes = syms;
        if (hipStreamSynchronize(st) != hipSuccess) goto fail;
    } else {
        uint4* t16 = (uint4*)(m + hdr);
        uint8_t* tl = m + hdr + kTok16Bytes;
        if (launch_onpair_prepare(dict_bytes, dict_lens, n_tokens, t16, tl, err, bad, st) != hipSuccess) goto fail;
        int hbad = 0;
        if (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) goto fail;
        if (hipStreamSynchronize(st) != hipSuccess) goto fail;
        if (hbad) { (void)hipFree(d->mem); delete d; return FD_EBADDICT; }
        d->tok16 = t16;
        d->tok_len = tl;
    }
    *out = d;
    return FD_OK;
fail:
    (void)hipFree(d->mem);
    delete d;
    return FD_EHIP;
}

fd_status fd_dict_destroy(fd_dict* dict) {
    if (!dict) return FD_EINVAL;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != dict->device) (void)hipSetDevice(dict->device);
    // cached batch graphs that read this dictionary go first: a handle created
    // later at the same address must never replay them
    batch_forget_dict(dict->id, dict->device);
    hipError_t e = hipFree(dict->mem);
    if (cur != dict->device) (void)hipSetDevice(cur);
    delete dict;
    return e == hipSuccess ? FD_OK : FD_EHIP;
}

fd_codec fd_dict_codec(const fd_dict* dict) { return dict ? dict->codec : (fd_codec)0; }
int32_t fd_dict_size(const fd_dict* dict) { return dict ? dict->n : -1; }

}  // extern "C"
