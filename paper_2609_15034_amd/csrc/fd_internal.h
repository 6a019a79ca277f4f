// Internal declarations shared by the decode kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastdecode.h"

namespace fd {

constexpr int kFsst8 = FD_FSST8;
constexpr int kOnpair16 = FD_ONPAIR16;
constexpr int kOnpair12 = FD_ONPAIR12;
// (internal) the 12-bit expand pass with a 16 KiB staging window: for columns
// whose tiles decode to at most about one such window (short tokens, as
// FSST-12's), where the smaller window lets four workgroups share a CU
constexpr int kOnpair12s = 4;

constexpr int kWG = 256;            // threads per workgroup
constexpr int kNWave = kWG / 64;    // waves per workgroup
constexpr int kWinFsst = 16384;     // LDS staging window (bytes), FSST-8
constexpr int kWinOnpair = 32768;   // LDS staging window (bytes), OnPair-16 (3 workgroups per CU by VGPRs: room for a pass)
// A tile is a fixed range of code positions: tile t of a column holds the
// codes at positions [t T, (t + 1) T) of its code buffer that lie inside the
// decode range [code_offsets[0], code_offsets[n]).  T is a multiple of the
// codes in a 16-byte chunk (16 FSST-8, 8 OnPair) and at most one pass of a
// workgroup less one chunk (a tile whose buffer is not 16-byte aligned then
// still fits one pass).
constexpr int kTileMaxFsst = 8192 - 16;
constexpr int kTileMaxOnpair = 4096 - 8;
// Each tile finds its strings from a coarse index: sample j is code offset
// j G, and coarse[t] is the last sample below the tile's first position.
constexpr int kCoarseShiftMin = 6;     // G >= 64
constexpr int kCoarseShiftMax = 10;    // G <= 1024
constexpr int kBlkShift = 6;        // tiles per look-back block: 64
constexpr int kBlk = 1 << kBlkShift;

// decode modes
constexpr int kModeLookback = 0;    // single pass, decoupled look-back for tile cursors
constexpr int kModeTotals = 1;      // three-phase: tile totals only
// without a tuning, the three phases from this many tiles per resident
// expand-pass workgroup on (the single pass below)
constexpr int kAutoTilesPerWorkgroup = 4;
constexpr int kModeExpand = 2;      // three-phase / sidecar: expand with stored tile cursors (checked)
// Tile queues.  Workgroups take tiles from counters in device memory.  One
// counter takes about 12 ns per device-scope atomic on the same address, a
// limit the decode of a 1 GiB column (about 10^5 tiles) reaches, so a decode
// that needs no order splits its tiles into kQueues contiguous ranges, each
// with its own counter in its own 256-byte line; workgroup b starts on range
// b % kQueues (the workgroups of one XCD, as the dispatcher deals them out)
// and moves on to the next ranges when its own runs out.  The single pass
// keeps one queue: its look-back needs the tiles taken in order.
// A counter block: word 0 counts finished workgroups, queue q's counter is
// word kQueueStride * (q + 1).
constexpr int kQueues = 8;
constexpr int kQueueStride = 64;
constexpr size_t kCounterBlockBytes = 4 * (size_t)kQueueStride * (kQueues + 1);

// tile state words (look-back): 2 flag bits + 62 value bits
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint64_t kFlagMask = 3ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;          // look-back sleeps before giving up

// error keys: (rank << 4) | status; the smallest key wins
constexpr uint64_t kRankInternal = 0;             // look-back wait limit exceeded
constexpr uint64_t kRankDict = 0;
constexpr uint64_t kRankOffsets = 1;
constexpr uint64_t kRankData = 2;                 // + code position
constexpr uint64_t kRankSidecar = (1ull << 58) - 1;   // stored cursors that do not match the codes
constexpr uint64_t kRankOverflow = 1ull << 58;
constexpr uint64_t kRankCapacity = (1ull << 58) + 1;

struct DecodeParams {
    const uint8_t* codes;          // code stream (uint8 or uint16 codes)
    int64_t n_codes;
    const void* code_off;          // int32 / int64, n_strings + 1
    int64_t n_strings;
    // FSST-8: packed symbols
    const uint8_t* dict_bytes;
    const uint8_t* dict_lens;
    int32_t n_sym;
    const unsigned long long* fsst_tab;   // prepared table (256 zero-padded symbols), or null
    const uint8_t* fsst_len;       // prepared lengths (0x80: not a symbol, 0: escape), or null
    // OnPair-16: prepared fixed-stride dictionary
    const uint4* tok16;
    const uint8_t* tok_len;
    // outputs
    void* out_off;
    uint8_t* out;
    int64_t out_cap;
    // tiling
    int64_t n_tiles;               // ceil(n_codes / tile_codes), at least 1
    int64_t tile_codes;            // T
    int64_t* coarse;               // per tile: the coarse sample group its strings start in
    int32_t g_shift;               // log2 of the coarse sample stride G
    int32_t off_pref;              // code offsets a tile prefetches from its coarse sample on
    // workspace
    unsigned long long* err;
    unsigned* counters;            // a counter block (kCounterBlockBytes): tile queues, finished workgroups
    unsigned long long* tagg;      // per tile: aggregate (look-back) / total / cursor (three phases, sidecar:
                                   // n_tiles + 1 int64 entries, the last the decoded total)
    unsigned long long* bstate;    // per block of kBlk tiles: look-back state
    int32_t* status;               // caller's device status (may be null)
    int32_t* status2;              // workspace status slot
};

int decode_occupancy(int codec, int index_bits, int mode);
hipError_t launch_decode(int codec, int index_bits, int mode, const DecodeParams& p, int grid, hipStream_t st);
hipError_t launch_reset(unsigned long long* err, unsigned* counters, unsigned long long* z, int64_t n,
                        hipStream_t st);
// Exclusive scan of v[0, n) in place; with err non-null it then publishes the
// status of the errors recorded so far to *status / *status2.
hipError_t launch_scan_totals(unsigned long long* v, int64_t n, const unsigned long long* err, int32_t* status,
                              int32_t* status2, hipStream_t st);
// Selective decode: compact the codes of the rows rows[0, n_rows) of a column
// into dst (uint8 for FSST-8, uint16 for OnPair-16 and widened OnPair-12) with
// their offsets new_off[0, n_rows] (index_bits wide), using bsum (one word
// per 1,024 rows, plus one) and src (n_rows words) as scratch; a copy
// workgroup handles rows_per_wg (1..1,024) rows.  Bad rows or offsets record EOFFSETS; more than max_codes
// codes record ENOMEM (the stream is then cut there).
hipError_t launch_take_compact(int codec, int index_bits, const int64_t* rows, int64_t n_rows,
                               const void* code_off, int64_t n_strings, int64_t n_codes, const uint8_t* codes,
                               unsigned long long* bsum, int64_t max_codes, void* new_off, int64_t* src, uint8_t* dst,
                               int rows_per_wg, unsigned long long* err, hipStream_t st);
// Three-phase mode: every tile's decoded total into p.tagg[0, n_tiles) (no
// validation), on a grid of resident workgroups over `cus` compute units.
hipError_t launch_tile_totals(int codec, int index_bits, const DecodeParams& p, int cus, hipStream_t st);
// Exclusive scan of v[0, n) in place; bsum: ceil(n / 1024) + 1 words of scratch.
hipError_t launch_scan_multi(unsigned long long* v, int64_t n, unsigned long long* bsum, hipStream_t st);
int batch_occupancy(int codec, int index_bits, int mode);
// mode: kModeLookback, or kModeExpand with each column's p.tagg pointing at the
// group's scanned totals at the column's first tile
hipError_t launch_decode_batch(int codec, int index_bits, int mode, const DecodeParams* cols, const int64_t* first_tile,
                               int32_t n_cols, int64_t total, unsigned* ctr, int grid, hipStream_t st);
// A batch group's tile totals in global tile order into out[0, total).
hipError_t launch_tile_totals_batch(int codec, int index_bits, const DecodeParams* cols, const int64_t* first_tile,
                                    int32_t n_cols, int64_t total, unsigned long long* out, int cus, hipStream_t st);
hipError_t launch_batch_reset(unsigned long long* z, int64_t n, unsigned long long* errs, int32_t n_cols,
                              hipStream_t st);
hipError_t launch_batch_status(const unsigned long long* errs, int32_t n_cols, int32_t* status, int32_t* status2,
                               hipStream_t st);
int chunks_per_lane(int codec);   // 16-byte code chunks each lane holds per super-pass
int codes_per_chunk(int codec);
hipError_t launch_onpair_prepare(const uint8_t* bytes, const uint8_t* lens, int32_t n_tok, uint4* tok16,
                                 uint8_t* tok_len, unsigned long long* err, int* bad_flag, hipStream_t st);

// host runtime helpers shared by the single-column and batch entry points
int64_t codes_per_pass(fd_codec c);
int64_t tile_codes_max(fd_codec c);
// Tile size of a decode: 0 = the largest; else a multiple of the codes per
// chunk in [that, the largest]; -1 when invalid.
int64_t tile_codes_for(fd_codec c, int64_t requested);
int64_t tiles_of(int64_t n_codes, int64_t tile_codes);
// The coarse index stride of a column (log2): about half the strings of a
// tile at the column's mean codes per string, within [2^6, 2^10].
int coarse_shift(int64_t n_codes, int64_t n_strings, int64_t tile_codes);
// How many code offsets a tile prefetches from its coarse sample on: its
// expected strings with a margin plus one stride of the index, at most what
// the kernel holds (256 FSST-8, 1,024 OnPair).
int offsets_prefetch_count(fd_codec c, int64_t n_codes, int64_t n_strings, int64_t tile_codes, int g_shift);
// The coarse index of a column into p.coarse (n_tiles words, zeroed before),
// or of every column of a batch group (cols: the device table; max_samples:
// the largest ceil(n_strings / G) of its columns).
hipError_t launch_coarse_one(int index_bits, const DecodeParams& p, hipStream_t st);
hipError_t launch_coarse_batch(int index_bits, const DecodeParams* cols, int32_t n_cols, int64_t max_samples,
                               hipStream_t st);
int dev_cus();   // compute units of the current device
// Batch graph cache: drop (after synchronizing the device) every cached graph
// whose columns use the dictionary with this id; called by fd_dict_destroy.
void batch_forget_dict(uint64_t dict_id, int device);
int resident_grid(int codec, int index_bits, int mode);
int resident_grid_batch(int codec, int index_bits, int mode);

// Kernel timing while a profile is open (fd_profile_begin): prof_begin records
// a start event on `st` for a launch of `kind` (an fd_prof_kind) and returns
// its slot, or -1 when the kind is not selected or no profile is open;
// prof_end records the slot's end event.
int prof_begin(int kind, hipStream_t st);
void prof_end(int slot, hipStream_t st);

// A launch bracketed by prof_begin / prof_end.
template <class F>
hipError_t timed(int kind, hipStream_t st, F&& launch) {
    const int slot = prof_begin(kind, st);
    const hipError_t e = launch();
    prof_end(slot, st);
    return e;
}

}  // namespace fd

// A prepared dictionary (device-resident, immutable after creation).
struct fd_dict {
    fd_codec codec;
    int32_t n;
    int device;
    uint64_t id;            // unique per handle over the process's life (graph cache keys)
    void* mem;              // single device allocation owned by the handle
    const uint8_t* bytes;   // FSST-8: packed symbols (copy)
    const uint8_t* lens;    // FSST-8: lengths (copy)
    const unsigned long long* fsst_tab;   // FSST-8: the decode table, 256 zero-padded 8-byte symbols
    const uint8_t* fsst_len;              // FSST-8: per code: length, 0x80 if not a symbol, 0 for 255
    const uint4* tok16;     // OnPair-16: fixed 16-byte entries, 65,536 of them
    const uint8_t* tok_len; // OnPair-16: 65,536 lengths (0 = invalid code)
};
