// Decode kernels for FSST-8 and OnPair-16 string columns on gfx950 (CDNA4).
//
// Work decomposition.  A tile is a fixed range of T code positions (the
// paper's fixed-size batches of codes, design overview): tile t holds the
// codes at positions [t T, (t + 1) T) of the buffer that lie inside the decode
// range [code_offsets[0], code_offsets[n]), so every tile but the last at each
// end is full and strings may cross tiles.  A workgroup (4 waves of 64 lanes)
// decodes one tile at a time and takes tiles from a global counter in
// increasing order.  Inside a tile the code range is cut into 16-byte-aligned
// chunks (16 FSST codes or 8 OnPair codes); lane l owns P consecutive chunks,
// so its codes are contiguous in the stream and stay in registers from the
// length scan to the emit.  T is at most one pass of the workgroup (256 lanes
// x P chunks) less one chunk, so a tile is always one pass.
//
// Steps per tile (the stages of the paper's Algorithm 1, re-cut for wave64
// and LDS):
//   load    - P 16-byte loads per lane (the input stage);
//   parity  - FSST-8: a position is a literal iff the run of 255 bytes right
//             before it has odd length; lanes classify their codes with a
//             bit-parallel carry trick, and the run parity entering a lane
//             comes from ballots over the wave and the waves of the workgroup;
//             the parity entering the tile comes from the run of 255 bytes
//             just before its first code;
//   lengths - decoded length per code (token length, 0 for an escape, 1 for a
//             literal), lane totals and per-code prefixes inside each chunk;
//   scan    - workgroup exclusive scan of lane totals (WarpPrefixSum at
//             workgroup scope);
//   cursor  - the tile's output position by a two-level decoupled look-back
//             (tiles inside a block of 64, then block totals), the on-device
//             replacement of the paper's per-batch sidecar;
//   emit    - each lane copies its tokens in order into an LDS staging window
//             placed at the destination's 16-byte alignment; it writes whole
//             8/16-byte entries and lets its own next token overwrite the
//             excess (the copy-and-advance idea of OnPair's CPU loop), and
//             writes exact lengths where the excess would leave its range;
//   drain   - aligned 16-byte nontemporal stores, byte stores only for the
//             head and tail of the range (the drain stage);
//   offsets - Arrow offsets of the strings starting in the tile, from the
//             per-code prefixes kept in LDS; the tile finds its strings from a
//             coarse index (every G-th code offset, built by k_coarse) and
//             checks every code offset it reads.
// All arithmetic is integer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fd_internal.h"

namespace fd {

// --------------------------------------------------------------------------
// device helpers
// --------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// The thread's index as an opaque value: the decode loop runs for many
// tiles, and values derived from the index would otherwise be hoisted out of
// it and kept live (spilled) across the whole loop body; recomputing them
// costs an instruction or two.
__device__ __forceinline__ unsigned ltid() {
    unsigned t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// values the workgroup shares through LDS are uniform: keep them in SGPRs
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t uniform32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const unsigned lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (unsigned)d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint64_t y = __shfl_xor(x, d, 64);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ void record_error(unsigned long long* err, uint64_t rank, int status) {
    atomicMin(err, (unsigned long long)((rank << 4) | (uint64_t)status));
}

// Expand mode: tile t's stored cursor, checked against the next tile's
// (stored cursor + the tile's decoded total = the next stored cursor, and
// tile 0 starts at 0).  A mismatch records ESIDECAR and gives -1: the tile
// then writes nothing.  A sidecar that passes every tile's check is the
// exclusive prefix of the decoded tile totals, entry for entry.  Entries are
// kept below 2^62 even when every tile's check passes on a shifted sidecar,
// so output positions derived from them cannot wrap.
__device__ __forceinline__ int64_t checked_cursor(const DecodeParams& p, int64_t t, int64_t cur, int64_t nxt,
                                                  uint64_t total) {
    const bool ok = cur >= 0 && (t != 0 || cur == 0) && nxt >= cur && nxt <= (int64_t)kValueMask &&
                    (uint64_t)(nxt - cur) == total;
    if (!ok) record_error(p.err, kRankSidecar, FD_ESIDECAR);
    return ok ? cur : -1;
}

__device__ __forceinline__ uint64_t data_error_key(int64_t pos, int status) {
    return ((uint64_t)(pos + (int64_t)kRankData) << 4) | (uint64_t)status;
}

// minimum over the wave of per-lane error keys (UINT64_MAX = none), one atomic
__device__ __forceinline__ void wave_record_error(unsigned long long* err, uint64_t key) {
    if (__ballot(key != ~0ull)) {
        const uint64_t m = wave_min_u64(key);
        if (lane_id() == 0) atomicMin(err, (unsigned long long)m);
    }
}

// Loads through global (not generic) addresses: a generic load also counts
// against the LDS wait counter, so every later wait for an LDS access would
// wait for it too.
#define FD_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ u32x4 gload16_nt(uintptr_t a) { return __builtin_nontemporal_load((const FD_GLOBAL u32x4*)a); }
__device__ __forceinline__ uint32_t gload4_nt(uintptr_t a) {
    return __builtin_nontemporal_load((const FD_GLOBAL uint32_t*)a);
}
__device__ __forceinline__ uint32_t gload1(uintptr_t a) { return *(const FD_GLOBAL uint8_t*)a; }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Escape classification of one lane's FSST-8 codes.
//   F   - bit j set when code j is 255 (and inside the tile)
//   cin - 1 when code 0 is a literal (the run of 255 before the lane is odd)
// A 255 read where a code is expected is an escape, the code after an escape
// is a literal.  Inside a run of 255 starting in the "code" state, escapes sit
// at the run's even offsets.  Runs whose start is at an even bit position are
// isolated with one addition (the carry clears exactly those runs).
__device__ __forceinline__ void classify_escapes(uint32_t F, uint32_t cin, uint32_t& esc, uint32_t& lit) {
    const uint32_t EVEN = 0x55555555u, ODD = 0xaaaaaaaau;
    const uint32_t S = F & ~(F << 1);                     // run starts
    uint32_t Se = S & EVEN;                               // runs starting at even positions
    if (cin) Se &= ~1u;                                   // a run at 0 continues an odd run
    const uint32_t Re = F & ~(F + Se);                    // bits of even-start runs
    const uint32_t Ro = F & ~Re;
    esc = (Re & EVEN) | (Ro & ODD);
    lit = (esc << 1) | cin;
}

// The escape parity entering a tile applies at its first code, bit f of the
// first lane's mask (f = the codes of the first chunk before the tile, 0..15
// when the code buffer is not 16-byte aligned).  For f > 0 it is placed as one
// escape at bit f - 1 (an out-of-tile position, whose length and output are
// masked anyway), so that the bit-parallel classification sees the run
// parity right where the tile starts; the carry into bit 0 is then 0.
__device__ __forceinline__ uint32_t tile_entry_mask(int64_t f, uint32_t cin) {
    return (f > 0 && f < 32 && cin) ? (1u << (uint32_t)(f - 1)) : 0u;
}

// 0x80 in each byte of x that is 255, 0 elsewhere
__device__ __forceinline__ uint32_t ff_bytes(uint32_t x) { return ((x & 0x7f7f7f7fu) + 0x01010101u) & x & 0x80808080u; }

// The 255 mask of 32 codes (bit 4d + b: byte b of dword d is 255) from the
// ff_bytes of its eight dwords: an 8-bit dot product with the weights
// 1, 2, 4, 8 (dword 2i) and 16 .. 128 (dword 2i + 1) gathers byte i of the
// mask, scaled by 128, in one full-rate instruction per dword.
__device__ __forceinline__ uint32_t ff_mask32(const uint32_t m[8]) {
    uint32_t d[4];
#pragma unroll
    for (int i = 0; i < 4; i++)
        d[i] = __builtin_amdgcn_udot4(m[2 * i + 1], 0x80402010u,
                                      __builtin_amdgcn_udot4(m[2 * i], 0x08040201u, 0u, false), false);
    return (d[0] >> 7) | (d[1] << 1) | (d[2] << 9) | (d[3] << 17);
}

// expand 4 bits into bit 7 of each byte of a dword
// 4 bits -> bytes 0x01 / 0x00 (a 24-bit multiply places bit k at bit 8k)
__device__ __forceinline__ uint32_t nib_to_bytes(uint32_t nib) { return ((nib & 0xfu) * 0x00204081u) & 0x01010101u; }
__device__ __forceinline__ uint32_t bits_to_byte_msb(uint32_t nib) { return nib_to_bytes(nib) << 7; }
// 4 bits -> bytes 0xFF / 0x00 with a byte permute (selector byte 12 reads as
// 0x00, 13 as 0xFF); written as (b << 8) - b the compiler folds it into a
// quarter-rate 32-bit multiply by 255
__device__ __forceinline__ uint32_t nib_to_ff(uint32_t nib) {
    return __builtin_amdgcn_perm(0u, 0u, nib_to_bytes(nib) | 0x0c0c0c0cu);
}

// --------------------------------------------------------------------------
// configuration
// --------------------------------------------------------------------------
constexpr int kMaxWin = 8;    // staging windows per super-pass, at most (64 KiB / (WIN - 256) + 1 = 5)
template <int CODEC> struct Cfg;
template <> struct Cfg<kFsst8> {
    static constexpr int CB = 1;      // bytes per code
    static constexpr int CPC = 16;    // codes per 16-byte chunk
    static constexpr int P = 2;       // chunks per lane
    static constexpr int CPL = 32;    // codes per lane
    static constexpr int W = 8;       // bytes written per token (fixed-stride entry)
    static constexpr int WIN = kWinFsst;   // LDS staging window (bytes)
};
template <> struct Cfg<kOnpair16> {
    static constexpr int CB = 2;
    static constexpr int CPC = 8;
    static constexpr int P = 2;
    static constexpr int CPL = 16;
    static constexpr int W = 16;
    static constexpr int WIN = kWinOnpair;
};
// OnPair-12 (and FSST-12: the same decode with tokens of at most 8 bytes):
// 12-bit codes packed least significant bit first, two codes in three bytes.
// A chunk is 8 codes = 12 bytes, unpacked at load into the OnPair-16 register
// layout; everything after the load is the OnPair-16 path.
template <> struct Cfg<kOnpair12> {
    static constexpr int CB = 0;      // (not whole bytes: see PACKED)
    static constexpr int CPC = 8;
    static constexpr int P = 2;
    static constexpr int CPL = 16;
    static constexpr int W = 16;
    static constexpr int WIN = kWinOnpair;
};
template <> struct Cfg<kOnpair12s> : Cfg<kOnpair12> {
    static constexpr int WIN = kWinFsst;
};
template <int CODEC> constexpr bool kPacked12 = CODEC == kOnpair12 || CODEC == kOnpair12s;
// Code offsets each thread prefetches at a tile's start (the first block of
// the tile's strings, read from the coarse index's sample on): enough for the
// usual strings per tile (about 100 FSST-8 log lines, 500-800 short OnPair
// strings) and the entries before the tile's first string.
template <int CODEC> constexpr int kOffR = CODEC == kFsst8 ? 1 : 4;
template <int CODEC> constexpr bool kIsOnpair = CODEC == kOnpair16 || kPacked12<CODEC>;

// bytes of a 12-bit packed stream of n codes
__host__ __device__ __forceinline__ int64_t packed12_bytes(int64_t n) { return (n * 12 + 7) / 8; }

template <int CODEC> struct SmemT {
    static constexpr int P = Cfg<CODEC>::P, CPC = Cfg<CODEC>::CPC;
    // staging window, zero before the assembly (+32: the last entries' ORs
    // reach up to 24 bytes past their start; the drain's 16-byte reads)
    alignas(16) uint8_t stage[Cfg<CODEC>::WIN + 32];
    uint8_t pre8[kWG * P * CPC];          // per code: prefix inside its chunk | escape bit
    uint32_t lane_pre[kWG];               // per lane: exclusive prefix inside the tile
    uint16_t cbase[kWG * P];              // per chunk: prefix inside its lane
    int64_t off[1 + kWG * kOffR<CODEC>];  // code offsets S0 - 1 .. S0 + kWG R - 1 of the tile (prefetched)
    uint64_t fsst_tab[CODEC == kFsst8 ? 256 : 1];
    uint8_t fsst_len[CODEC == kFsst8 ? 256 : 4];
    alignas(16) uint8_t len12[kPacked12<CODEC> ? 4096 : 16];   // 12-bit codes: the lengths of their 4,096 tokens
    uint32_t wsum[kNWave];
    uint32_t wlast[kNWave];               // total of each wave's last lane
    uint32_t wpar[kNWave];
    int64_t hdr[2];                       // the column's decode range [code_offsets[0], code_offsets[n])
    int64_t pfirst[2][kNWave];            // offsets: per-wave first index past the tile, double-buffered
    uint32_t vote[2][kNWave];             // offsets: per-wave "first string found" flags
    uint32_t cin;                         // FSST-8: escape parity entering the tile
    int64_t cursor;
    uint32_t wbase[kMaxWin + 1];          // staging windows: first output byte of each
    uint32_t nwin;
    int32_t next_id;
};

// Geometry of a tile: its code range, the string starts it owns and its
// 16-byte chunks.
struct Geom {
    int64_t a, b;       // the tile's codes [a, b) inside the decode range (a <= b)
    int64_t own_lo, own_hi;   // it writes the offsets of strings starting in [own_lo, own_hi)
    int64_t pos0;       // code position of byte 0 of chunk 0 (may be negative)
    int64_t nchunk;
    uintptr_t base;     // address of chunk 0
};

// Tile t of a column whose decode range is [ca, cb) (clamped to the buffer,
// so bad offsets cannot move a tile outside it; they are reported by the
// offsets step).  The last tile also owns the strings that start at the end.
template <int CODEC>
__device__ __forceinline__ Geom make_geom(const DecodeParams& p, int64_t t, int64_t ca, int64_t cb) {
    using C = Cfg<CODEC>;
    Geom g;
    const int64_t T = p.tile_codes;
    ca = min(max(ca, (int64_t)0), p.n_codes);
    cb = min(max(cb, ca), p.n_codes);
    g.own_lo = t * T;
    g.own_hi = (t + 1 >= p.n_tiles) ? INT64_MAX : (t + 1) * T;
    g.a = min(max(g.own_lo, ca), cb);
    g.b = min(max((t + 1) * T, g.a), cb);
    const uintptr_t lo = (uintptr_t)p.codes;
    if constexpr (kPacked12<CODEC>) {
        // chunks are groups of 8 codes (12 bytes) from the start of the stream
        g.pos0 = g.a & ~(int64_t)7;
        g.base = lo + (uintptr_t)(g.pos0 / 8) * 12u;
        g.nchunk = (g.b > g.a) ? (g.b - g.pos0 + 7) / 8 : 0;
    } else {
        g.base = (lo + (uintptr_t)g.a * C::CB) & ~(uintptr_t)15;
        g.nchunk = (g.b > g.a) ? (int64_t)((lo + (uintptr_t)g.b * C::CB - g.base + 15) >> 4) : 0;
        g.pos0 = ((int64_t)g.base - (int64_t)lo) / C::CB;
    }
    return g;
}

// The last tile with work: the one that holds the end of the decode range
// (it owns the strings that start there).  The tiles after it have no codes
// and no strings.
__device__ __forceinline__ int64_t last_tile(const DecodeParams& p, int64_t ca, int64_t cb) {
    ca = min(max(ca, (int64_t)0), p.n_codes);
    cb = min(max(cb, ca), p.n_codes);
    return min(cb / p.tile_codes, p.n_tiles - 1);
}

// The first tile with work: the one that holds the start of the decode range.
// The tiles before it have no codes and no strings.
__device__ __forceinline__ int64_t first_tile(const DecodeParams& p, int64_t ca, int64_t cb) {
    ca = min(max(ca, (int64_t)0), p.n_codes);
    return min(ca / p.tile_codes, last_tile(p, ca, cb));
}

// The column's decode range, read once per column (two uniform loads).
template <typename IDX>
__device__ __forceinline__ void column_range(const DecodeParams& p, int64_t& ca, int64_t& cb) {
    const IDX* co = (const IDX*)p.code_off;
    ca = (int64_t)co[0];
    cb = (int64_t)co[p.n_strings];
}

// FSST-8: the escape parity entering code position a, i.e. the parity of the
// run of 255 bytes right before a, counted back to the previous other byte or
// to the start of the decode range ca (one wave; a loop step per 64 bytes of
// run).  In valid data no string ends inside an escape, so this stream-level
// parity is the one the string's own decode has.
// The lane's byte of the first window, a - 1 - lane (0x100 before ca): loaded
// ahead, one tile early, by fsst_window_byte.
__device__ __forceinline__ uint32_t fsst_window_byte(const uint8_t* codes, int64_t ca, int64_t a) {
    const int64_t q = a - 1 - (int64_t)lane_id();
    return q >= ca ? (uint32_t)codes[q] : 0x100u;
}

__device__ __forceinline__ uint32_t fsst_carry_in_from(const uint8_t* codes, int64_t ca, int64_t a, uint32_t first) {
    const uint64_t m0 = __ballot(first != 0xFFu);
    if (m0) return (uint32_t)(((int64_t)__ffsll((unsigned long long)m0) - 1) & 1);
    const int64_t lane = (int64_t)lane_id();
    int64_t run = 64;
    for (int64_t q0 = a - 65; q0 >= ca; q0 -= 64) {
        const int64_t q = q0 - lane;
        const bool stop = q < ca || codes[q] != 0xFF;
        const uint64_t m = __ballot(stop);
        if (m) {
            run += (int64_t)__ffsll((unsigned long long)m) - 1;
            break;
        }
        run += 64;
    }
    return (uint32_t)(run & 1);
}

__device__ __forceinline__ uint32_t fsst_carry_in(const uint8_t* codes, int64_t ca, int64_t a) {
    const int64_t lane = (int64_t)lane_id();
    int64_t run = 0;
    for (int64_t q0 = a - 1; q0 >= ca; q0 -= 64) {
        const int64_t q = q0 - lane;
        const bool stop = q < ca || codes[q] != 0xFF;
        const uint64_t m = __ballot(stop);
        if (m) {
            run += (int64_t)__ffsll((unsigned long long)m) - 1;
            break;
        }
        run += 64;
    }
    return (uint32_t)(run & 1);
}

// Issue the loads of one super-pass's chunks (P per lane).  Chunks that only
// partly overlap the code buffer (its first and last 16 bytes when they are not
// 16-byte aligned) are read byte by byte, only inside the buffer.  Fully
// unrolled, so that the compiler can count the loads in flight.
template <int CODEC>
__device__ __forceinline__ void codes_load_at(const DecodeParams& p, const Geom& g, int64_t k0, uint32_t w[][4]) {
    using C = Cfg<CODEC>;
    if constexpr (kPacked12<CODEC>) {
        // 12 bytes per chunk; three dword loads when the chunk is whole and
        // dword-aligned, bytes otherwise (only inside the stream)
        const uintptr_t lo = (uintptr_t)p.codes, hi = lo + (uintptr_t)packed12_bytes(p.n_codes);
#pragma unroll
        for (int c = 0; c < C::P; c++) {
            const int64_t k = k0 + c;
            const uintptr_t ca = g.base + (uintptr_t)k * 12u;
            uint32_t x = 0, y = 0, z = 0;
            if (k < g.nchunk) {
                if (ca + 12 <= hi && (ca & 3u) == 0) {
                    x = gload4_nt(ca);
                    y = gload4_nt(ca + 4);
                    z = gload4_nt(ca + 8);
                } else {
                    uint32_t d[3] = {0, 0, 0};
#pragma unroll
                    for (int j = 0; j < 12; j++) {
                        const uintptr_t a = ca + j;
                        if (a >= lo && a < hi) d[j >> 2] |= gload1(a) << (8 * (j & 3));
                    }
                    x = d[0]; y = d[1]; z = d[2];
                }
            }
            // 8 codes of 12 bits, least significant first, into 16-bit halves
            const uint32_t c0 = x & 0xfffu, c1 = (x >> 12) & 0xfffu;
            const uint32_t c2 = __builtin_amdgcn_alignbit(y, x, 24) & 0xfffu, c3 = (y >> 4) & 0xfffu;
            const uint32_t c4 = (y >> 16) & 0xfffu, c5 = __builtin_amdgcn_alignbit(z, y, 28) & 0xfffu;
            const uint32_t c6 = (z >> 8) & 0xfffu, c7 = z >> 20;
            w[c][0] = c0 | (c1 << 16);
            w[c][1] = c2 | (c3 << 16);
            w[c][2] = c4 | (c5 << 16);
            w[c][3] = c6 | (c7 << 16);
        }
        return;
    }
    const uintptr_t lo = (uintptr_t)p.codes, hi = lo + (uintptr_t)p.n_codes * C::CB;
#pragma unroll
    for (int c = 0; c < C::P; c++) {
        const int64_t k = k0 + c;
        const uintptr_t ca = g.base + (uintptr_t)k * 16;
        w[c][0] = w[c][1] = w[c][2] = w[c][3] = 0;
        if (k < g.nchunk) {
            if (ca >= lo && ca + 16 <= hi) {
                const u32x4 v = gload16_nt(ca);
                w[c][0] = v.x; w[c][1] = v.y; w[c][2] = v.z; w[c][3] = v.w;
            } else {
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    const uintptr_t x = ca + j;
                    if (x >= lo && x < hi) w[c][j >> 2] |= gload1(x) << (8 * (j & 3));
                }
            }
        }
    }
}

// The chunks of super-pass sp that lane ltid() owns.
template <int CODEC>
__device__ __forceinline__ void codes_load(const DecodeParams& p, const Geom& g, int sp, uint32_t w[][4]) {
    codes_load_at<CODEC>(p, g, (int64_t)sp * kWG * Cfg<CODEC>::P + (int64_t)ltid() * Cfg<CODEC>::P, w);
}

// Per-lane state of one super-pass between its length scan and its emit.
template <int CODEC> struct Lane {
    static constexpr int P = Cfg<CODEC>::P;
    uint32_t w[P][4];      // code bytes, chunk by chunk
    uint32_t valid;        // bit j: code j inside the tile's code range
    uint32_t lit;          // FSST-8: literal positions
    uint32_t tot;          // decoded bytes of the lane
    uint32_t lane_pre;     // exclusive prefix of the lane inside the super-pass
    uint32_t lenp[P][Cfg<CODEC>::CPC / 4];   // per-code lengths, packed bytes
    u32x4 tok[kIsOnpair<CODEC> ? Cfg<CODEC>::CPC : 1];   // OnPair token entries of the chunk being assembled
};

// Load the FSST-8 table into LDS (once per workgroup).  Lengths 0 / above 8
// record EBADDICT and leave every code invalid (no symbol byte is read).
// fsst_len[c]: symbol length, 0x80 for codes that are not symbols, 0 for the
// escape code 255.
template <typename S>
__device__ void fsst_build_table(S& s, const DecodeParams& p) {
    constexpr int CPT = 256 / kWG;     // codes per thread, consecutive
    const unsigned tid = ltid();
    if (p.fsst_tab) {                  // prepared with the dictionary: a copy
#pragma unroll
        for (int i = 0; i < CPT; i++) {
            const int c = (int)tid * CPT + i;
            s.fsst_tab[c] = p.fsst_tab[c];
            s.fsst_len[c] = p.fsst_len[c];
        }
        __syncthreads();
        return;
    }
    uint32_t len[CPT], tl = 0;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < CPT; i++) {
        const int c = (int)tid * CPT + i;
        len[i] = 0;
        if (c < p.n_sym) {
            len[i] = p.dict_lens[c];
            bad |= (len[i] == 0 || len[i] > 8);
        }
        tl += len[i];
    }
    bad = __syncthreads_or(bad);
    if (bad) {
        if (tid == 0) record_error(p.err, kRankDict, FD_EBADDICT);
#pragma unroll
        for (int i = 0; i < CPT; i++) {
            const int c = (int)tid * CPT + i;
            s.fsst_tab[c] = 0;
            s.fsst_len[c] = (c == 255) ? 0 : 0x80;
        }
        __syncthreads();
        return;
    }
    const unsigned lane = tid & 63, wv = tid >> 6;
    const uint32_t incl = wave_incl_scan(tl);
    if (lane == 63) s.wsum[wv] = incl;
    __syncthreads();
    uint32_t start = incl - tl;
    for (unsigned i = 0; i < wv; i++) start += s.wsum[i];
#pragma unroll
    for (int i = 0; i < CPT; i++) {
        const int c = (int)tid * CPT + i;
        uint64_t v = 0;
        for (uint32_t j = 0; j < len[i]; j++) v |= (uint64_t)p.dict_bytes[start + j] << (8 * j);
        start += len[i];
        s.fsst_tab[c] = v;
        s.fsst_len[c] = (c == 255) ? 0 : (c < p.n_sym ? (uint8_t)len[i] : (uint8_t)0x80);
    }
    __syncthreads();
}

// 12-bit codes name at most 4,096 tokens: their lengths are copied into LDS
// (from the prepared dictionary's length table) once per workgroup and
// dictionary.
template <typename S>
__device__ void len12_load(S& s, const DecodeParams& p) {
    for (unsigned i = ltid(); i < 4096 / 16; i += kWG) ((uint4*)s.len12)[i] = ((const uint4*)p.tok_len)[i];
    __syncthreads();
}

// --------------------------------------------------------------------------
// per-chunk length scans
// --------------------------------------------------------------------------
// FSST-8: 16 codes; lit/valid/esc are the chunk's 16 bits.  Writes the
// per-code prefix bytes (| escape bit) and lengths, returns the chunk total.
template <typename S>
__device__ __forceinline__ uint32_t fsst_chunk_lengths(S& s, const uint32_t (&w)[4], uint32_t lit, uint32_t valid,
                                                       uint32_t esc, uint32_t (&pre)[4], uint32_t (&lenp)[4],
                                                       uint32_t& bad) {
    // the chunk's 16 length reads are all issued before any of them is used
    uint32_t lws[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t vn = (valid >> (q * 4)) & 0xfu;
        const uint32_t ln = (lit >> (q * 4)) & vn & 0xfu;
        // literals and codes outside the tile read as 255 (length 0 in the table)
        const uint32_t x = w[q] | nib_to_ff((~vn & 0xfu) | ln);
        lws[q] = (uint32_t)s.fsst_len[x & 0xffu] | ((uint32_t)s.fsst_len[(x >> 8) & 0xffu] << 8) |
                 ((uint32_t)s.fsst_len[(x >> 16) & 0xffu] << 16) | ((uint32_t)s.fsst_len[x >> 24] << 24);
    }
    // codes that are not symbols (rare: one scalar branch skips them in most waves)
    if (__ballot(((lws[0] | lws[1] | lws[2] | lws[3]) & 0x80808080u) != 0u)) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t m = lws[q] & 0x80808080u;
            bad |= (((m >> 7) | (m >> 14) | (m >> 21) | (m >> 28)) & 0xfu) << (q * 4);
            lws[q] &= 0x7f7f7f7fu;
        }
    }
    uint32_t ctot = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t vn = (valid >> (q * 4)) & 0xfu;
        const uint32_t ln = (lit >> (q * 4)) & vn & 0xfu;
        const uint32_t lw = lws[q] + nib_to_bytes(ln);   // a literal is one byte
        // per-code prefix inside the chunk, as bytes (every partial sum stays below 128)
        const uint32_t incl = (lw << 8) + (lw << 16) + (lw << 24);
        pre[q] = (__builtin_amdgcn_perm(0u, ctot, 0x00000000u) + incl) | bits_to_byte_msb((esc >> (q * 4)) & 0xfu);
        lenp[q] = lw;
        ctot = __builtin_amdgcn_sad_u8(lw, 0u, ctot);
    }
    return ctot;
}

// OnPair-16: 8 codes with gathered lengths lv.
__device__ __forceinline__ uint32_t onpair_chunk_lengths(const uint32_t (&lv)[8], uint32_t valid, uint32_t (&pre)[2],
                                                         uint32_t (&lenp)[2], uint32_t& bad) {
    uint32_t ctot = 0;
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const uint32_t vb = nib_to_bytes(valid >> (q * 4)) * 0xffu;   // 0xFF per code inside the tile
        const uint32_t lw = (lv[q * 4] | (lv[q * 4 + 1] << 8) | (lv[q * 4 + 2] << 16) | (lv[q * 4 + 3] << 24)) & vb;
        // a code inside the tile with length 0 is not a token
        const uint32_t z = ~(((lw & 0x7f7f7f7fu) + 0x7f7f7f7fu) | lw) & vb & 0x80808080u;
        if (__ballot(z != 0u)) bad |= (((z >> 7) | (z >> 14) | (z >> 21) | (z >> 28)) & 0xfu) << (q * 4);
        // per-code prefix inside the chunk, as bytes (every partial sum stays below 256)
        pre[q] = __builtin_amdgcn_perm(0u, ctot, 0x00000000u) + (lw << 8) + (lw << 16) + (lw << 24);
        lenp[q] = lw;
        ctot = __builtin_amdgcn_sad_u8(lw, 0u, ctot);
    }
    return ctot;
}

// --------------------------------------------------------------------------
// length scan of one super-pass (codes already in L.w).  Writes pre8, cbase,
// lane_pre and the staging windows to LDS and returns the super-pass total.
// `carry` is the FSST-8 escape parity entering the super-pass (updated).
// Windows are runs of whole lanes: lane l belongs to window lane_pre / K with
// K = WIN - (largest lane output), so no lane straddles a window edge.
// --------------------------------------------------------------------------
template <int CODEC, typename S>
__device__ __forceinline__ uint32_t lengths(S& s, const DecodeParams& p, const Geom& g, int sp, Lane<CODEC>& L,
                                            uint32_t& carry, bool gather_tokens,
                                            const __amdgpu_buffer_rsrc_t& r_len,
                                            const __amdgpu_buffer_rsrc_t& r_tok) {
    using C = Cfg<CODEC>;
    constexpr int P = C::P, CPC = C::CPC, CPL = C::CPL;
    const unsigned tid = ltid(), lane = tid & 63, wv = tid >> 6;
    const int64_t k0 = (int64_t)sp * kWG * P + (int64_t)tid * P;
    const int64_t q0 = g.pos0 + k0 * CPC;
    {
        const int64_t lo = min(max(g.a - q0, (int64_t)0), (int64_t)CPL);
        const int64_t hi = min(max(g.b - q0, (int64_t)0), (int64_t)CPL);
        const uint32_t mhi = hi >= 32 ? 0xffffffffu : ((1u << (uint32_t)hi) - 1u);
        const uint32_t mlo = lo >= 32 ? 0xffffffffu : ((1u << (uint32_t)lo) - 1u);
        L.valid = mhi & ~mlo;
    }
    uint32_t tot = 0, bad = 0;
    uint32_t pre8w[P][CPC / 4];
    uint16_t cb[P];
    if constexpr (CODEC == kFsst8) {
        uint32_t ffb[P * 4];                      // 0x80 in each byte that is 255
#pragma unroll
        for (int c = 0; c < P; c++)
#pragma unroll
            for (int q = 0; q < 4; q++) ffb[c * 4 + q] = ff_bytes(L.w[c][q]);
        uint32_t F = ff_mask32(ffb) & L.valid;    // bit j: code j is 255
        // the parity entering the tile, at its first code
        if (tid == 0) F |= tile_entry_mask(g.a - q0, carry);
        const bool all_ff = (F == 0xffffffffu);
        const uint32_t trail = __clz(~F);                       // 255s at the top of the lane
        const uint64_t M = __ballot(!all_ff), T = __ballot(trail & 1u);
        const uint64_t m = M & ((1ull << lane) - 1ull);
        if (lane == 0) s.wpar[wv] = M ? (1u | ((uint32_t)((T >> (63 - __clzll(M))) & 1ull) << 1)) : 0u;
        __syncthreads();
        // the parity entering the tile (written to s.cin by wave 0 before the
        // barrier); applied at the first code already when the tile starts
        // inside a chunk
        const uint32_t c0 = g.a > g.pos0 ? 0u : uniform32(s.cin);
        uint32_t cw = c0, cout = c0;
#pragma unroll
        for (int i = 0; i < kNWave; i++) {
            const uint32_t v = s.wpar[i];
            if ((v & 1u) && i < (int)wv) cw = v >> 1;
            if (v & 1u) cout = v >> 1;
        }
        carry = cout;
        const uint32_t cin = m ? (uint32_t)((T >> (63 - __clzll(m))) & 1ull) : cw;
        uint32_t esc;
        classify_escapes(F, cin, esc, L.lit);
        L.lit &= L.valid;
#pragma unroll
        for (int c = 0; c < P; c++) {
            cb[c] = (uint16_t)tot;
            tot += fsst_chunk_lengths(s, L.w[c], L.lit >> (16 * c), L.valid >> (16 * c), esc >> (16 * c), pre8w[c],
                                      L.lenp[c], bad);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        // the token lengths only: the lengths (and so the tile total the
        // look-back publishes) wait for nothing else
        uint32_t lv[P][8];
#pragma unroll
        for (int c = 0; c < P; c++)
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint32_t cj = (L.w[c][j >> 1] >> (16 * (j & 1))) & 0xffffu;
                if constexpr (kPacked12<CODEC>)
                    lv[c][j] = s.len12[cj & 0xfffu];
                else
                    lv[c][j] = __builtin_amdgcn_raw_buffer_load_b8(r_len, cj, 0, 0);
            }
        // (the token entries are gathered by the assembly of the lane's window;
        // these two parameters are unused but kept: without them the register
        // allocation of the OnPair-16 kernel changes, from 4 spills to 64-90)
        (void)gather_tokens;
        (void)r_tok;
#pragma unroll
        for (int c = 0; c < P; c++) {
            uint32_t cbad = 0;
            cb[c] = (uint16_t)tot;
            tot += onpair_chunk_lengths(lv[c], L.valid >> (8 * c), pre8w[c], L.lenp[c], cbad);
            bad |= cbad << (8 * c);
        }
    }
    const uint64_t errkey = bad ? data_error_key(q0 + __builtin_ctz(bad), FD_EBADCODE) : ~0ull;
    wave_record_error(p.err, errkey);
    L.tot = tot;
    const uint32_t incl = wave_incl_scan(tot);
    if (lane == 63) {
        s.wsum[wv] = incl;
        s.wlast[wv] = tot;
    }
    __builtin_memcpy(&s.pre8[tid * P * CPC], pre8w, P * CPC);
#pragma unroll
    for (int c = 0; c < P; c++) s.cbase[tid * P + c] = cb[c];
    __syncthreads();
    uint32_t basew = 0, total = 0;
#pragma unroll
    for (int i = 0; i < kNWave; i++) {
        const uint32_t v = s.wsum[i];
        basew += (i < (int)wv) ? v : 0u;
        total += v;
    }
    L.lane_pre = basew + incl - tot;
    s.lane_pre[tid] = L.lane_pre;
    // staging windows: window of a lane = lane_pre / K; first lanes record
    // bases (window 0 starts at 0).  A tile whose output fits one window (the
    // usual case) needs no barrier here: its window count and end are read
    // after the cursor step's barrier.
    constexpr uint32_t K = C::WIN - C::CPL * C::W;   // a lane writes at most CPL * W bytes
    if (uniform32(total) < K) {
        if (tid == 0) {
            s.nwin = 1;
            s.wbase[0] = 0;
            s.wbase[1] = total;
        }
        return uniform32(total);
    }
    {
        const uint32_t wl = L.lane_pre / K;
        const uint32_t tprev = __shfl_up(tot, 1u);
        const uint32_t pprev = lane ? L.lane_pre - tprev : (wv ? basew - s.wlast[wv - 1] : 0u);
        const uint32_t wprev = tid ? pprev / K : 0xffffffffu;
        if (wl != wprev) s.wbase[wl] = L.lane_pre;
        if (tid == kWG - 1) {
            s.nwin = wl + 1;
            s.wbase[wl + 1] = total;
        }
    }
    __syncthreads();
    return uniform32(total);
}

// --------------------------------------------------------------------------
// assembly of one window into s.stage.  Lanes of other windows return.  The
// result does not depend on the output position, so it can overlap the
// look-back.
// --------------------------------------------------------------------------
// 128 bits as two 64-bit halves (little-endian byte order: byte 0 is the low
// byte of lo)
struct U128 {
    uint64_t lo, hi;
};

// OR the 16 bytes (lo, hi) into the staging window at byte offset q: three
// 64-bit LDS ORs at the aligned words q & ~7 .. (q & ~7) + 16, the last two
// only where they carry bytes.  Aligned atomics cost a fraction of a store at
// a byte-granular address, and ORing into zeroed memory leaves every other
// byte as it is, so entries and lanes need no order among themselves.
__device__ __forceinline__ void lds_or16(uint8_t* stage, int q, uint64_t lo, uint64_t hi) {
    const uint32_t o8 = 8u * ((uint32_t)q & 7u), rs = 63u - o8;
    const uint64_t r0 = lo << o8;
    const uint64_t r1 = (hi << o8) | ((lo >> 1) >> rs);      // (two shifts: o8 = 0 needs no select)
    const uint64_t r2 = (hi >> 1) >> rs;
    unsigned long long* d = (unsigned long long*)&stage[q & ~7];
    __hip_atomic_fetch_or(d, (unsigned long long)r0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (r1) __hip_atomic_fetch_or(d + 1, (unsigned long long)r1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (r2) __hip_atomic_fetch_or(d + 2, (unsigned long long)r2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Every token (FSST-8: every pair of tokens) is ORed as a whole 16-byte
// entry, zero past its length, into the zeroed window at its offset.
template <typename S>
__device__ __forceinline__ void fsst_chunk_emit(S& s, const uint32_t (&w)[4], uint32_t lit, const uint32_t (&lenp)[4],
                                                int& q) {
    // the table reads run one pair ahead of the writes (source order keeps
    // them ahead: the compiler cannot tell the staging and the table apart)
    uint64_t n0 = s.fsst_tab[w[0] & 0xffu], n1 = s.fsst_tab[(w[0] >> 8) & 0xffu];
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
        const uint32_t l0 = (lenp[j >> 2] >> (8 * (j & 3))) & 0xffu;
        const uint32_t l1 = (lenp[(j + 1) >> 2] >> (8 * ((j + 1) & 3))) & 0xffu;
        const uint32_t b0 = (w[j >> 2] >> (8 * (j & 3))) & 0xffu;
        const uint32_t b1 = (w[(j + 1) >> 2] >> (8 * ((j + 1) & 3))) & 0xffu;
        uint64_t v0 = n0;
        uint64_t v1 = n1;
        if (j + 2 < 16) {
            n0 = s.fsst_tab[(w[(j + 2) >> 2] >> (8 * ((j + 2) & 3))) & 0xffu];
            n1 = s.fsst_tab[(w[(j + 3) >> 2] >> (8 * ((j + 3) & 3))) & 0xffu];
        }
        if ((lit >> j) & 1u) v0 = b0;             // (an escape, a code that is not a symbol and a
        if ((lit >> (j + 1)) & 1u) v1 = b1;       // code outside the tile read zero entries)
        // the pair: v0 | v1 << 8 * l0 over 128 bits, l0 in 0..8; each shift is
        // split in two of at most 32 bits, so l0 = 0 and l0 = 8 need no select
        const uint32_t sl = 4u * l0, sr = 32u - sl;
        lds_or16(s.stage, q, v0 | ((v1 << sl) << sl), (v1 >> sr) >> sr);
        q += (int)(l0 + l1);
        if ((j & 3) == 2) __builtin_amdgcn_sched_barrier(0);
    }
}

// (codes outside the tile were gathered as zero entries)
template <typename S>
__device__ __forceinline__ void onpair_chunk_emit(S& s, const u32x4* tok, const uint32_t (&lenp)[2], int& q) {
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const uint32_t l = (lenp[j >> 2] >> (8 * (j & 3))) & 0xffu;
        const u32x4 v = tok[j];
        lds_or16(s.stage, q, ((uint64_t)v.y << 32) | v.x, ((uint64_t)v.w << 32) | v.z);
        q += (int)l;
        if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
}

template <int CODEC, typename S>
__device__ __forceinline__ void assemble(S& s, Lane<CODEC>& L, int win, int c, const __amdgpu_buffer_rsrc_t& r_tok) {
    using C = Cfg<CODEC>;
    constexpr uint32_t K = C::WIN - C::CPL * C::W;
    if ((int)(L.lane_pre / K) != win || L.tot == 0) return;
    if constexpr (kIsOnpair<CODEC>) {
        // the chunk's token entries (one chunk at a time: the entries of all
        // the lane's chunks at once would not fit the registers); codes
        // outside the tile read past the entries, which the buffer load's
        // range check returns as zero
#pragma unroll
        for (int cc = 0; cc < C::P; cc++)
            if (cc == c) {
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const uint32_t cj = (L.w[cc][j >> 1] >> (16 * (j & 1))) & 0xffffu;
                    const uint32_t off = ((L.valid >> (cc * 8 + j)) & 1u) ? cj << 4 : 65536u * 16u;
                    L.tok[j] = __builtin_amdgcn_raw_buffer_load_b128(r_tok, off, 0, 0);
                }
            }
    }
    // the chunk starts after the lane's earlier chunks
    uint32_t cbase = 0;
#pragma unroll
    for (int cc = 0; cc < C::P; cc++)
#pragma unroll
        for (int i = 0; i < C::CPC / 4; i++)
            if (cc < c) cbase = __builtin_amdgcn_sad_u8(L.lenp[cc][i], 0u, cbase);
    const int lane0 = (int)(L.lane_pre - (win == 0 ? 0u : s.wbase[win]));
    int q = lane0 + (int)cbase;
    // opaque copies: keeps the compiler from hoisting every per-code predicate
    // out of the window loop (they would all stay live)
    uint32_t lit = L.lit >> (C::CPC * c), lenp[C::CPC / 4], w[4];
    asm volatile("" : "+v"(lit));
#pragma unroll
    for (int i = 0; i < C::CPC / 4; i++) { lenp[i] = L.lenp[c][i]; asm volatile("" : "+v"(lenp[i])); }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        w[i] = L.w[c][i];
        if constexpr (CODEC == kFsst8) {
            // codes outside the tile read as 255, whose table entry is zero (as
            // for an escape and a code that is not a symbol): nothing to mask later
            w[i] |= nib_to_ff(~(L.valid >> (C::CPC * c + 4 * i)));
        }
        asm volatile("" : "+v"(w[i]));
    }
    if constexpr (CODEC == kFsst8) fsst_chunk_emit(s, w, lit, lenp, q);
    else onpair_chunk_emit(s, L.tok, lenp, q);
}

// Zero the staging window before an assembly (whole 16-byte words, every
// thread a share).
template <typename S>
__device__ __forceinline__ void stage_zero(S& s) {
    constexpr int n = (int)sizeof(s.stage) / 16;
    for (int i = (int)ltid(); i < n; i += kWG) *(u32x4*)&s.stage[16 * i] = u32x4{0, 0, 0, 0};
}

// Drain window `win` (super-pass output bytes [wbase[win], wbase[win+1]))
// to the output, whose super-pass output starts at position O: aligned 16-byte
// nontemporal stores read from the staging at the output's alignment, byte
// stores for the partial head / tail chunks; nothing at or past out_cap.
template <typename S>
__device__ __forceinline__ void drain(S& s, const DecodeParams& p, int64_t O, int win) {
    const int b0 = (int)s.wbase[win];
    const int len = (int)s.wbase[win + 1] - b0;
    const int64_t X = O + b0;                                     // output position of stage[0]
    const int shift = (int)(((uintptr_t)p.out + (uintptr_t)X) & 15u);
    const int64_t cap_rel = p.out_cap - X;
    const int hi_all = (int)min((int64_t)len, max(cap_rel, (int64_t)0));
    const int nch = (shift + len + 15) >> 4;
    for (int c = ltid(); c < nch; c += kWG) {
        const int s0 = c * 16 - shift;
        if (s0 >= 0 && s0 + 16 <= hi_all) {
            // five dword-aligned LDS reads realigned in registers (a byte-granular
            // 16-byte LDS read costs several times as much)
            const uint32_t* sw = (const uint32_t*)&s.stage[s0 & ~3];
            const uint32_t r = (uint32_t)s0 & 3u;
            const uint32_t d0 = sw[0], d1 = sw[1], d2 = sw[2], d3 = sw[3], d4 = sw[4];
            u32x4 v;
            v.x = __builtin_amdgcn_alignbyte(d1, d0, r);
            v.y = __builtin_amdgcn_alignbyte(d2, d1, r);
            v.z = __builtin_amdgcn_alignbyte(d3, d2, r);
            v.w = __builtin_amdgcn_alignbyte(d4, d3, r);
            __builtin_nontemporal_store(v, (u32x4*)(p.out + X + s0));
        }
    }
    // the partial chunks: the first one and the one holding the last byte
    // below the capacity, one byte per lane
    if (ltid() < 32 && hi_all > 0) {
        const int c_last = (shift + hi_all - 1) >> 4;
        const int c = ltid() < 16 ? 0 : c_last;
        const int s0 = c * 16 - shift;
        const bool full = s0 >= 0 && s0 + 16 <= hi_all;
        const int y = s0 + (int)(ltid() & 15u);
        if (!full && (ltid() < 16 || c_last != 0) && y >= 0 && y < hi_all) p.out[X + y] = s.stage[y];
    }
}

// A thread's share of the prefetched code offsets: entries S0 + r kWG + tid
// (consecutive threads, consecutive entries), and thread 0 also the entry
// before S0.
template <int CODEC, typename IDX> struct OffRegs {
    static constexpr int R = kOffR<CODEC>;
    IDX v[R];
    IDX before;
};

template <int CODEC, typename IDX>
__device__ __forceinline__ void offsets_prefetch(const DecodeParams& p, int64_t S0, OffRegs<CODEC, IDX>& r) {
    const IDX* co = (const IDX*)p.code_off;
    const int64_t i0 = S0 + (int64_t)ltid();
    const int64_t lim = min(S0 + (int64_t)p.off_pref - 1, p.n_strings);
#pragma unroll
    for (int k = 0; k < OffRegs<CODEC, IDX>::R; k++)
        r.v[k] = (i0 + (int64_t)k * kWG <= lim) ? co[i0 + (int64_t)k * kWG] : (IDX)0;
    r.before = (ltid() == 0 && S0 > 0) ? co[S0 - 1] : (IDX)0;
}

template <int CODEC, typename IDX, typename S>
__device__ __forceinline__ void offsets_stage(S& s, const OffRegs<CODEC, IDX>& r) {
    constexpr int R = OffRegs<CODEC, IDX>::R;
    const unsigned tid = ltid();
#pragma unroll
    for (int k = 0; k < R; k++) s.off[1 + k * kWG + tid] = (int64_t)r.v[k];
    if (tid == 0) s.off[0] = (int64_t)r.before;
}

// Decoded bytes of the tile's codes before code position x (a <= x <= b).
template <int CODEC, typename S>
__device__ __forceinline__ uint32_t local_prefix(S& s, const Geom& g, int64_t x, uint32_t total) {
    using C = Cfg<CODEC>;
    if (x >= g.b) return total;
    const int64_t r = x - g.pos0;
    const int k = (int)(r / C::CPC), jj = (int)(r - (int64_t)k * C::CPC);
    uint32_t e = s.pre8[k * C::CPC + jj];
    if constexpr (CODEC == kFsst8) e &= 0x7fu;
    return s.lane_pre[k / C::P] + (uint32_t)s.cbase[k] + e;
}

// Arrow offsets of the strings starting in the tile (output position O, total
// decoded bytes `total`; OUT = false: no output, the checks only), the FSST-8
// dangling-escape check of the strings that end in it, and the checks of
// every code offset it reads.
//
// The tile reads the code offsets from index G gcur on (gcur: its coarse
// group, so code_offsets[G gcur] is below its first position) in steps of one
// per thread, until the first index e whose offset is at or past own_hi.  On
// valid offsets its first string comes at most G entries after G gcur, and e
// is the next tile's first string, which lies within G entries after the next
// tile's start G gnext: both are checked, so that the ranges the tiles read
// meet end to end and every pair of adjacent offsets is compared by some
// tile (a decreasing pair anywhere is found, whatever the coarse index holds).
template <int CODEC, typename IDX, bool OUT, typename S>
__device__ __forceinline__ void tile_offsets(S& s, const DecodeParams& p, const Geom& g, int64_t t, int64_t O,
                                             uint32_t total, uint32_t cin, int64_t ca, int64_t gcur, int64_t gnext) {
    constexpr int R = kOffR<CODEC>;
    const IDX* co = (const IDX*)p.code_off;
    IDX* oo = (IDX*)p.out_off;
    const unsigned tid = ltid(), lane = tid & 63, w = tid >> 6;
    const int64_t n = p.n_strings;
    const int64_t G = (int64_t)1 << p.g_shift;
    const int64_t S0 = min(max(gcur, (int64_t)0) << p.g_shift, n);
    bool bad = false, found = false;
    int64_t e = INT64_MAX;               // the first index at or past own_hi
    // blocks of up to kWG R entries, entry base + k kWG + tid for thread tid:
    // the first block is the off_pref entries prefetched into LDS, any further
    // one (a tile with many strings) is loaded here
    int64_t span = p.off_pref;
    for (int64_t base = S0, blk = 0; base <= n; base += span, span = (int64_t)kWG * R, blk++) {
        int64_t wfirst = INT64_MAX;      // the wave's first entry at or past own_hi
        bool wfound = false;
#pragma unroll
        for (int k = 0; k < R; k++) {
            const int64_t idx = (int64_t)k * kWG + tid;
            const int64_t i = base + idx;
            const bool in = idx < span && i <= n;
            int64_t v = 0, vp = 0;
            if (in) {
                if (blk == 0) {
                    v = s.off[1 + idx];
                    vp = s.off[idx];
                } else {
                    v = (int64_t)co[i];
                    vp = i > 0 ? (int64_t)co[i - 1] : 0;
                }
                if (i == 0) bad |= v < 0;
                else bad |= v < vp;
                if (i == n) bad |= v > p.n_codes;
            }
            const bool past = in && v >= g.own_hi;
            if (in && !past && v >= g.own_lo) {
                const int64_t x = min(max(v, g.a), g.b);
                if constexpr (OUT) oo[i] = (IDX)(O + (int64_t)local_prefix<CODEC>(s, g, x, total));
                if constexpr (CODEC == kFsst8) {
                    // the string ending at v ends with an escape iff v is a literal position
                    if (v > ca && x == v) {
                        const bool esc = (x == g.a) ? (cin != 0)
                                                    : ((s.pre8[(int)(x - 1 - g.pos0)] & 0x80u) != 0u);
                        if (esc) atomicMin(p.err, (unsigned long long)data_error_key(x - 1, FD_EESCAPE));
                    }
                }
            }
            // entries rise with k, then with the lane: the wave's first past one is
            // in the lowest k with any, at the lowest such lane
            const uint64_t bp = __ballot(past);
            if (bp && wfirst == INT64_MAX)
                wfirst = base + (int64_t)k * kWG + (int64_t)(w * 64) + (int64_t)__ffsll((unsigned long long)bp) - 1;
            wfound = wfound || __ballot(in && v >= g.own_lo) != 0;
        }
        // the workgroup's: through LDS, slots alternating between blocks (one barrier each)
        if (lane == 0) {
            s.pfirst[blk & 1][w] = wfirst;
            s.vote[blk & 1][w] = wfound ? 1u : 0u;
        }
        __syncthreads();
        bool any_found = false;
#pragma unroll
        for (int q = 0; q < kNWave; q++) {
            e = min(e, s.pfirst[blk & 1][q]);
            any_found = any_found || s.vote[blk & 1][q] != 0u;
        }
        e = uniform64(e);
        found = found || any_found;
        if (e != INT64_MAX) break;
        // on valid offsets the tile's first string comes by index S0 + G (or
        // there is none: then the column ends before the tile, and S0 = n)
        const int64_t last = base + span - 1;
        if (!found && last >= S0 + G && last < n) {
            bad = true;
            break;
        }
    }
    if (tid == 0 && t + 1 < p.n_tiles) {
        const int64_t S1 = min(max(gnext, (int64_t)0) << p.g_shift, n);
        const int64_t ee = (e == INT64_MAX) ? n + 1 : e;
        if (ee < S1 || ee > S1 + G) bad = true;
    }
    if (bad) record_error(p.err, kRankOffsets, FD_EOFFSETS);
}

// --------------------------------------------------------------------------
// decoupled look-back over tiles grouped in blocks of kBlk (wave 0 only).  The
// exclusive prefix of tile t of block b is the sum of the aggregates of the
// earlier tiles of block b plus the inclusive prefix of block b - 1, which
// comes from the block states (empty, the block's aggregate, or its inclusive
// prefix) by walking back over aggregates to the first inclusive prefix.  The
// last tile of a block publishes the block's aggregate and then its inclusive
// prefix.  With PREV, a tile that finds block b - 1's state still empty sums
// the aggregates of that block's kBlk tiles instead (each published as soon as
// its tile knew its total, long before the block's last tile learns the
// block's), and the first kHelpers tiles of block b also publish block b - 1's
// inclusive prefix.  Publishers of one state all write the same value; a state
// overwritten by an older kind is still correct.  Split in parts so that the
// loads of the first round overlap the assembly.
// --------------------------------------------------------------------------
constexpr int kHelpers = 2;
static_assert(kBlk <= 64, "one lane of wave 0 per tile of a block");

struct LookBack {
    uint64_t in_v;      // lane l: aggregate of tile l of the block (l < jt)
    uint64_t prev_v;    // lane l: aggregate of tile l of the previous block
    uint64_t blk_v;     // lane l: state of block b - 1 - l
    uint64_t inb = 0;   // sum of the earlier tiles of the block, once known
    bool inb_ok = false;
};

__device__ __forceinline__ uint64_t lb_load(const unsigned long long* a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lb_publish(unsigned long long* a, uint64_t v) {
    __hip_atomic_store(a, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the missing values of the first round, again (one round trip)
template <bool PREV>
__device__ __forceinline__ void lb_reload(const DecodeParams& p, int64_t blk, int jt, LookBack& lb) {
    const unsigned lane = ltid() & 63;
    if ((int)lane < jt && (lb.in_v & kFlagMask) == 0) lb.in_v = lb_load(&p.tagg[(blk << kBlkShift) + lane]);
    if (PREV && blk >= 1 && (int)lane < kBlk && (lb.prev_v & kFlagMask) == 0)
        lb.prev_v = lb_load(&p.tagg[((blk - 1) << kBlkShift) + lane]);
    const int64_t idx = blk - 1 - (int64_t)lane;
    if (idx >= 0 && (lb.blk_v & kFlagMask) != kFlagIncl) lb.blk_v = lb_load(&p.bstate[idx]);
}

template <bool PREV>
__device__ __forceinline__ void lookback_issue(const DecodeParams& p, int64_t t, uint64_t A, LookBack& lb) {
    const unsigned lane = ltid() & 63;
    const int64_t blk = t >> kBlkShift;
    const int jt = (int)(t & (kBlk - 1));
    if (lane == 0)
        __hip_atomic_store(&p.tagg[t], (unsigned long long)(kFlagAgg | A), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // values that are not needed start as found (an aggregate of 0 / an
    // inclusive prefix of 0), the others as empty
    lb.in_v = (int)lane < jt ? 0ull : kFlagAgg;
    lb.prev_v = PREV && blk >= 1 && (int)lane < kBlk ? 0ull : kFlagAgg;
    lb.blk_v = blk - 1 - (int64_t)lane >= 0 ? 0ull : kFlagIncl;
    lb_reload<PREV>(p, blk, jt, lb);
}

// Block b - 1's aggregate from its tiles, when its state is still empty and
// every tile's aggregate has arrived (lane 0 holds block b - 1's state).
__device__ __forceinline__ bool lb_prev_from_tiles(LookBack& lb, uint64_t& agg) {
    const unsigned lane = ltid() & 63;
    const uint64_t v0 = __shfl(lb.blk_v, 0);
    if ((v0 & kFlagMask) != 0 || __ballot((lb.prev_v & kFlagMask) == 0) != 0) return false;
    agg = wave_sum_u64(lb.prev_v & kValueMask);
    if (lane == 0) lb.blk_v = kFlagAgg | agg;
    return true;
}

// Midway through the tile's assembly: the sums known from the first round are
// taken and published (the block aggregate by the block's last tile, the
// previous block's aggregate by whoever sees all its tiles), and the values
// still missing are loaded again.
template <bool PREV>
__device__ __forceinline__ void lookback_mid(const DecodeParams& p, int64_t t, uint64_t A, LookBack& lb) {
    const unsigned lane = ltid() & 63;
    const int64_t blk = t >> kBlkShift;
    const int jt = (int)(t & (kBlk - 1));
    if (__ballot((lb.in_v & kFlagMask) == 0) == 0) {
        lb.inb = wave_sum_u64(lb.in_v & kValueMask);
        lb.inb_ok = true;
        if (jt == kBlk - 1 && lane == 0) lb_publish(&p.bstate[blk], kFlagAgg | (lb.inb + A));
    }
    uint64_t agg;
    if (PREV && blk >= 1) (void)lb_prev_from_tiles(lb, agg);
    lb_reload<PREV>(p, blk, jt, lb);
}

// Completes the look-back; returns the exclusive prefix of tile t.
template <bool PREV>
__device__ __forceinline__ uint64_t lookback_finish(const DecodeParams& p, int64_t t, uint64_t A, LookBack lb) {
    const unsigned lane = ltid() & 63;
    const int64_t blk = t >> kBlkShift;
    const int jt = (int)(t & (kBlk - 1));
    bool fail = false;
    uint32_t spins = 0;
    uint64_t inb = lb.inb;
    for (; !lb.inb_ok;) {
        if (__ballot((lb.in_v & kFlagMask) == 0) == 0) {
            inb = wave_sum_u64(lb.in_v & kValueMask);
            break;
        }
        if (++spins >= kSpinLimit) { fail = true; break; }
        __builtin_amdgcn_s_sleep(1);
        lb_reload<PREV>(p, blk, jt, lb);     // all first-round values in one round trip
    }
    if (!lb.inb_ok && jt == kBlk - 1 && lane == 0) lb_publish(&p.bstate[blk], kFlagAgg | (inb + A));
    // walk back over the block states: lane l holds block j - l
    uint64_t bb = 0;
    int64_t j = blk - 1;
    bool prev_incl = false;              // block b - 1's inclusive prefix was published
    while (j >= 0 && !fail) {
        uint64_t agg;
        if (PREV && j == blk - 1) (void)lb_prev_from_tiles(lb, agg);
        const uint64_t v = lb.blk_v;
        const uint64_t fl = v & kFlagMask;
        const uint64_t incl = __ballot(fl == kFlagIncl);
        const uint64_t empty = __ballot(fl == 0);
        const int first = incl ? (int)__ffsll((unsigned long long)incl) - 1 : 63;
        const uint64_t need = (first >= 63) ? ~0ull : ((2ull << first) - 1ull);
        if (empty & need) {
            if (++spins >= kSpinLimit) { fail = true; break; }
            __builtin_amdgcn_s_sleep(1);
            if (j == blk - 1) {
                lb_reload<PREV>(p, blk, 0, lb);
            } else {
                const int64_t idx = j - (int64_t)lane;
                if (idx >= 0 && fl != kFlagIncl) lb.blk_v = lb_load(&p.bstate[idx]);
            }
        } else {
            if (j == blk - 1 && (incl & 1ull)) prev_incl = true;
            bb += wave_sum_u64(((int)lane <= first) ? (v & kValueMask) : 0ull);
            if (incl) break;
            j -= 64;
            const int64_t idx = j - (int64_t)lane;
            lb.blk_v = kFlagIncl;
            if (idx >= 0) lb.blk_v = lb_load(&p.bstate[idx]);
        }
    }
    if (fail && lane == 0) record_error(p.err, kRankInternal, FD_EHIP);
    const uint64_t excl = bb + inb;
    if (!fail && lane == 0) {
        if (PREV && blk >= 1 && !prev_incl && jt < kHelpers) lb_publish(&p.bstate[blk - 1], kFlagIncl | bb);
        if (jt == kBlk - 1) lb_publish(&p.bstate[blk], kFlagIncl | (excl + A));
    }
    return excl;
}

// The next tile's codes are loaded into registers during the current tile's
// drain, except in the FSST-8 passes whose positions are known (expand,
// sidecar): there the eight registers would cost a fifth workgroup per CU,
// which measured 3-4% faster than the prefetch.  The FSST-8 single pass keeps
// the prefetch (without it, at five workgroups, it spilled and ran 9% slower).
template <int CODEC, int MODE> constexpr bool kPrefetchCodes = !(CODEC == kFsst8 && MODE != kModeLookback);
// Waves per SIMD the decode kernels are compiled for: FSST-8 five workgroups
// per CU without the code prefetch (at most 96 VGPRs; their LDS, 31.5 KiB
// each, fits five), four with it; the OnPair kernels three (their 32 KiB
// staging window leaves room in the LDS for three workgroups).
template <int CODEC, int MODE>
constexpr int kMinWaves = CODEC == kFsst8 ? (kPrefetchCodes<CODEC, MODE> ? 4 : 5) : CODEC == kOnpair12s ? 4 : 3;

// Whether the look-back sums the previous block's tiles (measured: FSST-8
// gains, OnPair-16, whose tiles publish later and wait mostly inside their
// own block, loses to the extra loads).
template <int CODEC> constexpr bool kPrevTiles = CODEC == kFsst8;

// --------------------------------------------------------------------------
// where a launch's tiles come from: one column, or a batch of columns whose
// tiles are numbered consecutively (column c owns ids first_tile[c] ..
// first_tile[c + 1] - 1; each column has its own look-back state)
// --------------------------------------------------------------------------
struct OneColumn {
    static constexpr bool kBatch = false;
    const DecodeParams& p;
    __device__ int64_t n_tiles() const { return p.n_tiles; }
    __device__ unsigned* counter() const { return p.counters; }
    __device__ int column(int64_t, int) const { return 0; }
    __device__ const DecodeParams& params(int) const { return p; }
    __device__ int64_t first(int) const { return 0; }
};

struct ColumnBatch {
    static constexpr bool kBatch = true;
    const DecodeParams* __restrict__ cols;
    const int64_t* __restrict__ first_tile;   // n_cols + 1
    int32_t n_cols;
    int64_t total;
    unsigned* ctr;
    __device__ int64_t n_tiles() const { return total; }
    __device__ unsigned* counter() const { return ctr; }
    // the column of global tile id v (v < total); `hint` is a likely answer
    __device__ int column(int64_t v, int hint) const {
        if (first_tile[hint] <= v && v < first_tile[hint + 1]) return hint;
        int lo = 0, hi = n_cols - 1;            // the last c with first_tile[c] <= v
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first_tile[mid] <= v) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    __device__ const DecodeParams& params(int c) const { return cols[c]; }
    __device__ int64_t first(int c) const { return first_tile[c]; }
};

// --------------------------------------------------------------------------
// The tile queues of a launch (thread 0 of a workgroup uses them): tiles
// [0, n_all) split into nq contiguous ranges, range q taken in order through
// its counter.  take() issues the atomic on the current range; resolve()
// turns its result into a tile id.  When the current range is used up it
// reads all the counters at once (one round trip, not one atomic per range)
// and moves on to the first later range that still had tiles, or returns
// n_all when none had: a counter only grows, so a range seen used up stays
// so, and a workgroup stops only after it has seen every range used up.
// Each tile is taken exactly once (by the atomic that returned its index).
// --------------------------------------------------------------------------
struct TileQueue {
    unsigned* base;       // counter block
    int64_t n_all;
    int nq, q;
    __device__ TileQueue(unsigned* b, int64_t n, int queues)
        : base(b), n_all(n), nq(queues), q((int)(blockIdx.x % (unsigned)queues)) {}
    __device__ int64_t lo(int k) const { return (int64_t)k * n_all / nq; }
    __device__ unsigned* ctr(int k) const { return &base[kQueueStride * (k + 1)]; }
    __device__ unsigned take() const { return atomicAdd(ctr(q), 1u); }
    __device__ int64_t resolve(unsigned raw) {
        for (;;) {
            const int64_t t = lo(q) + (int64_t)raw;
            if (t < lo(q + 1)) return t;
            if (nq == 1) return n_all;
            unsigned c[kQueues];
#pragma unroll
            for (int k = 0; k < kQueues; k++)
                c[k] = k < nq ? __hip_atomic_load(ctr(k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
            int next = -1;
            for (int i = 1; i < nq && next < 0; i++) {
                const int k = (q + i) % nq;
                if (lo(k) + (int64_t)c[k] < lo(k + 1)) next = k;
            }
            if (next < 0) return n_all;
            q = next;
            raw = take();
        }
    }
};

// --------------------------------------------------------------------------
// the decode loop of one workgroup: tiles from the queues until they run out
// --------------------------------------------------------------------------
template <int CODEC, typename IDX, int MODE, typename SRC>
__device__ __forceinline__ void decode_tiles(SmemT<CODEC>& s, const SRC& src) {
    using C = Cfg<CODEC>;
    constexpr int P = C::P;
    const unsigned tid = ltid(), wv = tid >> 6;
    int64_t n_all = src.n_tiles();
    if constexpr (!SRC::kBatch) {
        // a single column's tiles past the one holding the end of its decode
        // range have no work (a slice of the code buffer; a selection decoded
        // in a buffer sized for more codes): the queues cover only the tiles
        // up to it, so that no workgroup starts on a range of empty tiles
        const DecodeParams& p0 = src.params(0);
        int64_t x0 = 0, x1 = 0;
        if (tid == 0) {
            column_range<IDX>(p0, x0, x1);
            s.hdr[0] = x0;
            s.hdr[1] = x1;
        }
        __syncthreads();
        n_all = min(n_all, last_tile(p0, uniform64(s.hdr[0]), uniform64(s.hdr[1])) + 1);
    }
    // Tiles come from counters (dynamic shares measured faster than fixed
    // ones: they spread the workgroups of a CU over different steps of their
    // tiles).  The look-back needs them taken in increasing order: one queue.
    TileQueue tq(src.counter(), n_all, MODE == kModeLookback ? 1 : kQueues);
    if (tid == 0) s.next_id = (int32_t)tq.resolve(tq.take());
    __syncthreads();
    int64_t v = (int64_t)(uint32_t)uniform32((uint32_t)s.next_id);
    int col = -1;
    const void* table_src = nullptr;      // the table in LDS (FSST-8 symbols, 12-bit lengths)
    int64_t ca = 0, cb = 0;               // the column's decode range
    int64_t t_first = 0, t_last = -1;     // its tiles with work (divisions once per column)
    // loaded during the previous tile for tile id pf_v (same column): its
    // coarse groups, its stored cursor and the next tile's (expand mode) and,
    // FSST-8, wave 0's bytes of the window before its first code.  Kept as
    // loaded (per-lane registers) until the tile starts, so that nothing
    // waits for them earlier.
    int64_t pf_v = -1, pf_g0 = 0, pf_g1 = 0, pf_c0 = 0, pf_c1 = 0;
    uint32_t pf_byte = 0;
    uint32_t pf_w[P][4];                  // and its codes (their loads overlap this tile's drain and offsets)
    if constexpr (CODEC == kFsst8 && !SRC::kBatch) {
        fsst_build_table(s, src.params(0));
        table_src = (const void*)1;
    }
    if constexpr (kPacked12<CODEC> && !SRC::kBatch) {
        len12_load(s, src.params(0));
        table_src = (const void*)1;
    }
    while (v < n_all) {
        const int c = src.column(v, col < 0 ? 0 : col);
        const DecodeParams& p = src.params(c);
        if (c != col) {
            if constexpr (SRC::kBatch) {
                // a column of another dictionary: its table (columns of one
                // prepared dictionary share it)
                if constexpr (CODEC == kFsst8) {
                    if (p.fsst_tab ? (const void*)p.fsst_tab != table_src : true) {
                        fsst_build_table(s, p);
                        table_src = p.fsst_tab;
                    }
                }
                if constexpr (kPacked12<CODEC>) {
                    if ((const void*)p.tok_len != table_src) {
                        len12_load(s, p);
                        table_src = p.tok_len;
                    }
                }
            }
            col = c;
            int64_t x0 = 0, x1 = 0;
            if (tid == 0) column_range<IDX>(p, x0, x1);
            if (tid == 0) { s.hdr[0] = x0; s.hdr[1] = x1; }
            __syncthreads();
            ca = uniform64(s.hdr[0]);
            cb = uniform64(s.hdr[1]);
            t_first = first_tile(p, ca, cb);
            t_last = last_tile(p, ca, cb);
        }
        const int64_t t = v - src.first(col);
        const bool after = t > t_last;
        if (after || t < t_first) {
            // a tile outside the decode range: no codes, no strings.  Past the
            // tile that holds the range's end, no later tile of the column looks
            // at it; before the one holding its start, the look-back of the tiles
            // after it reads it as a total of zero
            if (!SRC::kBatch && after) break;
            if (tid == 0) {
                if constexpr (MODE == kModeLookback) {
                    if (!after) {
                        lb_publish(&p.tagg[t], kFlagAgg);
                        if ((t & (kBlk - 1)) == kBlk - 1) lb_publish(&p.bstate[t >> kBlkShift], kFlagIncl);
                    }
                }
                s.next_id = (int32_t)tq.resolve(tq.take());
            }
            __syncthreads();
            v = (int64_t)(uint32_t)uniform32((uint32_t)s.next_id);
            __syncthreads();
            continue;
        }
        const Geom g = make_geom<CODEC>(p, t, ca, cb);
        // OnPair-16 gathers go through range-checked buffer loads (FSST-8 keeps its table in LDS)
        const __amdgpu_buffer_rsrc_t r_len = make_rsrc(
            kIsOnpair<CODEC> ? (const void*)p.tok_len : (const void*)p.codes, kIsOnpair<CODEC> ? 65536u : 0u);
        const __amdgpu_buffer_rsrc_t r_tok = make_rsrc(
            kIsOnpair<CODEC> ? (const void*)p.tok16 : (const void*)p.codes, kIsOnpair<CODEC> ? 65536u * 16u : 0u);

        // the coarse groups of this tile and the next (uniform loads, usually
        // made during the previous tile), the codes, then the first block of
        // the tile's code offsets: all in flight together, the offsets waited
        // for only after the length scan
        const bool pf = pf_v == v;
        const int64_t gcur = uniform64(pf ? pf_g0 : p.coarse[t]);
        const int64_t gnext = uniform64(pf ? pf_g1 : ((t + 1 < p.n_tiles) ? p.coarse[t + 1] : 0));
        // expand mode: the stored cursors of this tile and the next (used at the cursor step)
        int64_t cur0 = 0, cur1 = 0;
        if constexpr (MODE == kModeExpand) {
            cur0 = pf ? pf_c0 : (int64_t)p.tagg[t];
            cur1 = pf ? pf_c1 : (int64_t)p.tagg[t + 1];
        }
        Lane<CODEC> L;
        if (kPrefetchCodes<CODEC, MODE> && pf) {
#pragma unroll
            for (int c = 0; c < P; c++)
#pragma unroll
                for (int i = 0; i < 4; i++) L.w[c][i] = pf_w[c][i];
        } else {
            codes_load<CODEC>(p, g, 0, L.w);
        }
        OffRegs<CODEC, IDX> orr;
        offsets_prefetch<CODEC, IDX>(p, min(max(gcur, (int64_t)0) << p.g_shift, p.n_strings), orr);
        uint32_t s_cin_local = 0;
        if constexpr (CODEC == kFsst8) {
            if (wv == 0) {
                const int64_t ca_c = min(max(ca, (int64_t)0), p.n_codes);
                const uint32_t first = pf ? pf_byte : fsst_window_byte(p.codes, ca_c, g.a);
                s_cin_local = fsst_carry_in_from(p.codes, ca_c, g.a, first);
                if (tid == 0) s.cin = s_cin_local;
            }
        }
        // (the previous tile's drain is done: its last barrier)
        if constexpr (MODE != kModeTotals) stage_zero(s);
        // FSST-8: the entry parity, computed by wave 0 and shared through s.cin
        // at the length scan's first barrier
        uint32_t carry = 0;
        if constexpr (CODEC == kFsst8) {
            if (wv == 0) carry = s_cin_local;
        }
        // the id after this tile, published at the cursor step.  Without a
        // look-back it is requested now, so that the atomic's round trip
        // overlaps the length scan and the assembly; the single pass requests
        // it at the cursor step (tiles then start in about the order of their
        // ids, which its look-back wants)
        uint32_t nid = 0;
        if (MODE != kModeLookback && tid == 0) nid = tq.take();

        const uint32_t tot = lengths<CODEC>(s, p, g, 0, L, carry, true, r_len, r_tok);
        uint32_t cin = 0;
        if constexpr (CODEC == kFsst8) cin = uniform32(s.cin);    // (written before the scan's barriers)
        offsets_stage<CODEC, IDX>(s, orr);      // read after later barriers
        if constexpr (MODE == kModeTotals) {
            // the sidecar build: every check of the decode, the tile's total, no output
            if (tid == 0) {
                p.tagg[t] = tot;
                s.next_id = (int32_t)tq.resolve(nid);
            }
            __syncthreads();            // the staged offsets
            tile_offsets<CODEC, IDX, false>(s, p, g, t, 0, tot, cin, ca, gcur, gnext);
            v = (int64_t)(uint32_t)uniform32((uint32_t)s.next_id);
            __syncthreads();            // this tile's LDS is free for the next
            continue;
        }
        LookBack lb{};
        if constexpr (MODE == kModeLookback) {
            if (wv == 0) lookback_issue<kPrevTiles<CODEC>>(p, t, tot, lb);
        }
        assemble<CODEC>(s, L, 0, 0, r_tok);
        if constexpr (MODE == kModeLookback) {
            if (wv == 0) lookback_mid<kPrevTiles<CODEC>>(p, t, tot, lb);
        }
#pragma unroll
        for (int cc = 1; cc < P; cc++) assemble<CODEC>(s, L, 0, cc, r_tok);
        if constexpr (MODE == kModeLookback) {
            if (wv == 0) {
                const uint64_t ex = lookback_finish<kPrevTiles<CODEC>>(p, t, tot, lb);
                if (tid == 0) s.cursor = (int64_t)ex;
            }
        } else {
            if (tid == 0) {
                int64_t cur = cur0, nxt = cur1;
                if constexpr (SRC::kBatch) {
                    // a batch group's cursors are scanned over all its columns:
                    // relative to the column's first tile
                    const int64_t b0 = (int64_t)p.tagg[0];
                    cur -= b0;
                    nxt -= b0;
                }
                s.cursor = checked_cursor(p, t, cur, nxt, tot);
            }
        }
        // the next tile's id
        if (tid == 0) s.next_id = (int32_t)tq.resolve(MODE == kModeLookback ? tq.take() : nid);
        __syncthreads();
        const int64_t cursor = uniform64(s.cursor);
        // the next tile's coarse groups and first window, loaded now (they
        // arrive during this tile's drain and offsets)
        {
            const int64_t vn = (int64_t)(uint32_t)uniform32((uint32_t)s.next_id);
            pf_v = -1;
            if (vn < n_all && src.column(vn, col) == col) {
                const int64_t tn = vn - src.first(col);
                if (tn >= t_first && tn <= t_last) {
                    pf_v = vn;
                    pf_g0 = p.coarse[tn];
                    pf_g1 = (tn + 1 < p.n_tiles) ? p.coarse[tn + 1] : 0;
                    if constexpr (MODE == kModeExpand) {
                        pf_c0 = (int64_t)p.tagg[tn];
                        pf_c1 = (int64_t)p.tagg[tn + 1];
                    }
                    const Geom gn = make_geom<CODEC>(p, tn, ca, cb);
                    if constexpr (kPrefetchCodes<CODEC, MODE>) codes_load<CODEC>(p, gn, 0, pf_w);
                    if constexpr (CODEC == kFsst8) {
                        if (wv == 0) pf_byte = fsst_window_byte(p.codes, min(max(ca, (int64_t)0), p.n_codes), gn.a);
                    }
                }
            }
        }
        if (cursor >= 0) {
            const int nwin = (int)uniform32(s.nwin);
            for (int win = 0; win < nwin; win++) {
                // window 0 was assembled before the cursor step's barrier
                if (win > 0) {
                    __syncthreads();            // the previous window's drain is done
                    stage_zero(s);
                    __syncthreads();
#pragma unroll
                    for (int cc = 0; cc < P; cc++) assemble<CODEC>(s, L, win, cc, r_tok);
                    __syncthreads();
                }
                drain(s, p, cursor, win);
            }
            tile_offsets<CODEC, IDX, true>(s, p, g, t, cursor, tot, cin, ca, gcur, gnext);
            if (tid == 0) {
                const int64_t endv = cursor + (int64_t)tot;
                if (sizeof(IDX) == 4 && endv > (int64_t)INT32_MAX) record_error(p.err, kRankOverflow, FD_EOVERFLOW);
                if (endv > p.out_cap) record_error(p.err, kRankCapacity, FD_ECAPACITY);
            }
        }
        v = (int64_t)(uint32_t)uniform32((uint32_t)s.next_id);
        __syncthreads();                // this tile's LDS is free for the next
    }
}

// --------------------------------------------------------------------------
// the decode kernels: one column, or a batch of columns of one codec and
// offset width (the statuses of a batch are collected by k_batch_status)
// --------------------------------------------------------------------------
template <int CODEC, typename IDX, int MODE>
__global__ void __launch_bounds__(kWG, (kMinWaves<CODEC, MODE>)) k_decode(DecodeParams p) {
    __shared__ SmemT<CODEC> s;
    decode_tiles<CODEC, IDX, MODE>(s, OneColumn{p});

    // the last workgroup to finish publishes the status
    if (MODE != kModeTotals) {
        __threadfence();
        if (ltid() == 0) {
            const unsigned prev = atomicAdd(&p.counters[0], 1u);
            if (prev == gridDim.x - 1) {
                __threadfence();
                const unsigned long long e = __hip_atomic_load(p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int st = (e == ~0ull) ? FD_OK : (int)(e & 15ull);
                if (p.status) *p.status = st;
                if (p.status2) *p.status2 = st;
            }
        }
    }
}

template <int CODEC, typename IDX, int MODE>
__global__ void __launch_bounds__(kWG, (kMinWaves<CODEC, MODE>)) k_decode_batch(const DecodeParams* __restrict__ cols,
                                                      const int64_t* __restrict__ first_tile, int32_t n_cols,
                                                      int64_t total, unsigned* ctr) {
    __shared__ SmemT<CODEC> s;
    decode_tiles<CODEC, IDX, MODE>(s, ColumnBatch{cols, first_tile, n_cols, total, ctr});
}

// Statuses of a batch: column c's error word -> status[c]; the first error in
// column order -> status[n_cols] (one workgroup).
__global__ void __launch_bounds__(256) k_batch_status(const unsigned long long* errs, int32_t n_cols,
                                                      int32_t* status, int32_t* status2) {
    __shared__ int s_first;
    if (ltid() == 0) s_first = n_cols;
    __syncthreads();
    for (int c = ltid(); c < n_cols; c += blockDim.x) {
        const unsigned long long e = errs[c];
        const int st = (e == ~0ull) ? FD_OK : (int)(e & 15ull);
        if (status) status[c] = st;
        if (st != FD_OK) atomicMin(&s_first, c);
    }
    __syncthreads();
    if (ltid() == 0) {
        int st = FD_OK;
        if (s_first < n_cols) {
            const unsigned long long e = errs[s_first];
            st = (int)(e & 15ull);
        }
        if (status) status[n_cols] = st;
        if (status2) *status2 = st;
    }
}

// Workspace reset of a batch: n words zeroed, then the n_cols error words set to "none".
__global__ void k_batch_reset(unsigned long long* z, int64_t n, unsigned long long* errs, int32_t n_cols) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + ltid();
    for (int64_t k = i0; k < n; k += (int64_t)gridDim.x * blockDim.x) z[k] = 0;
    for (int64_t k = i0; k < n_cols; k += (int64_t)gridDim.x * blockDim.x) errs[k] = ~0ull;
}

// --------------------------------------------------------------------------
// workspace reset, cursor scan (three-phase mode), OnPair dictionary repack
// --------------------------------------------------------------------------
__global__ void k_reset(unsigned long long* err, unsigned* counters, unsigned long long* z, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + ltid();
    if (i == 0) {
        if (err) *err = ~0ull;
        for (int q = 0; q <= kQueues; q++) counters[q * kQueueStride] = 0;
    }
    for (int64_t k = i; k < n; k += (int64_t)gridDim.x * blockDim.x) z[k] = 0;
}

// Single-workgroup exclusive scan of tile totals into tile cursors (in place);
// with err non-null, the status of the errors recorded so far is published
// after it (the sidecar build, whose totals pass publishes none).
__global__ void __launch_bounds__(1024) k_scan_totals(unsigned long long* v, int64_t n,
                                                      const unsigned long long* err, int32_t* status,
                                                      int32_t* status2) {
    __shared__ uint64_t s_w[16];
    __shared__ uint64_t s_carry;
    const unsigned tid = ltid(), lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + tid;
        const uint64_t x = i < n ? v[i] : 0;
        uint64_t incl = x;
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(incl, d, 64);
            if (lane >= (unsigned)d) incl += y;
        }
        if (lane == 63) s_w[w] = incl;
        __syncthreads();
        uint64_t pre = s_carry, tot = 0;
        for (int k = 0; k < 16; k++) {
            if (k < (int)w) pre += s_w[k];
            tot += s_w[k];
        }
        if (i < n) v[i] = pre + incl - x;
        __syncthreads();
        if (tid == 0) s_carry += tot;
        __syncthreads();
    }
    if (err && tid == 0) {
        const unsigned long long e = *err;
        const int st = (e == ~0ull) ? FD_OK : (int)(e & 15ull);
        if (status) *status = st;
        if (status2) *status2 = st;
    }
}

// Repack an OnPair dictionary (packed bytes + lengths) into fixed 16-byte
// entries and a full 65,536-entry length table (0 for codes >= n_tok).
// 256 workgroups of 256 threads; workgroup g handles codes [256 g, 256 g + 256).
// A length of 0 or above 16 records EBADDICT and leaves every code invalid.
__global__ void __launch_bounds__(256) k_onpair_prepare(const uint8_t* bytes, const uint8_t* lens, int32_t n_tok,
                                                         uint4* tok16, uint8_t* tok_len, unsigned long long* err,
                                                         int* bad_flag) {
    __shared__ uint32_t s_w[4];
    __shared__ uint64_t s_red[4];
    const unsigned tid = ltid(), lane = tid & 63, w = tid >> 6;
    const int32_t c0 = (int32_t)blockIdx.x * 256;
    bool bad = false;
    uint64_t before = 0;
    for (int32_t c = tid; c < n_tok; c += 256) {
        const uint32_t l = lens[c];
        bad |= (l == 0 || l > 16);
        if (c < c0) before += l;
    }
    bad = __syncthreads_or(bad);
    if (bad) {
        tok16[c0 + tid] = make_uint4(0, 0, 0, 0);
        tok_len[c0 + tid] = 0;
        if (blockIdx.x == 0 && tid == 0) {
            record_error(err, kRankDict, FD_EBADDICT);
            if (bad_flag) *bad_flag = 1;
        }
        return;
    }
    before = wave_sum_u64(before);
    if (lane == 0) s_red[w] = before;
    const int32_t c = c0 + (int32_t)tid;
    const uint32_t l = (c < n_tok) ? lens[c] : 0u;
    const uint32_t incl = wave_incl_scan(l);
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    const uint64_t base = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    uint32_t ex = incl - l;
    for (unsigned i = 0; i < w; i++) ex += s_w[i];
    uint32_t v[4] = {0, 0, 0, 0};
    const uint8_t* src = bytes + base + ex;
    for (uint32_t j = 0; j < l; j++) v[j >> 2] |= (uint32_t)src[j] << (8 * (j & 3));
    tok16[c] = make_uint4(v[0], v[1], v[2], v[3]);
    tok_len[c] = (uint8_t)l;
}

// --------------------------------------------------------------------------
// three-phase mode, first phase: every tile's decoded total, streamed (no
// validation and no assembly; the expand phase validates everything and
// checks each tile's total against the cursors scanned from these).  One wave
// per tile, without barriers, so that many tiles' loads are in flight: the
// wave walks the tile's chunks 64 lanes x P at a time, loading each step's
// chunks one step ahead.  The FSST-8 escape parity entering a tile comes from
// the run of 255 bytes just before it; inside the tile it runs on across
// strings exactly as in the expand phase's scan (in valid data no string ends
// inside a run of escapes of odd length).
// OnPair-16 token lengths as nibbles in LDS (32 KiB): 16 lengths (bytes of
// 0..16) become 8 bytes, code 2k in the low nibble of byte k, each length l
// stored as (l - 1) mod 16 (so 1..16 as 0..15; byte-wise, l + 15 <= 31 does
// not carry).  Dword k then holds codes 8k..8k+7, code 8k + i at bits 4i.
__device__ __forceinline__ void nib_table_load(uint8_t* s_nib, const uint8_t* tok_len) {
    for (unsigned i = ltid(); i < 65536 / 16; i += blockDim.x) {
        const uint4 a = ((const uint4*)tok_len)[i];
        const uint32_t x[4] = {a.x, a.y, a.z, a.w};
        uint32_t h[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t y = (x[k] + 0x0f0f0f0fu) & 0x0f0f0f0fu;
            const uint32_t z = y | (y >> 4);
            h[k] = (z & 0xffu) | ((z >> 8) & 0xff00u);
        }
        ((uint2*)s_nib)[i] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
}

// A code's length from the nibble table: the nibble plus one; codes at or
// past the dictionary's size count 0.
__device__ __forceinline__ uint32_t nib_length(const uint8_t* s_nib, uint32_t cj, int32_t n_tok) {
    const uint32_t nib = ((uint32_t)s_nib[cj >> 1] >> ((cj & 1u) * 4u)) & 0xfu;
    return (int)cj < n_tok ? nib + 1u : 0u;
}

// --------------------------------------------------------------------------
template <int CODEC, typename IDX>
__global__ void __launch_bounds__(kWG) k_tile_totals(DecodeParams p) {
    using C = Cfg<CODEC>;
    constexpr int P = C::P, CPC = C::CPC, CPL = C::CPL;
    constexpr int64_t CPI = 64 * P;               // chunks per step of a wave
    __shared__ uint8_t s_len[256];
    __shared__ alignas(16) uint8_t s_len12[kPacked12<CODEC> ? 4096 : 16];
    __shared__ alignas(16) uint8_t s_nib[CODEC == kOnpair16 ? 32768 : 16];
    const unsigned tid = ltid(), lane = tid & 63;
    if constexpr (kPacked12<CODEC>) {             // 12-bit codes: their 4,096 lengths
        for (unsigned i = tid; i < 4096 / 16; i += kWG) ((uint4*)s_len12)[i] = ((const uint4*)p.tok_len)[i];
        __syncthreads();
    }
    if constexpr (CODEC == kOnpair16) {           // OnPair-16: the lengths as nibbles
        nib_table_load(s_nib, p.tok_len);
        __syncthreads();
    }
    if constexpr (CODEC == kFsst8) {
        // per code its length: 0 for the escape and for codes that are not symbols
        for (unsigned c = tid; c < 256; c += kWG) {
            uint32_t l;
            if (p.fsst_len) {
                l = p.fsst_len[c];
                l = (l & 0x80u) ? 0u : l;
            } else {
                l = ((int)c < p.n_sym) ? (uint32_t)p.dict_lens[c] : 0u;
            }
            s_len[c] = (c == 255) ? 0 : (uint8_t)l;
        }
        __syncthreads();
    }
    const __amdgpu_buffer_rsrc_t r_len = make_rsrc(
        kIsOnpair<CODEC> ? (const void*)p.tok_len : (const void*)p.codes, kIsOnpair<CODEC> ? 65536u : 0u);
    int64_t ca, cb;                               // the decode range
    column_range<IDX>(p, ca, cb);
    ca = uniform64(ca);
    cb = uniform64(cb);
    const int64_t ca_c = min(max(ca, (int64_t)0), p.n_codes);
    const int64_t nw = (int64_t)gridDim.x * kNWave;
    // the tiles outside [first_tile, last_tile] have zero totals (zeroed)
    const int64_t t_end = last_tile(p, ca, cb) + 1;
    for (int64_t t = first_tile(p, ca, cb) + (int64_t)blockIdx.x * kNWave + (tid >> 6); t < t_end; t += nw) {
        const Geom g = make_geom<CODEC>(p, t, ca, cb);
        const int64_t steps = (g.nchunk + CPI - 1) / CPI;
        uint32_t carry = 0;
        if constexpr (CODEC == kFsst8) carry = fsst_carry_in(p.codes, ca_c, g.a);
        uint64_t total = 0;
        uint32_t wn[P][4];                        // the next step's chunks, loaded a step ahead
        if (steps > 0) codes_load_at<CODEC>(p, g, (int64_t)lane * P, wn);
        for (int64_t it = 0; it < steps; it++) {
            const int64_t k0 = it * CPI + (int64_t)lane * P;
            uint32_t w[P][4];
#pragma unroll
            for (int c = 0; c < P; c++)
#pragma unroll
                for (int q = 0; q < 4; q++) w[c][q] = wn[c][q];
            if (it + 1 < steps) codes_load_at<CODEC>(p, g, k0 + CPI, wn);
            // the lane's codes inside the tile, bits [lo, hi) of 32 (tile-relative, so 32-bit)
            const int32_t rel = (int32_t)(k0 * CPC);
            const int32_t lo = min(max((int32_t)(g.a - g.pos0) - rel, 0), CPL);
            const int32_t hi = min(max((int32_t)(g.b - g.pos0) - rel, 0), CPL);
            const uint32_t valid = (uint32_t)(~0ull << lo) & ~(uint32_t)(~0ull << hi);
            uint32_t tot = 0;
            if constexpr (CODEC == kFsst8) {
                uint32_t m[P * 4];                // 0x80 in each byte that is 255
#pragma unroll
                for (int c = 0; c < P; c++)
#pragma unroll
                    for (int q = 0; q < 4; q++) m[c * 4 + q] = ff_bytes(w[c][q]);
                // Common case: every code of the step is inside the tile and no
                // two 255 are adjacent (text never holds a literal 255), the
                // parity entering the step included.  Then every 255 is an
                // escape and a literal is simply the code after a 255: the 255
                // bytes shifted by one code, across dwords and from the lane below.
                const int64_t s0 = g.pos0 + it * CPI * CPC;   // the step's first code
                bool fast = uniform32(s0 >= g.a && s0 + CPI * CPC <= g.b ? 1u : 0u) != 0;
                uint32_t L[P * 4];                // 0x80 in each byte that is a literal
                uint64_t E = 0;                   // lanes whose last code is 255
                if (fast) {
                    E = __ballot(m[P * 4 - 1] >> 31);
                    uint32_t prev = (uint32_t)(((E << 1) | carry) >> lane) << 31, adj = 0;
#pragma unroll
                    for (int d = 0; d < P * 4; d++) {
                        L[d] = __builtin_amdgcn_alignbit(m[d], prev, 24);
                        adj |= m[d] & L[d];       // a 255 after a 255 (or after the carry)
                        prev = m[d];
                    }
                    fast = __ballot(adj != 0u) == 0;
                }
                if (fast) {
                    carry = (uint32_t)(E >> 63);
#pragma unroll
                    for (int d = 0; d < P * 4; d++) {
                        // literals count 1 each and read as 255 (length 0, as escapes)
                        const uint32_t x = w[d >> 2][d & 3] | L[d] | (L[d] - (L[d] >> 7));
                        tot += (uint32_t)__builtin_popcount(L[d]);
                        tot += (uint32_t)s_len[x & 0xffu] + (uint32_t)s_len[(x >> 8) & 0xffu] +
                               (uint32_t)s_len[(x >> 16) & 0xffu] + (uint32_t)s_len[x >> 24];
                    }
                } else {
                    uint32_t F = ff_mask32(m) & valid;   // bit j: code j is 255
                    if (it == 0) {                // the parity entering the tile, at its first code
                        if (lane == 0) F |= tile_entry_mask(g.a - g.pos0, carry);
                        if (g.a > g.pos0) carry = 0;
                    }
                    // the parity entering each lane: the trailing run of the nearest
                    // lower lane that is not all escapes, else the previous step's
                    const bool all_ff = (F == 0xffffffffu);
                    const uint32_t trail = __clz(~F);
                    const uint64_t M = __ballot(!all_ff), T = __ballot(trail & 1u);
                    const uint64_t mb = M & ((1ull << lane) - 1ull);
                    const uint32_t cin = mb ? (uint32_t)((T >> (63 - __clzll(mb))) & 1ull) : carry;
                    if (M) carry = (uint32_t)((T >> (63 - __clzll(M))) & 1ull);
                    uint32_t esc, lit;
                    classify_escapes(F, cin, esc, lit);
                    lit &= valid;
                    // literals count 1 each; they and the codes outside the tile are
                    // read as 255, whose length is 0 (as an escape's), so every other
                    // code adds its table length
                    tot = (uint32_t)__builtin_popcount(lit);
                    const uint32_t fix = ~valid | lit;
#pragma unroll
                    for (int c = 0; c < P; c++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const uint32_t x = w[c][q] | nib_to_ff(fix >> (c * 16 + q * 4));
                            tot += (uint32_t)s_len[x & 0xffu] + (uint32_t)s_len[(x >> 8) & 0xffu] +
                                   (uint32_t)s_len[(x >> 16) & 0xffu] + (uint32_t)s_len[x >> 24];
                        }
                }
            } else {
                const int64_t s0 = g.pos0 + it * CPI * CPC;   // the step's first code
                const bool full = uniform32(s0 >= g.a && s0 + CPI * CPC <= g.b ? 1u : 0u) != 0;
                if (CODEC == kOnpair16 && full && p.n_sym >= 65536) {
                    // every code of the step inside the tile and a token: each
                    // dword of codes (two) reads two dwords of the nibble table
                    // and extracts the nibbles at 4 (code mod 8), whose offsets
                    // the bit-field extract takes from the low five bits of its
                    // operand; the + 1 of every length is added once
                    const uint32_t* s_nib32 = (const uint32_t*)s_nib;
                    tot = (uint32_t)(P * CPC);
#pragma unroll
                    for (int c = 0; c < P; c++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const uint32_t x = w[c][q];
                            tot += __builtin_amdgcn_ubfe(s_nib32[(x & 0xffffu) >> 3], x << 2, 4u) +
                                   __builtin_amdgcn_ubfe(s_nib32[x >> 19], (x >> 14) & 0x1cu, 4u);
                        }
                } else if (kPacked12<CODEC> && full) {
#pragma unroll
                    for (int c = 0; c < P; c++)
#pragma unroll
                        for (int j = 0; j < CPC; j++)
                            tot += s_len12[(w[c][j >> 1] >> (16 * (j & 1))) & 0xfffu];
                } else {
#pragma unroll
                    for (int c = 0; c < P; c++)
#pragma unroll
                        for (int j = 0; j < CPC; j++) {
                            const int b = c * CPC + j;
                            const uint32_t cj = (w[c][j >> 1] >> (16 * (j & 1))) & 0xffffu;
                            uint32_t l;
                            if constexpr (kPacked12<CODEC>)
                                l = s_len12[cj & 0xfffu];
                            else
                                l = nib_length(s_nib, cj, p.n_sym);
                            tot += ((valid >> b) & 1u) ? l : 0u;
                        }
                }
            }
            total += tot;
        }
        total = wave_sum_u64(total);
        if (lane == 0) p.tagg[t] = total;
    }
}

// The same totals with a workgroup per tile (OnPair: the length table in LDS
// serves four waves; batches: all waves of a workgroup work on one column, so
// its LDS table serves them).  The source's tile v goes to out[v]; each
// workgroup takes tiles blockIdx.x, + gridDim.x, ... of one column, or a
// contiguous range of a batch's tiles, and reloads its table when the
// dictionary changes.
template <int CODEC, typename IDX, typename SRC>
__device__ void totals_tiles_wg(const SRC& src, unsigned long long* out) {
    using C = Cfg<CODEC>;
    constexpr int P = C::P, CPC = C::CPC, CPL = C::CPL;
    // OnPair-16: the 65,536 token lengths as nibbles in LDS (16 stored as 0),
    // read once per workgroup and dictionary instead of a gather per code
    constexpr bool kNib = CODEC == kOnpair16;
    __shared__ uint8_t s_len[256];
    __shared__ alignas(16) uint8_t s_len12[kPacked12<CODEC> ? 4096 : 16];
    __shared__ alignas(16) uint8_t s_nib[kNib ? 32768 : 16];
    __shared__ uint32_t s_wpar[kNWave];
    __shared__ uint64_t s_wsum[kNWave];
    __shared__ int64_t s_nb[2];
    const unsigned tid = ltid(), lane = tid & 63, wv = tid >> 6;
    __shared__ uint32_t s_cin;
    const void* table = nullptr;                  // the dictionary whose lengths are in LDS
    int col = 0, hdr_col = -1;
    int64_t ca = 0, cb = 0;                       // the decode range of column hdr_col
    // one column: tiles blockIdx.x, + gridDim.x, ...; a batch: a contiguous
    // range of tiles per workgroup, so that it reloads its table only where
    // its range crosses into a column of another dictionary
    const int64_t n_all = src.n_tiles();
    const int64_t v_begin = SRC::kBatch ? (int64_t)blockIdx.x * n_all / gridDim.x : (int64_t)blockIdx.x;
    const int64_t v_end = SRC::kBatch ? ((int64_t)blockIdx.x + 1) * n_all / gridDim.x : n_all;
    const int64_t v_step = SRC::kBatch ? 1 : (int64_t)gridDim.x;
    for (int64_t v = v_begin; v < v_end; v += v_step) {
        col = src.column(v, col);
        const DecodeParams& p = src.params(col);
        const int64_t t = v - src.first(col);
        if constexpr (CODEC == kFsst8) {
            const void* d = p.fsst_len ? (const void*)p.fsst_len : (const void*)p.dict_lens;
            if (d != table) {
                // per code its length: 0 for the escape and for codes that are not symbols
                for (unsigned c = tid; c < 256; c += kWG) {
                    uint32_t l;
                    if (p.fsst_len) {
                        l = p.fsst_len[c];
                        l = (l & 0x80u) ? 0u : l;
                    } else {
                        l = ((int)c < p.n_sym) ? (uint32_t)p.dict_lens[c] : 0u;
                    }
                    s_len[c] = (c == 255) ? 0 : (uint8_t)l;
                }
                table = d;
            }
        } else if constexpr (kPacked12<CODEC>) {
            if ((const void*)p.tok_len != table) {   // 12-bit codes: their 4,096 lengths
                for (unsigned i = tid; i < 4096 / 16; i += kWG) ((uint4*)s_len12)[i] = ((const uint4*)p.tok_len)[i];
                table = p.tok_len;
            }
        } else if constexpr (kNib) {
            if ((const void*)p.tok_len != table) {
                nib_table_load(s_nib, p.tok_len);
                table = p.tok_len;
            }
        }
        const __amdgpu_buffer_rsrc_t r_len = make_rsrc(
            kIsOnpair<CODEC> ? (const void*)p.tok_len : (const void*)p.codes, kIsOnpair<CODEC> ? 65536u : 0u);
        if (col != hdr_col) {
            if (tid == 0) column_range<IDX>(p, s_nb[0], s_nb[1]);
            __syncthreads();                      // s_nb, and the table when it was reloaded
            ca = uniform64(s_nb[0]);
            cb = uniform64(s_nb[1]);
            hdr_col = col;
        }
        if (t > last_tile(p, ca, cb) || t < first_tile(p, ca, cb)) continue;   // zero totals (zeroed)
        const Geom g = make_geom<CODEC>(p, t, ca, cb);
        if constexpr (CODEC == kFsst8) {
            if (wv == 0) {
                const uint32_t ci = fsst_carry_in(p.codes, min(max(ca, (int64_t)0), p.n_codes), g.a);
                if (tid == 0) s_cin = ci;
            }
        }
        __syncthreads();                          // s_cin, and the table when it was reloaded
        uint32_t carry = 0;
        if constexpr (CODEC == kFsst8) carry = uniform32(s_cin);
        uint64_t total = 0;
        for (int sp = 0; sp < (g.nchunk > 0 ? 1 : 0); sp++) {
            uint32_t w[P][4];
            codes_load<CODEC>(p, g, sp, w);
            const int64_t k0 = (int64_t)sp * kWG * P + (int64_t)tid * P;
            const int64_t q0 = g.pos0 + k0 * CPC;
            const int64_t lo = min(max(g.a - q0, (int64_t)0), (int64_t)CPL);
            const int64_t hi = min(max(g.b - q0, (int64_t)0), (int64_t)CPL);
            const uint32_t mhi = hi >= 32 ? 0xffffffffu : ((1u << (uint32_t)hi) - 1u);
            const uint32_t mlo = lo >= 32 ? 0xffffffffu : ((1u << (uint32_t)lo) - 1u);
            const uint32_t valid = mhi & ~mlo;
            uint32_t tot = 0;
            if constexpr (CODEC == kFsst8) {
                uint32_t ffb[P * 4];              // 0x80 in each byte that is 255
#pragma unroll
                for (int c = 0; c < P; c++)
#pragma unroll
                    for (int q = 0; q < 4; q++) ffb[c * 4 + q] = ff_bytes(w[c][q]);
                uint32_t F = ff_mask32(ffb) & valid;   // bit j: code j is 255
                if (tid == 0) F |= tile_entry_mask(g.a - q0, carry);   // the parity entering the tile
                if (g.a > g.pos0) carry = 0;
                const bool all_ff = (F == 0xffffffffu);
                const uint32_t trail = __clz(~F);
                const uint64_t M = __ballot(!all_ff), T = __ballot(trail & 1u);
                const uint64_t m = M & ((1ull << lane) - 1ull);
                if (lane == 0) s_wpar[wv] = M ? (1u | ((uint32_t)((T >> (63 - __clzll(M))) & 1ull) << 1)) : 0u;
                __syncthreads();
                uint32_t cw = carry, cout = carry;
#pragma unroll
                for (int i = 0; i < kNWave; i++) {
                    const uint32_t vw = s_wpar[i];
                    if ((vw & 1u) && i < (int)wv) cw = vw >> 1;
                    if (vw & 1u) cout = vw >> 1;
                }
                carry = cout;
                const uint32_t cin = m ? (uint32_t)((T >> (63 - __clzll(m))) & 1ull) : cw;
                uint32_t esc, lit;
                classify_escapes(F, cin, esc, lit);
                lit &= valid;
                // literals count 1 each; they and the codes outside the tile read
                // as 255 (length 0)
                tot = (uint32_t)__builtin_popcount(lit);
                const uint32_t fix = ~valid | lit;
#pragma unroll
                for (int c = 0; c < P; c++)
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const uint32_t x = w[c][q] | nib_to_ff(fix >> (c * 16 + q * 4));
                        tot += (uint32_t)s_len[x & 0xffu] + (uint32_t)s_len[(x >> 8) & 0xffu] +
                               (uint32_t)s_len[(x >> 16) & 0xffu] + (uint32_t)s_len[x >> 24];
                    }
                __syncthreads();                  // s_wpar of the next super-pass
            } else {
#pragma unroll
                for (int c = 0; c < P; c++)
#pragma unroll
                    for (int q = 0; q < CPC / 4; q++) {
                        uint32_t lw = 0;          // four lengths as bytes, codes outside the tile masked
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const int j = q * 4 + r;
                            const uint32_t cj = (w[c][j >> 1] >> (16 * (j & 1))) & 0xffffu;
                            if constexpr (kPacked12<CODEC>) {
                                lw |= (uint32_t)s_len12[cj & 0xfffu] << (8 * r);
                            } else if constexpr (kNib) {
                                lw |= nib_length(s_nib, cj, p.n_sym) << (8 * r);
                            } else {
                                lw |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r_len, cj, 0, 0) << (8 * r);
                            }
                        }
                        lw &= nib_to_bytes(valid >> (c * CPC + q * 4)) * 0xffu;
                        tot = __builtin_amdgcn_sad_u8(lw, 0u, tot);
                    }
            }
            total += tot;
        }
        total = wave_sum_u64(total);
        if (lane == 0) s_wsum[wv] = total;
        __syncthreads();
        if (tid == 0) {
            uint64_t sum = 0;
#pragma unroll
            for (int i = 0; i < kNWave; i++) sum += s_wsum[i];
            out[v] = sum;
        }
        __syncthreads();                          // s_wsum, s_cin and the table of the next tile
    }
}

template <int CODEC, typename IDX>
__global__ void __launch_bounds__(kWG) k_tile_totals_wg(DecodeParams p) {
    totals_tiles_wg<CODEC, IDX>(OneColumn{p}, p.tagg);
}

// A batch group's tile totals, in global tile order: out[v] for tile v.
template <int CODEC, typename IDX>
__global__ void __launch_bounds__(kWG) k_tile_totals_batch(const DecodeParams* __restrict__ cols,
                                                           const int64_t* __restrict__ first_tile, int32_t n_cols,
                                                           int64_t total, unsigned long long* out) {
    totals_tiles_wg<CODEC, IDX>(ColumnBatch{cols, first_tile, n_cols, total, nullptr}, out);
}

// --------------------------------------------------------------------------
// The coarse string index of a column.  Sample j is code_offsets[min(j G, n)]
// (j = 0 .. J, J = ceil(n / G)); coarse[t] is the largest j whose sample lies
// below tile t's first position t T (0 when none does, which the zeroed array
// already holds).  Sample j covers the tiles t >= 1 with c_j < t T <= c_{j+1}
// (c_{J+1} taken as past the last tile).  A wave handles 64 samples and writes
// their tiles together, a loop step per 64 tiles, so a sample spanning many
// tiles (a very long string) does not serialise one lane.  On decreasing
// offsets some tiles keep their zero or get any candidate: the decode's
// offsets step checks what it reads against the index and reports EOFFSETS.
// --------------------------------------------------------------------------
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t x) {
    const unsigned lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= (unsigned)d) x += y;
    }
    return x;
}

template <typename IDX>
__device__ __forceinline__ void coarse_column(const DecodeParams& p) {
    const unsigned lane = lane_id();
    const IDX* co = (const IDX*)p.code_off;
    const int64_t n = p.n_strings, T = p.tile_codes, nt = p.n_tiles;
    const int sh = p.g_shift;
    const int64_t J = (n + ((int64_t)1 << sh) - 1) >> sh;
    // only the tiles up to the one after the tile holding the end of the
    // range are read (the later ones are skipped by the decode)
    const int64_t cb = min(max((int64_t)co[n], (int64_t)0), p.n_codes);
    const int64_t t_max = min(cb / T + 1, nt - 1);
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + ltid(); j - (int64_t)lane <= J; j += step) {
        int64_t t_lo = 0, len = 0;
        if (j <= J) {
            const int64_t c0 = (int64_t)co[min(j << sh, n)];
            const int64_t c1 = (j < J) ? (int64_t)co[min((j + 1) << sh, n)] : INT64_MAX;
            const int64_t lo_t = max(c0 < 0 ? (int64_t)1 : c0 / T + 1, (int64_t)1);
            const int64_t hi_t = (c1 == INT64_MAX) ? t_max : (c1 < 0 ? (int64_t)-1 : min(c1 / T, t_max));
            if (hi_t >= lo_t) {
                t_lo = lo_t;
                len = hi_t - lo_t + 1;
            }
        }
        const int64_t incl = wave_incl_scan64(len);
        const int64_t total = __shfl(incl, 63, 64);
        const int64_t excl = incl - len;
        for (int64_t kb = 0; kb < total; kb += 64) {   // uniform: every lane takes part in the shuffles
            const int64_t k = kb + (int64_t)lane;
            // the lane whose range holds entry k: the count of lanes ending at or before k
            int o = 0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1)
                if (__shfl(incl, o + d - 1, 64) <= k) o += d;
            o = min(o, 63);
            const int64_t tk = __shfl(t_lo, o, 64) + (k - __shfl(excl, o, 64));
            if (k < total) p.coarse[tk] = j - (int64_t)lane + o;
        }
    }
}

template <typename IDX>
__global__ void __launch_bounds__(256) k_coarse(DecodeParams p) {
    coarse_column<IDX>(p);
}

template <typename IDX>
__global__ void __launch_bounds__(256) k_coarse_batch(const DecodeParams* __restrict__ cols, int32_t n_cols) {
    for (int32_t c = (int32_t)blockIdx.y; c < n_cols; c += (int32_t)gridDim.y) coarse_column<IDX>(cols[c]);
}

// Exclusive scan of v[0, n) in place across workgroups of 1,024 entries:
// block sums (k_block_sums), a scan of those (k_scan_totals), then each
// block's local scan plus its base (k_block_scan).  bsum holds one word per
// block plus one.
constexpr int kScanBlock = 1024;
__global__ void __launch_bounds__(256) k_block_sums(const unsigned long long* v, int64_t n, unsigned long long* bsum) {
    __shared__ uint64_t s_w[kNWave];
    const unsigned tid = ltid();
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanBlock / 256; k++) {
        const int64_t i = base + tid + 256 * k;
        if (i < n) sum += v[i];
    }
    sum = wave_sum_u64(sum);
    if (lane_id() == 0) s_w[tid >> 6] = sum;
    __syncthreads();
    if (tid == 0) {
        uint64_t t = 0;
        for (int i = 0; i < 256 / 64; i++) t += s_w[i];
        bsum[blockIdx.x] = t;
        if (blockIdx.x == 0) bsum[gridDim.x] = 0;
    }
}

__global__ void __launch_bounds__(256) k_block_scan(unsigned long long* v, int64_t n, const unsigned long long* bsum) {
    __shared__ uint64_t s_w[kNWave];
    constexpr int R = kScanBlock / 256;
    const unsigned tid = ltid(), lane = lane_id(), w = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * R;   // R consecutive entries per thread
    uint64_t x[R], tsum = 0;
#pragma unroll
    for (int k = 0; k < R; k++) {
        x[k] = (base + k < n) ? v[base + k] : 0;
        tsum += x[k];
    }
    uint64_t incl = tsum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(incl, d, 64);
        if (lane >= (unsigned)d) incl += y;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    uint64_t run = bsum[blockIdx.x] + incl - tsum;
    for (unsigned k = 0; k < w; k++) run += s_w[k];
#pragma unroll
    for (int k = 0; k < R; k++) {
        if (base + k < n) v[base + k] = run;
        run += x[k];
    }
}

// --------------------------------------------------------------------------
// selective decode: the strings a row list names, compacted into one code
// stream (strings are independently decodable, so each keeps its codes
// whole), which the decode kernels then expand as a column of their own
// --------------------------------------------------------------------------
constexpr int kTakeRows = 1024;     // rows per workgroup of the compaction kernels (256 threads x 4)

// The code range of row i of the list, or an empty one (recording EOFFSETS
// when err is given) for a row outside the column or with code offsets that
// are not ordered and inside the code stream.
template <typename IDX>
__device__ __forceinline__ void take_row(const int64_t* rows, int64_t i, const IDX* code_off, int64_t n_strings,
                                         int64_t n_codes, unsigned long long* err, int64_t& a, int64_t& len) {
    a = 0;
    len = 0;
    const int64_t r = rows[i];
    if (r < 0 || r >= n_strings) {
        if (err) record_error(err, kRankOffsets, FD_EOFFSETS);
        return;
    }
    const int64_t x = (int64_t)code_off[r], y = (int64_t)code_off[r + 1];
    if (x < 0 || y < x || y > n_codes) {
        if (err) record_error(err, kRankOffsets, FD_EOFFSETS);
        return;
    }
    a = x;
    len = y - x;
}

// Pass 1: the code count of every block of kTakeRows rows (bsum[blk]), and a
// zero after the last for the scan that follows.
template <typename IDX>
__global__ void __launch_bounds__(256) k_take_sizes(const int64_t* rows, int64_t n_rows, const IDX* code_off,
                                                    int64_t n_strings, int64_t n_codes, unsigned long long* bsum,
                                                    unsigned long long* err) {
    __shared__ uint64_t s_w[kNWave];
    const unsigned tid = ltid(), w = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTakeRows;
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kTakeRows / 256; k++) {
        const int64_t i = base + tid + 256 * k;
        if (i < n_rows) {
            int64_t a, len;
            take_row(rows, i, code_off, n_strings, n_codes, err, a, len);
            sum += (uint64_t)len;
        }
    }
    sum = wave_sum_u64(sum);
    if (lane_id() == 0) s_w[w] = sum;
    __syncthreads();
    if (tid == 0) {
        bsum[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (blockIdx.x == 0) bsum[gridDim.x] = 0;
    }
}

// Pass 3 (after the exclusive scan of the block counts): each row's offset in
// the compacted stream (new_off, clamped to max_codes, recording ENOMEM past
// it) and its first code in the column (src).
template <typename IDX>
__global__ void __launch_bounds__(256) k_take_offsets(const int64_t* rows, int64_t n_rows, const IDX* code_off,
                                                      int64_t n_strings, int64_t n_codes,
                                                      const unsigned long long* bsum, int64_t max_codes,
                                                      IDX* new_off, int64_t* src, unsigned long long* err) {
    __shared__ uint64_t s_w[kNWave];
    constexpr int R = kTakeRows / 256;
    const unsigned tid = ltid(), lane = lane_id(), w = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTakeRows;
    int64_t a[R], len[R];
    uint64_t tsum = 0;
#pragma unroll
    for (int k = 0; k < R; k++) {                 // thread t holds rows base + R t .. + R - 1
        const int64_t i = base + (int64_t)R * tid + k;
        a[k] = 0;
        len[k] = 0;
        if (i < n_rows) take_row(rows, i, code_off, n_strings, n_codes, nullptr, a[k], len[k]);
        tsum += (uint64_t)len[k];
    }
    uint64_t incl = tsum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(incl, d, 64);
        if (lane >= (unsigned)d) incl += y;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    uint64_t loc = bsum[blockIdx.x] + incl - tsum;
    for (unsigned k = 0; k < w; k++) loc += s_w[k];
    const uint64_t cap = (uint64_t)max_codes;
#pragma unroll
    for (int k = 0; k < R; k++) {
        const int64_t i = base + (int64_t)R * tid + k;
        if (i < n_rows) {
            new_off[i] = (IDX)min(loc, cap);
            src[i] = a[k];
        }
        loc += (uint64_t)len[k];
    }
    if (tid == 0 && blockIdx.x == gridDim.x - 1) {
        const uint64_t total = bsum[blockIdx.x] + s_w[0] + s_w[1] + s_w[2] + s_w[3];
        new_off[n_rows] = (IDX)min(total, cap);
        if (total > cap) record_error(err, kRankOffsets, FD_ENOMEM);
    }
}

// Pass 4: copy the selected codes, widening 12-bit codes to 16 bits.  A
// workgroup copies the codes of rows_per_wg consecutive rows (chosen so that
// it holds a few thousand codes at the column's mean codes per string: a few
// chunks per thread, whose loads can be in flight together); their offsets are
// staged in LDS.  The output is cut into chunks of 16 bytes (FSST-8) or 8
// bytes (OnPair) at its own alignment (the destination is 256-byte aligned):
// each thread takes a chunk, finds the row holding the chunk's first code by a
// binary search in LDS, gathers the chunk's codes row by row into registers
// and writes them with one store.  The chunks at the two ends of a workgroup's range
// (shared with the neighbouring workgroups) are written code by code, only
// for the workgroup's own codes.
template <int CIN, typename IDX>
__global__ void __launch_bounds__(256) k_take_copy(int64_t n_rows, int rows_per_wg, const uint8_t* __restrict__ codes,
                                                   const IDX* __restrict__ new_off, const int64_t* __restrict__ src,
                                                   uint8_t* __restrict__ dst) {
    constexpr int EO = CIN == kFsst8 ? 1 : 2;      // output bytes per code
    constexpr int CB = CIN == kFsst8 ? 16 : 8;     // bytes per output chunk (short OnPair rows: more threads)
    constexpr int CH = CB / EO;                    // codes per output chunk
    __shared__ int64_t s_off[kTakeRows + 1];
    __shared__ int64_t s_src[kTakeRows];
    const unsigned tid = ltid();
    const int64_t base = (int64_t)blockIdx.x * rows_per_wg;
    const int nr = (int)min((int64_t)rows_per_wg, n_rows - base);
    for (int j = tid; j <= nr; j += 256) {
        s_off[j] = (int64_t)new_off[base + j];
        if (j < nr) s_src[j] = src[base + j];
    }
    __syncthreads();
    const int64_t o0 = s_off[0], o1 = s_off[nr];  // this workgroup's codes [o0, o1) of the output
    const int64_t c_end = (o1 + CH - 1) / CH;
#pragma unroll 4
    for (int64_t c = o0 / CH + (int64_t)tid; c < c_end; c += 256) {
        const int64_t e0 = c * CH;
        const int64_t a = max(e0, o0), b = min(e0 + CH, o1);
        int lo = 0, hi = nr - 1;                  // the last row starting at or before a
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= a) lo = mid;
            else hi = mid - 1;
        }
        // the chunk's codes row by row: slots [ka, kb) of the chunk, the row's
        // codes from slot ks on (a row change inside a chunk is the rare case)
        const int ka = (int)(a - e0), kb = (int)(b - e0);
        int j = lo;
        int kn = (int)min(s_off[j + 1] - e0, (int64_t)CH);   // first slot past row j
        int64_t sb = s_src[j] - (s_off[j] - e0);             // source index of slot 0 in row j
        uint32_t v[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if (k < ka || k >= kb) continue;
            if (k >= kn) {                        // past rows that end before slot k (empty ones included)
                do { j++; } while (s_off[j + 1] <= e0 + k);
                kn = (int)min(s_off[j + 1] - e0, (int64_t)CH);
                sb = s_src[j] - (s_off[j] - e0);
            }
            const int64_t sc = sb + k;
            uint32_t x;
            if constexpr (CIN == kFsst8) {
                x = codes[sc];
            } else if constexpr (CIN == kOnpair16) {
                x = ((const uint16_t*)codes)[sc];
            } else {                              // code sc: bits [12 sc, 12 sc + 12), least significant first
                const int64_t bo = sc + (sc >> 1);
                const uint32_t w = (uint32_t)codes[bo] | ((uint32_t)codes[bo + 1] << 8);
                x = (w >> ((sc & 1) * 4)) & 0xfffu;
            }
            v[(k * EO) >> 2] |= x << (8 * ((k * EO) & 3));
        }
        if (a == e0 && b == e0 + CH) {
            if constexpr (CB == 16) *(u32x4*)(dst + e0 * EO) = u32x4{v[0], v[1], v[2], v[3]};
            else *(uint2*)(dst + e0 * EO) = make_uint2(v[0], v[1]);
        } else {
#pragma unroll
            for (int k = 0; k < CH; k++) {
                const int64_t e = e0 + k;
                if (e < a || e >= b) continue;
                const uint32_t x = (v[(k * EO) >> 2] >> (8 * ((k * EO) & 3))) & (EO == 1 ? 0xffu : 0xffffu);
                if constexpr (EO == 1) dst[e] = (uint8_t)x;
                else ((uint16_t*)dst)[e] = (uint16_t)x;
            }
        }
    }
}

// --------------------------------------------------------------------------
// host-side launch helpers
// --------------------------------------------------------------------------
template <int CODEC, typename IDX, int MODE>
static hipError_t launch_one(const DecodeParams& p, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_decode<CODEC, IDX, MODE>), dim3(grid), dim3(kWG), 0, st, p);
    return hipGetLastError();
}

template <int CODEC, typename IDX, int MODE>
static int occupancy_of() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_decode<CODEC, IDX, MODE>, kWG, 0) != hipSuccess) nb = 1;
    return nb < 1 ? 1 : nb;
}

#define FD_FOR_ALL(X)                                                                                  \
    X(kFsst8, int32_t, kModeLookback) X(kFsst8, int64_t, kModeLookback) X(kOnpair16, int32_t, kModeLookback) \
    X(kOnpair16, int64_t, kModeLookback) X(kFsst8, int32_t, kModeTotals) X(kFsst8, int64_t, kModeTotals)     \
    X(kOnpair16, int32_t, kModeTotals) X(kOnpair16, int64_t, kModeTotals) X(kFsst8, int32_t, kModeExpand)    \
    X(kFsst8, int64_t, kModeExpand) X(kOnpair16, int32_t, kModeExpand) X(kOnpair16, int64_t, kModeExpand)    \
    X(kOnpair12, int32_t, kModeLookback) X(kOnpair12, int64_t, kModeLookback) X(kOnpair12, int32_t, kModeTotals) \
    X(kOnpair12, int64_t, kModeTotals) X(kOnpair12, int32_t, kModeExpand) X(kOnpair12, int64_t, kModeExpand) \
    X(kOnpair12s, int32_t, kModeExpand) X(kOnpair12s, int64_t, kModeExpand)

int decode_occupancy(int codec, int index_bits, int mode) {
#define OCC(C, I, M) \
    if (codec == C && index_bits == (int)(sizeof(I) * 8) && mode == M) return occupancy_of<C, I, M>();
    FD_FOR_ALL(OCC)
#undef OCC
    return 1;
}

hipError_t launch_decode(int codec, int index_bits, int mode, const DecodeParams& p, int grid, hipStream_t st) {
#define L1(C, I, M) \
    if (codec == C && index_bits == (int)(sizeof(I) * 8) && mode == M) return launch_one<C, I, M>(p, grid, st);
    FD_FOR_ALL(L1)
#undef L1
    return hipErrorInvalidValue;
}

template <int CODEC, typename IDX, int MODE>
static int batch_occupancy_of() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_decode_batch<CODEC, IDX, MODE>, kWG, 0) != hipSuccess)
        nb = 1;
    return nb < 1 ? 1 : nb;
}

#define FD_BATCH_ALL(X)                                                                                      \
    X(kFsst8, int32_t, kModeLookback) X(kFsst8, int64_t, kModeLookback) X(kOnpair16, int32_t, kModeLookback) \
    X(kOnpair16, int64_t, kModeLookback) X(kOnpair12, int32_t, kModeLookback)                                \
    X(kOnpair12, int64_t, kModeLookback) X(kFsst8, int32_t, kModeExpand) X(kFsst8, int64_t, kModeExpand)      \
    X(kOnpair16, int32_t, kModeExpand) X(kOnpair16, int64_t, kModeExpand) X(kOnpair12, int32_t, kModeExpand)  \
    X(kOnpair12, int64_t, kModeExpand)

int batch_occupancy(int codec, int index_bits, int mode) {
#define BOCC(C, I, M) \
    if (codec == C && index_bits == (int)(sizeof(I) * 8) && mode == M) return batch_occupancy_of<C, I, M>();
    FD_BATCH_ALL(BOCC)
#undef BOCC
    return 1;
}

hipError_t launch_decode_batch(int codec, int index_bits, int mode, const DecodeParams* cols, const int64_t* first_tile,
                               int32_t n_cols, int64_t total, unsigned* ctr, int grid, hipStream_t st) {
#define BL(C, I, M)                                                                                        \
    if (codec == C && index_bits == (int)(sizeof(I) * 8) && mode == M) {                                    \
        hipLaunchKernelGGL((k_decode_batch<C, I, M>), dim3(grid), dim3(kWG), 0, st, cols, first_tile, n_cols, \
                           total, ctr);                                                                     \
        return hipGetLastError();                                                                           \
    }
    FD_BATCH_ALL(BL)
#undef BL
    return hipErrorInvalidValue;
}

template <int CODEC, typename IDX>
static int totals_batch_occupancy_of() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile_totals_batch<CODEC, IDX>, kWG, 0) != hipSuccess)
        nb = 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_tile_totals_batch(int codec, int index_bits, const DecodeParams* cols, const int64_t* first_tile,
                                    int32_t n_cols, int64_t total, unsigned long long* out, int cus, hipStream_t st) {
#define TB(C, I)                                                                                             \
    if (codec == C && index_bits == (int)(sizeof(I) * 8)) {                                                   \
        static int occ = 0;                                                                                   \
        if (!occ) occ = totals_batch_occupancy_of<C, I>();                                                    \
        const int64_t g = min(total, (int64_t)cus * occ);                                                     \
        hipLaunchKernelGGL((k_tile_totals_batch<C, I>), dim3((unsigned)max(g, (int64_t)1)), dim3(kWG), 0, st,  \
                           cols, first_tile, n_cols, total, out);                                             \
        return hipGetLastError();                                                                             \
    }
    TB(kFsst8, int32_t) TB(kFsst8, int64_t) TB(kOnpair16, int32_t) TB(kOnpair16, int64_t)
    TB(kOnpair12, int32_t) TB(kOnpair12, int64_t)
#undef TB
    return hipErrorInvalidValue;
}

hipError_t launch_batch_reset(unsigned long long* z, int64_t n, unsigned long long* errs, int32_t n_cols,
                              hipStream_t st) {
    int64_t blocks = (max(n, (int64_t)n_cols) + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_batch_reset, dim3((unsigned)blocks), dim3(256), 0, st, z, n, errs, n_cols);
    return hipGetLastError();
}

hipError_t launch_batch_status(const unsigned long long* errs, int32_t n_cols, int32_t* status, int32_t* status2,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_batch_status, dim3(1), dim3(256), 0, st, errs, n_cols, status, status2);
    return hipGetLastError();
}

int chunks_per_lane(int codec) {
    return codec == kFsst8 ? Cfg<kFsst8>::P : codec == kOnpair12 ? Cfg<kOnpair12>::P : Cfg<kOnpair16>::P;
}
int codes_per_chunk(int codec) {
    return codec == kFsst8 ? Cfg<kFsst8>::CPC : codec == kOnpair12 ? Cfg<kOnpair12>::CPC : Cfg<kOnpair16>::CPC;
}

hipError_t launch_reset(unsigned long long* err, unsigned* counters, unsigned long long* z, int64_t n,
                        hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_reset, dim3((unsigned)blocks), dim3(256), 0, st, err, counters, z, n);
    return hipGetLastError();
}

hipError_t launch_scan_totals(unsigned long long* v, int64_t n, const unsigned long long* err, int32_t* status,
                              int32_t* status2, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, v, n, err, status, status2);
    return hipGetLastError();
}

// Streamed totals of one column: a wave per tile with its loads a step ahead
// and the lengths in LDS (FSST-8's table, 12-bit codes' 4,096 bytes, OnPair-16's
// nibbles), or a workgroup per tile.
template <int CODEC> constexpr bool kTotalsPerWave = true;

template <int CODEC, typename IDX>
static int totals_occupancy_of() {
    int nb = 0;
    const void* k = kTotalsPerWave<CODEC> ? (const void*)k_tile_totals<CODEC, IDX>
                                          : (const void*)k_tile_totals_wg<CODEC, IDX>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kWG, 0) != hipSuccess) nb = 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_tile_totals(int codec, int index_bits, const DecodeParams& p, int cus, hipStream_t st) {
#define TT(C, I)                                                                                              \
    if (codec == C && index_bits == (int)(sizeof(I) * 8)) {                                                    \
        static int occ = 0;                                                                                    \
        if (!occ) occ = totals_occupancy_of<C, I>();                                                           \
        const int64_t g = min(p.n_tiles, (int64_t)cus * occ);                                                  \
        if (kTotalsPerWave<C>)                                                                                 \
            hipLaunchKernelGGL((k_tile_totals<C, I>), dim3((unsigned)max(g, (int64_t)1)), dim3(kWG), 0, st, p); \
        else                                                                                                   \
            hipLaunchKernelGGL((k_tile_totals_wg<C, I>), dim3((unsigned)max(g, (int64_t)1)), dim3(kWG), 0, st, p); \
        return hipGetLastError();                                                                              \
    }
    TT(kFsst8, int32_t) TT(kFsst8, int64_t) TT(kOnpair16, int32_t) TT(kOnpair16, int64_t)
    TT(kOnpair12, int32_t) TT(kOnpair12, int64_t)
#undef TT
    return hipErrorInvalidValue;
}

hipError_t launch_coarse_one(int index_bits, const DecodeParams& p, hipStream_t st) {
    const int64_t J = (p.n_strings + ((int64_t)1 << p.g_shift) - 1) >> p.g_shift;
    const int64_t blocks = min((J + 1 + 255) / 256, (int64_t)8192);
    if (index_bits == 32)
        hipLaunchKernelGGL(k_coarse<int32_t>, dim3((unsigned)blocks), dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL(k_coarse<int64_t>, dim3((unsigned)blocks), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_coarse_batch(int index_bits, const DecodeParams* cols, int32_t n_cols, int64_t max_samples,
                               hipStream_t st) {
    if (n_cols <= 0) return hipSuccess;
    const int64_t blocks = min((max_samples + 1 + 255) / 256, (int64_t)8192);
    const unsigned gy = (unsigned)min(n_cols, 32768);
    if (index_bits == 32)
        hipLaunchKernelGGL(k_coarse_batch<int32_t>, dim3((unsigned)blocks, gy), dim3(256), 0, st, cols, n_cols);
    else
        hipLaunchKernelGGL(k_coarse_batch<int64_t>, dim3((unsigned)blocks, gy), dim3(256), 0, st, cols, n_cols);
    return hipGetLastError();
}

hipError_t launch_scan_multi(unsigned long long* v, int64_t n, unsigned long long* bsum, hipStream_t st) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb < 1 || nb > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(256), 0, st, v, n, bsum);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, bsum, nb + 1, nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_block_scan, dim3((unsigned)nb), dim3(256), 0, st, v, n, bsum);
    return hipGetLastError();
}

hipError_t launch_take_compact(int codec, int index_bits, const int64_t* rows, int64_t n_rows,
                               const void* code_off, int64_t n_strings, int64_t n_codes, const uint8_t* codes,
                               unsigned long long* bsum, int64_t max_codes, void* new_off, int64_t* src, uint8_t* dst,
                               int rows_per_wg, unsigned long long* err, hipStream_t st) {
    const int64_t nblk = n_rows > 0 ? (n_rows + kTakeRows - 1) / kTakeRows : 1;
    if (nblk > (int64_t)INT32_MAX || rows_per_wg < 1 || rows_per_wg > kTakeRows) return hipErrorInvalidValue;
    const int64_t ncopy = (n_rows + rows_per_wg - 1) / rows_per_wg;
    if (ncopy > (int64_t)INT32_MAX) return hipErrorInvalidValue;
#define TAKE(C, I)                                                                                              \
    if (codec == C && index_bits == (int)(sizeof(I) * 8)) {                                                      \
        hipLaunchKernelGGL((k_take_sizes<I>), dim3((unsigned)nblk), dim3(256), 0, st, rows, n_rows,               \
                           (const I*)code_off, n_strings, n_codes, bsum, err);                                    \
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, bsum, nblk + 1, nullptr, nullptr, nullptr);  \
        hipLaunchKernelGGL((k_take_offsets<I>), dim3((unsigned)nblk), dim3(256), 0, st, rows, n_rows,             \
                           (const I*)code_off, n_strings, n_codes, bsum, max_codes, (I*)new_off, src, err);       \
        if (n_rows > 0)                                                                                           \
            hipLaunchKernelGGL((k_take_copy<C, I>), dim3((unsigned)ncopy), dim3(256), 0, st, n_rows, rows_per_wg, \
                               codes, (const I*)new_off, src, dst);                                               \
        return hipGetLastError();                                                                                 \
    }
    TAKE(kFsst8, int32_t) TAKE(kFsst8, int64_t) TAKE(kOnpair16, int32_t) TAKE(kOnpair16, int64_t)
    TAKE(kOnpair12, int32_t) TAKE(kOnpair12, int64_t)
#undef TAKE
    return hipErrorInvalidValue;
}

hipError_t launch_onpair_prepare(const uint8_t* bytes, const uint8_t* lens, int32_t n_tok, uint4* tok16,
                                 uint8_t* tok_len, unsigned long long* err, int* bad_flag, hipStream_t st) {
    hipLaunchKernelGGL(k_onpair_prepare, dim3(256), dim3(256), 0, st, bytes, lens, n_tok, tok16, tok_len, err,
                       bad_flag);
    return hipGetLastError();
}

}  // namespace fd
