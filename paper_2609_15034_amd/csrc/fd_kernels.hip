// Decode kernels for FSST-8 and OnPair-16 string columns on gfx950 (CDNA4).
//
// One workgroup (4 waves of 64 lanes) decodes one tile at a time; tiles are
// taken from a global counter in increasing order so that the decoupled
// look-back over earlier tiles always makes progress.
//
// A tile is a block of `sb` consecutive strings, so a tile always starts at a
// string boundary: the FSST-8 escape state is "expect a code" there (an escape
// never crosses a string).  Inside a tile, lane l of a pass owns the 16 code
// bytes of one 16-byte-aligned chunk of the code stream (16 FSST codes or 8
// OnPair codes).  Per pass:
//   1. load   - one 16-byte load per lane (the input stage of Algorithm 1,
//               with lane-contiguous chunks instead of a stride-32 layout);
//   2. parity - FSST-8 only: whether a lane starts on a literal follows from
//               the parity of the run of 255 bytes before it (ballots over the
//               wave, then over the waves of the workgroup);
//   3. length - decoded length of each code (token length, 0 for an escape, 1
//               for a literal) and the lane-serial prefix inside the chunk;
//   4. scan   - workgroup exclusive scan of lane totals (the WarpPrefixSum of
//               Algorithm 1 at workgroup scope);
//   5. cursor - the tile's output position: decoupled look-back over earlier
//               tiles' published totals (the on-device replacement of the
//               paper's per-batch sidecar), or a precomputed cursor;
//   6. emit   - every lane copies its tokens in order into an LDS staging
//               window placed at the destination's alignment (Algorithm 1's
//               emit stage); a lane writes whole 8/16-byte entries and lets its
//               own next token overwrite the excess (the copy-and-advance loop
//               of OnPair's CPU decoder), and writes exact lengths where the
//               excess would leave its own range;
//   7. drain  - aligned 16-byte stores of the staged window to the output,
//               byte stores only for the unaligned head / tail (Algorithm 1's
//               drain stage);
//   8. offsets - Arrow offsets of the strings that start in the pass, from the
//               per-code prefix kept in LDS.
// No floating point anywhere.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fd_internal.h"

namespace fd {

// --------------------------------------------------------------------------
// small device helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

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

// records the minimum of per-lane data-error keys of a wave (lanes without an
// error pass UINT64_MAX)
__device__ __forceinline__ void wave_record_error(unsigned long long* err, uint64_t key) {
    if (__ballot(key != ~0ull)) {
        uint64_t m = wave_min_u64(key);
        if (lane_id() == 0) atomicMin(err, (unsigned long long)m);
    }
}

__device__ __forceinline__ uint64_t data_error_key(int64_t pos, int status) {
    return ((uint64_t)(pos + kRankData) << 4) | (uint64_t)status;
}

// unaligned LDS stores (gfx950 supports unaligned DS access)
__device__ __forceinline__ void lds_put8(uint8_t* p, uint64_t v) { __builtin_memcpy(p, &v, 8); }
__device__ __forceinline__ void lds_put16(uint8_t* p, uint4 v) { __builtin_memcpy(p, &v, 16); }
__device__ __forceinline__ void lds_put4(uint8_t* p, uint32_t v) { __builtin_memcpy(p, &v, 4); }
__device__ __forceinline__ void lds_put2(uint8_t* p, uint32_t v) {
    uint16_t h = (uint16_t)v;
    __builtin_memcpy(p, &h, 2);
}

// Exact write of l (<= 8) bytes of v at p.
__device__ __forceinline__ void lds_put_exact8(uint8_t* p, uint64_t v, uint32_t l) {
    if (l == 8) {
        lds_put8(p, v);
        return;
    }
    uint32_t o = 0;
    if (l & 4) { lds_put4(p, (uint32_t)v); v >>= 32; o = 4; }
    if (l & 2) { lds_put2(p + o, (uint32_t)v); v >>= 16; o += 2; }
    if (l & 1) { p[o] = (uint8_t)v; }
}

// Exact write of l (<= 16) bytes of v at p.
__device__ __forceinline__ void lds_put_exact16(uint8_t* p, uint4 v, uint32_t l) {
    if (l == 16) {
        lds_put16(p, v);
        return;
    }
    uint64_t lo = ((uint64_t)v.y << 32) | v.x, hi = ((uint64_t)v.w << 32) | v.z;
    if (l & 8) { lds_put8(p, lo); p += 8; lo = hi; }
    lds_put_exact8(p, lo, l & 7);
}

// native 4 x u32 vector (the nontemporal builtins need a clang vector type)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// byte j (0..15) of a 16-byte value held as 4 dwords
__device__ __forceinline__ uint32_t byte_of(const uint32_t w[4], int j) { return (w[j >> 2] >> (8 * (j & 3))) & 0xffu; }

// --------------------------------------------------------------------------
// codec traits
// --------------------------------------------------------------------------
template <int CODEC> struct Codec;
template <> struct Codec<kFsst8> {
    static constexpr int CB = 1;       // bytes per code
    static constexpr int CPL = 16;     // codes per lane (one 16-byte chunk)
    static constexpr int MAXLEN = 8;
};
template <> struct Codec<kOnpair16> {
    static constexpr int CB = 2;
    static constexpr int CPL = 8;
    static constexpr int MAXLEN = 16;
};

// --------------------------------------------------------------------------
// shared memory
// --------------------------------------------------------------------------
struct Smem {
    uint8_t stage[kWin];                // staging window
    uint8_t pre8[kWG * 16];             // per code: lane-local exclusive prefix | escape bit
    uint32_t lane_pre[kWG];             // per lane: exclusive prefix inside the pass
    int64_t coff[kSbMax + 1];           // the tile's code offsets
    uint64_t fsst_tab[256];             // FSST-8 symbols, zero padded
    uint8_t fsst_len[256];              // FSST-8 symbol lengths (0 = not a symbol)
    uint32_t wtmp[kNWave];
    uint32_t wtmp2[kNWave];
    int64_t bcast[4];
    uint32_t flag;
};

// --------------------------------------------------------------------------
// workgroup helpers
// --------------------------------------------------------------------------
// exclusive scan of one uint32 per thread over the workgroup; returns the
// exclusive prefix and writes the workgroup total.  Contains two barriers.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* total, uint32_t* s_w) {
    const unsigned tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t incl = wave_incl_scan(x);
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kNWave; i++) {
        uint32_t v = s_w[i];
        base += (i < (int)w) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return base + incl - x;
}

// Load the FSST-8 table of packed symbols into LDS (once per workgroup).
// Records EBADDICT and zeroes the table when a length is 0 or above 8, in
// which case no symbol byte is read.
__device__ void fsst_build_table(Smem& s, const DecodeParams& p) {
    const unsigned tid = threadIdx.x;
    uint32_t len = 0;
    bool bad = false;
    for (unsigned c = tid; c < 256; c += kWG) {
        if ((int)c < p.n_sym) {
            len = p.dict_lens[c];
            bad = (len == 0 || len > 8);
        }
    }
    bad = __syncthreads_or(bad);
    if (bad) {
        if (tid == 0) record_error(p.err, kRankDict, FD_EBADDICT);
        for (unsigned c = tid; c < 256; c += kWG) { s.fsst_tab[c] = 0; s.fsst_len[c] = 0; }
        __syncthreads();
        return;
    }
    // kWG >= 256: one symbol per thread
    uint32_t total;
    uint32_t start = block_excl_scan(tid < 256 ? len : 0u, &total, s.wtmp);
    if (tid < 256) {
        uint64_t v = 0;
        for (uint32_t j = 0; j < len; j++) v |= (uint64_t)p.dict_bytes[start + j] << (8 * j);
        s.fsst_tab[tid] = v;
        s.fsst_len[tid] = (uint8_t)len;
    }
    __syncthreads();
}

// Read code_offsets[i] (int32 or int64).
template <typename IDX>
__device__ __forceinline__ int64_t load_off(const void* off, int64_t i) {
    return (int64_t)((const IDX*)off)[i];
}

// Load a 16-byte chunk at chunk_addr; only bytes inside [lo, hi) (addresses)
// are read, others are zero.
__device__ __forceinline__ void load_chunk(uintptr_t chunk_addr, uintptr_t lo, uintptr_t hi, uint32_t w[4]) {
    if (chunk_addr >= lo && chunk_addr + 16 <= hi) {
        u32x4 v = __builtin_nontemporal_load((const u32x4*)chunk_addr);
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else {
        w[0] = w[1] = w[2] = w[3] = 0;
        for (int j = 0; j < 16; j++) {
            uintptr_t a = chunk_addr + j;
            if (a >= lo && a < hi) w[j >> 2] |= (uint32_t)(*(const uint8_t*)a) << (8 * (j & 3));
        }
    }
}

// --------------------------------------------------------------------------
// the decode kernel
// --------------------------------------------------------------------------
// Per-pass register state of one lane.
template <int CODEC> struct Lane {
    uint32_t w[4];        // the 16 code bytes
    uint32_t valid;       // bit j: code j inside the tile's code range
    uint32_t lit_in;      // FSST-8: the lane starts on a literal
    uint32_t tot;         // decoded bytes of the lane
    uint32_t pre[Codec<CODEC>::CPL];
    uint32_t esc;         // FSST-8: bit j set when code j is an escape
    uint32_t lane_pre;    // exclusive prefix of the lane inside the pass
    uint4 tok[Codec<CODEC>::CPL == 8 ? 8 : 1];  // OnPair-16 token entries
    uint32_t tlen[Codec<CODEC>::CPL];
};

template <int CODEC, typename IDX, int MODE>
__global__ void __launch_bounds__(kWG) k_decode(DecodeParams p) {
    using C = Codec<CODEC>;
    constexpr int CPL = C::CPL;
    constexpr int CB = C::CB;
    __shared__ Smem s;
    const unsigned tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    if (CODEC == kFsst8) fsst_build_table(s, p);

    const uintptr_t codes_lo = (uintptr_t)p.codes;
    const uintptr_t codes_hi = codes_lo + (uintptr_t)p.n_codes * CB;
    const uintptr_t out_addr = (uintptr_t)p.out;

    for (;;) {
        // ---------------- acquire a tile ----------------
        if (tid == 0) s.bcast[0] = (int64_t)atomicAdd(&p.counters[0], 1u);
        __syncthreads();
        const int64_t t = s.bcast[0];
        __syncthreads();
        if (t >= p.n_tiles) break;

        const int64_t i0 = t * (int64_t)p.sb;
        const int64_t i1 = min(i0 + (int64_t)p.sb, p.n_strings);
        const int ns = (int)(i1 - i0);
        for (int j = tid; j <= ns; j += kWG) s.coff[j] = load_off<IDX>(p.code_off, i0 + j);
        __syncthreads();
        // validate the offsets of this tile
        {
            bool bad = false;
            for (int j = tid; j < ns; j += kWG) bad |= s.coff[j + 1] < s.coff[j];
            if (tid == 0) {
                if (t == 0 && s.coff[0] < 0) bad = true;
                if (i1 == p.n_strings && s.coff[ns] > p.n_codes) bad = true;
            }
            bad = __syncthreads_or(bad);
            if (bad && tid == 0) record_error(p.err, kRankOffsets, FD_EOFFSETS);
        }
        const int64_t a = min(max(s.coff[0], (int64_t)0), p.n_codes);
        const int64_t b = min(max(s.coff[ns], a), p.n_codes);
        // 16-byte-aligned chunks covering code positions [a, b)
        const uintptr_t base = (codes_lo + (uintptr_t)a * CB) & ~(uintptr_t)15;
        const int64_t nchunk = (b > a) ? (int64_t)((codes_lo + (uintptr_t)b * CB - base + 15) >> 4) : 0;
        const int npass = (int)((nchunk + kWG - 1) / kWG);
        // code position of byte 0 of chunk 0 (may be negative before the buffer)
        const int64_t pos0 = ((int64_t)base - (int64_t)codes_lo) / CB;

        // one pass: load + lengths + scan.  Returns the pass total.
        auto pass_lengths = [&](int pass, uint32_t& carry, Lane<CODEC>& L) -> uint32_t {
            const int64_t k = (int64_t)pass * kWG + tid;
            const uintptr_t caddr = base + (uintptr_t)k * 16;
            const int64_t cpos = pos0 + k * CPL;
            L.valid = 0;
            if (k < nchunk) {
                load_chunk(caddr, codes_lo, codes_hi, L.w);
#pragma unroll
                for (int j = 0; j < CPL; j++) {
                    const int64_t q = cpos + j;
                    if (q >= a && q < b) L.valid |= 1u << j;
                }
            } else {
                L.w[0] = L.w[1] = L.w[2] = L.w[3] = 0;
            }
            uint64_t errkey = ~0ull;
            L.tot = 0;
            L.esc = 0;
            if constexpr (CODEC == kFsst8) {
                // ---- escape parity: does this lane start on a literal? ----
                uint32_t ffm = 0;
#pragma unroll
                for (int j = 0; j < 16; j++) ffm |= (byte_of(L.w, j) == 0xffu ? 1u : 0u) << j;
                ffm &= L.valid;
                const bool all_ff = (ffm == 0xffffu);
                const uint32_t trail = __clz(~(ffm << 16));        // trailing run of 255 (from code 15 down)
                const uint64_t M = __ballot(!all_ff), T = __ballot(trail & 1u);
                const uint64_t m = M & ((1ull << lane) - 1ull);
                uint32_t wave_last = 0;                          // summary: bit0 has, bit1 parity
                if (M) wave_last = 1u | ((uint32_t)((T >> (63 - __clzll(M))) & 1ull) << 1);
                if (lane == 0) s.wtmp2[wv] = wave_last;
                __syncthreads();
                uint32_t c = carry;                              // parity carried into this wave
                for (int i = 0; i < (int)wv; i++) {
                    uint32_t v = s.wtmp2[i];
                    if (v & 1u) c = v >> 1;
                }
                uint32_t cin = m ? (uint32_t)((T >> (63 - __clzll(m))) & 1ull) : c;
                // carry out of the pass for the next pass
                uint32_t cout = carry;
                for (int i = 0; i < kNWave; i++) {
                    uint32_t v = s.wtmp2[i];
                    if (v & 1u) cout = v >> 1;
                }
                __syncthreads();
                carry = cout;
                L.lit_in = cin;
                // ---- lengths ----
                bool lit = cin != 0;
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    L.pre[j] = L.tot;
                    const uint32_t cj = byte_of(L.w, j);
                    if (!((L.valid >> j) & 1u)) {
                        lit = false;
                    } else if (lit) {
                        L.tot += 1;
                        lit = false;
                    } else if (cj == 255u) {
                        L.esc |= 1u << j;
                        lit = true;
                    } else {
                        const uint32_t l = s.fsst_len[cj];
                        L.tot += l;
                        if (l == 0 && errkey == ~0ull) errkey = data_error_key(cpos + j, FD_EBADCODE);
                    }
                }
            } else {
                // ---- OnPair-16: gather lengths and token entries ----
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const uint32_t cj = (L.w[j >> 1] >> (16 * (j & 1))) & 0xffffu;
                    if ((L.valid >> j) & 1u) {
                        L.tlen[j] = p.tok_len[cj];
                        L.tok[j] = p.tok16[cj];
                    } else {
                        L.tlen[j] = 0;
                    }
                }
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    L.pre[j] = L.tot;
                    L.tot += L.tlen[j];
                    if (((L.valid >> j) & 1u) && L.tlen[j] == 0 && errkey == ~0ull)
                        errkey = data_error_key(cpos + j, FD_EBADCODE);
                }
            }
            wave_record_error(p.err, errkey);
            uint32_t total;
            L.lane_pre = block_excl_scan(L.tot, &total, s.wtmp);
            return total;
        };

        int64_t cursor = 0;
        uint64_t tile_total = 0;
        Lane<CODEC> L;
        uint32_t carry = 0;
        uint32_t first_total = 0;

        auto publish_and_lookback = [&](uint64_t T) -> int64_t {
            // returns the exclusive prefix of this tile
            if constexpr (MODE == kModeLookback) {
                if (wv == 0) {
                    int64_t excl = 0;
                    if (t == 0) {
                        if (lane == 0)
                            __hip_atomic_store(&p.tstate[0], (unsigned long long)(kFlagIncl | T), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        if (lane == 0)
                            __hip_atomic_store(&p.tstate[t], (unsigned long long)(kFlagAgg | T), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        int64_t j = t - 1;
                        uint32_t spins = 0;
                        for (;;) {
                            const int64_t idx = j - (int64_t)lane;
                            uint64_t v = kFlagIncl;
                            if (idx >= 0)
                                v = __hip_atomic_load(&p.tstate[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            const uint64_t flag = v & kFlagMask;
                            const uint64_t incl = __ballot(flag == kFlagIncl);
                            const uint64_t empty = __ballot(flag == 0);
                            const int first = incl ? (int)__ffsll((unsigned long long)incl) - 1 : 63;
                            const uint64_t need = (first >= 63) ? ~0ull : ((2ull << first) - 1ull);
                            if (empty & need) {
                                // bounded wait: a predecessor that never publishes is an
                                // internal error, reported instead of hanging the device
                                if (++spins < kSpinLimit) {
                                    __builtin_amdgcn_s_sleep(1);
                                    continue;
                                }
                                if (lane == 0) record_error(p.err, kRankInternal, FD_EHIP);
                                break;
                            }
                            const uint64_t mine = ((int)lane <= first) ? (v & kValueMask) : 0ull;
                            excl += (int64_t)wave_sum_u64(mine);
                            if (incl) break;
                            j -= 64;
                        }
                        if (lane == 0)
                            __hip_atomic_store(&p.tstate[t], (unsigned long long)(kFlagIncl | (uint64_t)(excl + T)),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (lane == 0) s.bcast[1] = excl;
                }
                __syncthreads();
                int64_t r = s.bcast[1];
                __syncthreads();
                return r;
            } else if constexpr (MODE == kModeTotals) {
                if (tid == 0) p.tstate[t] = T;
                return 0;
            } else {
                return (int64_t)p.tstate[t];   // exclusive cursors precomputed
            }
        };

        if (npass <= 1) {
            if (npass == 1) first_total = pass_lengths(0, carry, L);
            tile_total = first_total;
            cursor = publish_and_lookback(tile_total);
        } else {
            uint32_t c2 = 0;
            for (int ps = 0; ps < npass; ps++) tile_total += pass_lengths(ps, c2, L);
            cursor = publish_and_lookback(tile_total);
        }

        if constexpr (MODE != kModeTotals) {
            uint64_t pass_base = 0;
            carry = 0;
            for (int ps = 0; ps < npass; ps++) {
                uint32_t ptotal = first_total;
                if (npass > 1) ptotal = pass_lengths(ps, carry, L);
                // keep per-code prefixes for the offsets of strings starting here
                {
                    uint32_t packed[CPL / 4];
#pragma unroll
                    for (int q = 0; q < CPL / 4; q++) {
                        uint32_t v = 0;
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const int j = 4 * q + r;
                            uint32_t e = L.pre[j];
                            if constexpr (CODEC == kFsst8) e |= ((L.esc >> j) & 1u) << 7;
                            v |= e << (8 * r);
                        }
                        packed[q] = v;
                    }
                    __builtin_memcpy(&s.pre8[tid * CPL], packed, CPL);
                    s.lane_pre[tid] = L.lane_pre;
                }
                // ---- emit into staging windows + drain ----
                const int64_t O = cursor + (int64_t)pass_base;       // pass output position
                const uint32_t shift = (uint32_t)((out_addr + (uintptr_t)O) & 15u);
                const int nwin = (int)((ptotal + shift + kWin - 1) / kWin);
                for (int win = 0; win < nwin; win++) {
                    const int64_t wbase = (int64_t)win * kWin;
                    int64_t q = (int64_t)shift + L.lane_pre - wbase;   // staging index of the lane's first byte
                    const int64_t qend = q + L.tot;
                    if (qend > 0 && q < kWin) {
                        const int64_t lim = qend < kWin ? qend : (int64_t)kWin;
                        if constexpr (CODEC == kFsst8) {
                            bool lit = L.lit_in != 0;
#pragma unroll
                            for (int j = 0; j < 16; j++) {
                                const uint32_t cj = byte_of(L.w, j);
                                if (!((L.valid >> j) & 1u)) {
                                    lit = false;
                                } else if (lit) {
                                    if (q >= 0 && q < kWin) s.stage[q] = (uint8_t)cj;
                                    q += 1;
                                    lit = false;
                                } else if (cj == 255u) {
                                    lit = true;
                                } else {
                                    const uint64_t v = s.fsst_tab[cj];
                                    const uint32_t l = s.fsst_len[cj];
                                    if (q >= 0 && q + 8 <= lim) {
                                        lds_put8(&s.stage[q], v);
                                    } else if (q >= 0 && q + l <= (int64_t)kWin) {
                                        lds_put_exact8(&s.stage[q], v, l);
                                    } else {
                                        for (uint32_t m = 0; m < l; m++) {
                                            const int64_t y = q + m;
                                            if (y >= 0 && y < kWin) s.stage[y] = (uint8_t)(v >> (8 * m));
                                        }
                                    }
                                    q += l;
                                }
                            }
                        } else {
#pragma unroll
                            for (int j = 0; j < 8; j++) {
                                const uint32_t l = L.tlen[j];
                                if (l) {
                                    const uint4 v = L.tok[j];
                                    if (q >= 0 && q + 16 <= lim) {
                                        lds_put16(&s.stage[q], v);
                                    } else if (q >= 0 && q + l <= (int64_t)kWin) {
                                        lds_put_exact16(&s.stage[q], v, l);
                                    } else {
                                        const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
                                        for (uint32_t m = 0; m < l; m++) {
                                            const int64_t y = q + m;
                                            if (y >= 0 && y < kWin) s.stage[y] = (uint8_t)byte_of(vv, (int)m);
                                        }
                                    }
                                    q += l;
                                }
                            }
                        }
                    }
                    __syncthreads();
                    // drain staging [s_lo, s_hi) to out[(O - shift + wbase) + s]
                    {
                        const int64_t s_lo = (win == 0) ? (int64_t)shift : 0;
                        const int64_t s_hi = min((int64_t)kWin, (int64_t)shift + (int64_t)ptotal - wbase);
                        const int64_t obase = O - (int64_t)shift + wbase;  // output position of staging index 0
                        const int64_t cap_hi = p.out_cap - obase;          // staging index limit by capacity
                        const int64_t hi_all = min(s_hi, cap_hi);
                        const int nch = (int)((s_hi + 15) >> 4);
                        for (int c = tid; c < nch; c += kWG) {
                            const int64_t lo = max((int64_t)c * 16, s_lo);
                            const int64_t hi = min((int64_t)c * 16 + 16, hi_all);
                            if (lo == (int64_t)c * 16 && hi == (int64_t)c * 16 + 16) {
                                u32x4 v;
                                __builtin_memcpy(&v, &s.stage[c * 16], 16);
                                __builtin_nontemporal_store(v, (u32x4*)(p.out + obase + c * 16));
                            } else {
                                for (int64_t y = lo; y < hi; y++) p.out[obase + y] = s.stage[y];
                            }
                        }
                    }
                    __syncthreads();
                }
                // ---- offsets of strings starting in this pass; dangling escapes ----
                {
                    const int64_t k_lo = (int64_t)ps * kWG, k_hi = k_lo + kWG;
                    for (int j = tid; j < ns; j += kWG) {
                        const int64_t st = min(max(s.coff[j], a), b);
                        if (st < b) {
                            const int64_t k = (int64_t)((codes_lo + (uintptr_t)st * CB - base) >> 4);
                            if (k >= k_lo && k < k_hi) {
                                const int li = (int)(k - k_lo);
                                const int jj = (int)(st - (pos0 + k * CPL));
                                uint32_t e = s.pre8[li * CPL + jj];
                                if constexpr (CODEC == kFsst8) e &= 0x7fu;
                                const int64_t val = O + (int64_t)s.lane_pre[li] + (int64_t)e;
                                ((IDX*)p.out_off)[i0 + j] = (IDX)val;
                            }
                        }
                        if constexpr (CODEC == kFsst8) {
                            const int64_t en = min(max(s.coff[j + 1], a), b);
                            if (en > st) {
                                const int64_t last = en - 1;
                                const int64_t k = (int64_t)((codes_lo + (uintptr_t)last * CB - base) >> 4);
                                if (k >= k_lo && k < k_hi) {
                                    const int li = (int)(k - k_lo);
                                    const int jj = (int)(last - (pos0 + k * CPL));
                                    if (s.pre8[li * CPL + jj] & 0x80u)
                                        atomicMin(p.err, (unsigned long long)data_error_key(last, FD_EESCAPE));
                                }
                            }
                        }
                    }
                }
                __syncthreads();
                pass_base += ptotal;
            }
            // strings that start at the end of the tile's code range; the final offset
            {
                const int64_t endv = cursor + (int64_t)tile_total;
                for (int j = tid; j < ns; j += kWG) {
                    const int64_t st = min(max(s.coff[j], a), b);
                    if (st >= b) ((IDX*)p.out_off)[i0 + j] = (IDX)endv;
                }
                if (tid == 0) {
                    if (i1 == p.n_strings) ((IDX*)p.out_off)[p.n_strings] = (IDX)endv;
                    if (sizeof(IDX) == 4 && endv > (int64_t)INT32_MAX) record_error(p.err, kRankOverflow, FD_EOVERFLOW);
                    if (endv > p.out_cap) record_error(p.err, kRankCapacity, FD_ECAPACITY);
                }
            }
        }
        __syncthreads();
    }

    // ---------------- completion: the last workgroup publishes the status ----------------
    if (MODE != kModeTotals) {
        __threadfence();
        if (tid == 0) {
            unsigned prev = atomicAdd(&p.counters[1], 1u);
            if (prev == gridDim.x - 1) {
                __threadfence();
                unsigned long long e = __hip_atomic_load(p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                int st = (e == ~0ull) ? FD_OK : (int)(e & 15ull);
                if (p.status) *p.status = st;
                if (p.status2) *p.status2 = st;
            }
        }
    }
}

// --------------------------------------------------------------------------
// workspace reset, cursor scan (three-phase mode), OnPair dictionary repack
// --------------------------------------------------------------------------
__global__ void k_reset(unsigned long long* err, unsigned* counters, unsigned long long* tstate, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (err) *err = ~0ull;
        counters[0] = 0;
        counters[1] = 0;
    }
    for (int64_t k = i; k < n; k += (int64_t)gridDim.x * blockDim.x) tstate[k] = 0;
}

// Single-workgroup exclusive scan of tile totals into tile cursors (in place).
__global__ void __launch_bounds__(1024) k_scan_totals(unsigned long long* tstate, int64_t n) {
    __shared__ uint64_t s_w[16];
    __shared__ uint64_t s_carry;
    const unsigned tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + tid;
        uint64_t x = i < n ? tstate[i] : 0;
        uint64_t incl = x;
        for (int d = 1; d < 64; d <<= 1) {
            uint64_t y = __shfl_up(incl, d, 64);
            if (lane >= (unsigned)d) incl += y;
        }
        if (lane == 63) s_w[w] = incl;
        __syncthreads();
        uint64_t pre = s_carry, tot = 0;
        for (int k = 0; k < 16; k++) {
            if (k < (int)w) pre += s_w[k];
            tot += s_w[k];
        }
        if (i < n) tstate[i] = pre + incl - x;
        __syncthreads();
        if (tid == 0) s_carry += tot;
        __syncthreads();
    }
}

// Repack an OnPair dictionary (packed bytes + lengths) into fixed 16-byte
// entries and a full 65,536-entry length table (0 for codes >= n_tok).
// Launched with 256 workgroups of 256 threads; workgroup g handles codes
// [256 g, 256 g + 256).  Records EBADDICT (and writes nothing else) when a
// length is 0 or above 16.
__global__ void __launch_bounds__(256) k_onpair_prepare(const uint8_t* bytes, const uint8_t* lens, int32_t n_tok,
                                                         uint4* tok16, uint8_t* tok_len, unsigned long long* err,
                                                         int* bad_flag) {
    __shared__ uint32_t s_w[4];
    __shared__ uint64_t s_red[4];
    const unsigned tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t c0 = (int32_t)blockIdx.x * 256;
    // validation of all lengths by every workgroup (64 KB read, cached)
    bool bad = false;
    uint64_t before = 0;
    for (int32_t c = tid; c < n_tok; c += 256) {
        uint32_t l = lens[c];
        bad |= (l == 0 || l > 16);
        if (c < c0) before += l;
    }
    bad = __syncthreads_or(bad);
    if (bad) {
        // every code becomes invalid (length 0); no token byte is read
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
    __syncthreads();
    const uint64_t base = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    const int32_t c = c0 + (int32_t)tid;
    const uint32_t l = (c < n_tok) ? lens[c] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan(l, &total, s_w);
    uint32_t v[4] = {0, 0, 0, 0};
    const uint8_t* src = bytes + base + ex;
    for (uint32_t j = 0; j < l; j++) v[j >> 2] |= (uint32_t)src[j] << (8 * (j & 3));
    tok16[c] = make_uint4(v[0], v[1], v[2], v[3]);
    tok_len[c] = (uint8_t)l;
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

int decode_occupancy(int codec, int index_bits, int mode) {
#define OCC(C, I, M) if (codec == C && index_bits == (sizeof(I) * 8) && mode == M) return occupancy_of<C, I, M>();
    OCC(kFsst8, int32_t, kModeLookback) OCC(kFsst8, int64_t, kModeLookback)
    OCC(kOnpair16, int32_t, kModeLookback) OCC(kOnpair16, int64_t, kModeLookback)
    OCC(kFsst8, int32_t, kModeTotals) OCC(kFsst8, int64_t, kModeTotals)
    OCC(kOnpair16, int32_t, kModeTotals) OCC(kOnpair16, int64_t, kModeTotals)
    OCC(kFsst8, int32_t, kModeExpand) OCC(kFsst8, int64_t, kModeExpand)
    OCC(kOnpair16, int32_t, kModeExpand) OCC(kOnpair16, int64_t, kModeExpand)
#undef OCC
    return 1;
}

hipError_t launch_decode(int codec, int index_bits, int mode, const DecodeParams& p, int grid, hipStream_t st) {
#define L1(C, I, M) if (codec == C && index_bits == (int)(sizeof(I) * 8) && mode == M) return launch_one<C, I, M>(p, grid, st);
    L1(kFsst8, int32_t, kModeLookback) L1(kFsst8, int64_t, kModeLookback)
    L1(kOnpair16, int32_t, kModeLookback) L1(kOnpair16, int64_t, kModeLookback)
    L1(kFsst8, int32_t, kModeTotals) L1(kFsst8, int64_t, kModeTotals)
    L1(kOnpair16, int32_t, kModeTotals) L1(kOnpair16, int64_t, kModeTotals)
    L1(kFsst8, int32_t, kModeExpand) L1(kFsst8, int64_t, kModeExpand)
    L1(kOnpair16, int32_t, kModeExpand) L1(kOnpair16, int64_t, kModeExpand)
#undef L1
    return hipErrorInvalidValue;
}

hipError_t launch_reset(unsigned long long* err, unsigned* counters, unsigned long long* tstate, int64_t n,
                        hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_reset, dim3((unsigned)blocks), dim3(256), 0, st, err, counters, tstate, n);
    return hipGetLastError();
}

hipError_t launch_scan_totals(unsigned long long* tstate, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, tstate, n);
    return hipGetLastError();
}

hipError_t launch_onpair_prepare(const uint8_t* bytes, const uint8_t* lens, int32_t n_tok, uint4* tok16,
                                 uint8_t* tok_len, unsigned long long* err, int* bad_flag, hipStream_t st) {
    hipLaunchKernelGGL(k_onpair_prepare, dim3(256), dim3(256), 0, st, bytes, lens, n_tok, tok16, tok_len, err,
                       bad_flag);
    return hipGetLastError();
}

}  // namespace fd
