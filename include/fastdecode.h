/*
 * fastdecode.h - C ABI of the MI355X (gfx950) string-column decoder.
 *
 * The library decodes string columns compressed with fixed-width-code
 * dictionary codecs into Arrow-style string arrays (offsets + bytes):
 *
 *   - FSST-8:    uint8 codes, a table of at most 255 symbols of 1..8 bytes;
 *                code 255 is the escape: the byte after it is copied as a
 *                one-byte literal (the escape mechanism of the paper's
 *                background section on dictionary-compressed strings);
 *   - OnPair-16: uint16 codes, a dictionary of at most 65,536 tokens of
 *                1..16 bytes, no escapes (same section; the paper's OnPair-16
 *                codec).
 *   - OnPair-12: 12-bit codes packed two to three bytes, a dictionary of at
 *                most 4,096 tokens of 1..16 bytes, no escapes (the 12-bit
 *                code width of the same section).  Code k is bits
 *                [12k, 12k + 12) of the byte stream, least significant bit
 *                first: codes x, y are the bytes x & 0xff,
 *                (x >> 8) | (y & 0xf) << 4, y >> 4.  The stream may start at
 *                any byte address; n_codes counts codes (the stream holds
 *                ceil(12 * n_codes / 8) bytes).  FSST-12 (4,096 symbols of
 *                1..8 bytes with every single byte present, so no escapes)
 *                decodes through this codec.  It needs a prepared dictionary
 *                (fd_dict_create, then fd_decode / fd_decode_ex / a batch);
 *                the raw-dictionary entry points fsst_decode and
 *                onpair_decode are FSST-8 and OnPair-16 only.
 *
 * Decoding looks every code's token up and concatenates the tokens in code
 * order (same section).  String i of a column is the code range
 * codes[code_offsets[i] .. code_offsets[i+1]); the output is
 * out_offsets[0] = 0, out_offsets[i+1] - out_offsets[i] = decoded length of
 * string i, and the decoded bytes of all strings back to back in out_bytes
 * (the variable-length string array of the evaluation section).
 *
 * Output positions are computed on the device by a prefix scan of decoded
 * lengths (the paper stores them per batch of codes in a "sidecar"; the
 * design section notes they can be regenerated at decode time).
 *
 * Conventions shared by every entry point:
 *   - Pointers named codes, code_offsets, dict_*, out_*, workspace and status
 *     are DEVICE pointers owned by the caller (for example torch tensors).
 *     The library never frees or retains them past the call's stream work.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  All device work
 *     of a call is enqueued on that stream.
 *   - index_bits selects the width of code_offsets AND out_offsets: 32
 *     (int32) or 64 (int64).
 *   - code_offsets must be non-decreasing with 0 <= code_offsets[0] and
 *     code_offsets[n_strings] <= n_codes; code_offsets[0] may be nonzero
 *     (a slice).  n_strings = 0 is valid (out_offsets[0] = 0 is written).
 *   - Errors the host can see (null pointers, bad widths, a workspace that is
 *     too small, sizes out of range) return at once and enqueue nothing.
 *   - Errors in the data are found on the device: FD_EBADDICT, FD_EOFFSETS,
 *     FD_EBADCODE, FD_EESCAPE, FD_EOVERFLOW, FD_ECAPACITY.  When several
 *     apply, the one reported is the first of: EBADDICT, EOFFSETS, the data
 *     error at the lowest code position, ESIDECAR (fd_decode_sidecar),
 *     EOVERFLOW, ECAPACITY.
 *     Without FD_ASYNC the call waits for the stream and returns the status.
 *     With FD_ASYNC the call returns FD_OK once enqueued and the final status
 *     is written to *status (a device int32) when the work completes.
 *   - On any error the contents of out_bytes are unspecified.  On
 *     FD_ECAPACITY out_offsets is complete (the caller may allocate
 *     out_offsets[n_strings] bytes and decode again).
 *   - The library never writes outside out_bytes[0, out_capacity) or
 *     out_offsets[0, n_strings].
 *   - Calls on different streams with different workspaces may run
 *     concurrently.  Two calls that share a workspace must be ordered.
 *   - No exception crosses this interface.
 */
#ifndef FASTDECODE_H
#define FASTDECODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fd_status {
    FD_OK = 0,
    FD_EINVAL = 1,     /* bad argument (host-side check)                          */
    FD_EBADCODE = 2,   /* a code >= the dictionary size                           */
    FD_EESCAPE = 3,    /* FSST-8: escape is the last code of a string             */
    FD_ECAPACITY = 4,  /* decoded total > out_capacity                            */
    FD_EOVERFLOW = 5,  /* index_bits = 32 and decoded total > INT32_MAX           */
    FD_EBADDICT = 6,   /* token length 0 or above the codec maximum               */
    FD_EOFFSETS = 7,   /* code_offsets decreasing, negative or past n_codes       */
    FD_EHIP = 8,       /* a HIP runtime call failed                               */
    FD_ENOMEM = 9,     /* allocation failed / request exceeds a memory budget     */
    FD_ESIDECAR = 10,  /* fd_decode_sidecar: stored positions differ from the codes */
    FD_ETIMEOUT = 11,  /* server: a wait or a queued request's deadline passed     */
    FD_ECANCELED = 12, /* server: the request was cancelled before it ran         */
    FD_EBUSY = 13      /* server: the request already runs or ran (not cancelled)  */
} fd_status;

typedef enum fd_codec { FD_FSST8 = 1, FD_ONPAIR16 = 2, FD_ONPAIR12 = 3 } fd_codec;

/* flags */
#define FD_ASYNC 1u

/* Human-readable name of a status. Never NULL. */
const char *fd_status_str(int status);

/* Library version string. */
const char *fd_version(void);

/* ------------------------------------------------------------------------- */
/* Workspace                                                                  */
/* ------------------------------------------------------------------------- */

/* Bytes of device workspace one decode of a column needs.  The workspace holds
 * the per-tile scan state of the decoded-length prefix sum (the on-device
 * replacement of the paper's per-batch sidecar, design section, design
 * overview), counters, the device error word and, for onpair_decode, the
 * prepared dictionary.  n_codes is the length of the code stream, n_strings
 * the number of strings.  Returns FD_EINVAL for negative sizes. */
fd_status fd_workspace_size(fd_codec codec, int64_t n_codes, int64_t n_strings, size_t *bytes);

/* Upper bound of the decoded size: n_codes * (8 for FSST-8, 16 for OnPair-16). */
fd_status fd_decoded_bound(fd_codec codec, int64_t n_codes, int64_t *bytes);

/* ------------------------------------------------------------------------- */
/* Single-column decode                                                       */
/* ------------------------------------------------------------------------- */

/* FSST-8 decode of one column (codec semantics: background section on
 * dictionary-compressed strings, the escape paragraph).
 *   codes[n_codes]              uint8 code stream (any alignment)
 *   code_offsets[n_strings+1]   int32 or int64 (index_bits)
 *   dict_bytes                  packed symbol bytes, sum(dict_lens) bytes
 *   dict_lens[n_symbols]        uint8 symbol lengths, each 1..8
 *   n_symbols                   0..255 (codes n_symbols..254 are FD_EBADCODE)
 *   out_offsets[n_strings+1]    written, index_bits wide
 *   out_bytes[out_capacity]     written
 *   workspace[workspace_bytes]  at least fd_workspace_size(FD_FSST8, ...)
 *   status                      device int32, required with FD_ASYNC, may be
 *                               NULL otherwise */
fd_status fsst_decode(const uint8_t *codes, int64_t n_codes, const void *code_offsets, int index_bits,
                      int64_t n_strings, const uint8_t *dict_bytes, const uint8_t *dict_lens, int32_t n_symbols,
                      void *out_offsets, uint8_t *out_bytes, int64_t out_capacity, void *workspace,
                      size_t workspace_bytes, int32_t *status, unsigned flags, void *hip_stream);

/* OnPair-16 decode of one column (same section; the paper's OnPair-16 codec).
 * Arguments as fsst_decode with uint16 codes (2-byte aligned), dict_lens each
 * 1..16 and n_tokens 0..65536.  The dictionary is repacked into fixed-stride
 * entries inside the workspace on every call (the paper does this repack
 * before timing, evaluation section); callers that decode many columns with one
 * dictionary should create an fd_dict once and use fd_decode. */
fd_status onpair_decode(const uint16_t *codes, int64_t n_codes, const void *code_offsets, int index_bits,
                        int64_t n_strings, const uint8_t *dict_bytes, const uint8_t *dict_lens, int32_t n_tokens,
                        void *out_offsets, uint8_t *out_bytes, int64_t out_capacity, void *workspace,
                        size_t workspace_bytes, int32_t *status, unsigned flags, void *hip_stream);

/* ------------------------------------------------------------------------- */
/* Device-resident dictionaries                                               */
/* ------------------------------------------------------------------------- */

/* An immutable device-resident dictionary, prepared once: for OnPair-16 the
 * tokens are repacked into fixed 16-byte entries so that a token's address
 * follows from its code (the fixed-stride dictionary of the introduction and of
 * the design section's decode stages) plus a 65,536-entry length table; an
 * OnPair-12 dictionary (at most 4,096 tokens) is repacked the same way; for
 * FSST-8 the packed symbols are copied and the decode table is built.  dict_bytes / dict_lens are device
 * pointers (read during the call only).  Validation runs on the device: the
 * call waits for hip_stream and returns FD_EBADDICT for a length of 0 or above
 * the codec maximum.  The handle owns library-allocated device memory on the
 * current device; destroy it after its last use on any stream has completed. */
typedef struct fd_dict fd_dict;

fd_status fd_dict_create(fd_codec codec, const uint8_t *dict_bytes, const uint8_t *dict_lens, int32_t n_tokens,
                         void *hip_stream, fd_dict **out);
fd_status fd_dict_destroy(fd_dict *dict);
fd_codec fd_dict_codec(const fd_dict *dict);
int32_t fd_dict_size(const fd_dict *dict);

/* Decode one column with a prepared dictionary (codec taken from the handle).
 * codes is uint8 (FSST-8), uint16 (OnPair-16) or the packed 12-bit byte
 * stream (OnPair-12, n_codes = codes in it); other arguments as
 * fsst_decode / onpair_decode.  For 12-bit codes the three-phase decode takes
 * an expand pass with a smaller staging window (faster for short tokens, as
 * FSST-12's) when out_capacity is at most 3.5 bytes per code; a larger
 * capacity gives the same result with the general 12-bit pass. */
fd_status fd_decode(const fd_dict *dict, const void *codes, int64_t n_codes, const void *code_offsets, int index_bits,
                    int64_t n_strings, void *out_offsets, uint8_t *out_bytes, int64_t out_capacity, void *workspace,
                    size_t workspace_bytes, int32_t *status, unsigned flags, void *hip_stream);

/* ------------------------------------------------------------------------- */
/* Tuning                                                                     */
/* ------------------------------------------------------------------------- */

/* Launch parameters of a decode.  A zero tile_codes or grid means
 * "automatic"; a NULL tuning makes every choice automatic.
 *   mode              0: one pass; each tile finds its output position by a
 *                        decoupled look-back over the totals published by
 *                        earlier tiles;
 *                     1: three phases (tile totals, a scan of the totals,
 *                        expansion), reading the code stream twice (the
 *                        "sidecar regenerated at decode time" variant the
 *                        paper measures in its design overview).
 *                     With a NULL tuning: mode 1 when the column has at
 *                     least four times as many tiles as workgroups resident
 *                     on the device, else mode 0 (fewer launches).
 *   tile_codes        codes per tile.  Tiles are fixed ranges of code
 *                     positions (the paper's fixed-size batches of codes,
 *                     design overview): tile t holds the codes at positions
 *                     [t * tile_codes, (t + 1) * tile_codes) of the code
 *                     buffer that lie inside the decode range, and strings
 *                     cross tiles freely.  0 = the largest, 8176 for FSST-8
 *                     and 4088 for OnPair-16 / OnPair-12 (a workgroup's pass
 *                     of 8192 / 4096 codes less one 16-byte chunk, so that a
 *                     tile of a buffer at any alignment is one pass); else a
 *                     multiple of 16 (FSST-8) or 8 (OnPair) up to that.
 *                     n_tiles = ceil(n_codes / tile_codes), at least 1.
 *   grid              workgroups to launch; automatic = all that can be
 *                     resident on the device.  Workgroups pull tiles from
 *                     counters: mode 1 splits the tiles into eight contiguous
 *                     ranges with a counter each, mode 0 takes them in order
 *                     from one.
 * The decoded result does not depend on the tuning. */
typedef struct fd_tuning {
    int32_t mode;
    int32_t tile_codes;
    int32_t grid;
    int32_t reserved;
} fd_tuning;

/* fd_workspace_size for a given tuning (NULL = automatic). */
fd_status fd_workspace_size_ex(fd_codec codec, int64_t n_codes, int64_t n_strings, const fd_tuning *tuning,
                               size_t *bytes);

/* fd_decode with explicit tuning (NULL = automatic). */
fd_status fd_decode_ex(const fd_dict *dict, const void *codes, int64_t n_codes, const void *code_offsets,
                       int index_bits, int64_t n_strings, void *out_offsets, uint8_t *out_bytes, int64_t out_capacity,
                       void *workspace, size_t workspace_bytes, int32_t *status, unsigned flags,
                       const fd_tuning *tuning, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fd_decode_ex
 * without a workspace argument.  Its scratch (tile totals, look-back states,
 * the coarse string index, counters and the error word) is a 4 MiB array the
 * library holds in device memory on each GPU it runs on, until the process
 * ends; nothing is allocated during the call.  A column needs about 16 bytes
 * per tile of it (a tile is tile_codes codes), so a column of up to about
 * 2.1 billion FSST-8 codes or 1.06 billion OnPair codes fits; a larger one
 * returns FD_EINVAL before the device is touched.  dict must be a prepared
 * dictionary; other arguments and statuses as fd_decode_ex.  Every call on one
 * GPU uses that GPU's one array: calls that overlap on a GPU (other streams,
 * other host threads) race and must be ordered by the caller. */
fd_status fd_decode_noalloc(const fd_dict *dict, const void *codes, int64_t n_codes, const void *code_offsets,
                            int index_bits, int64_t n_strings, void *out_offsets, uint8_t *out_bytes,
                            int64_t out_capacity, int32_t *status, unsigned flags, const fd_tuning *tuning,
                            void *hip_stream);

/* ------------------------------------------------------------------------- */
/* Persisted output positions (sidecar)                                       */
/* ------------------------------------------------------------------------- */

/* The paper stores, with each compressed column, the output position of every
 * fixed-size group of codes (its "sidecar", introduction and the design
 * section's paragraph on output placement), so that decoding needs no prefix
 * scan across groups; regenerating it at decode time costs 20-35% there.
 * Here a group is a tile (tile_codes consecutive code positions, see
 * fd_tuning), so the sidecar of a column under a tiling is an int64 array of
 * n_tiles + 1 entries (n_tiles = ceil(n_codes / tile_codes), at least 1):
 *     sidecar[k] = the decoded bytes of the codes at positions
 *                  [code_offsets[0], max(code_offsets[0], min(k * tile_codes,
 *                  code_offsets[n_strings]))),
 * the output position of tile k's first code (an FSST-8 escape adds no byte
 * and its literal one), and sidecar[n_tiles] the decoded total.
 * fd_sidecar_build computes it on the device from the codes.  It is 8 bytes
 * per tile (about 0.1% of the codes of the 1 GiB log column).
 *
 * fd_sidecar_layout: the tiling of a column (tuning as for fd_decode_ex; its
 * mode must be 0) and the number of sidecar entries.  The sidecar is valid
 * only with that tile_codes: store it beside the sidecar and pass it to the
 * decode in tuning->tile_codes. */
fd_status fd_sidecar_layout(fd_codec codec, int64_t n_codes, int64_t n_strings, const fd_tuning *tuning,
                            int32_t *tile_codes, int64_t *n_entries);

/* Compute the sidecar of a column on the device (a totals-only pass over the
 * codes and a scan of the tile totals), into the caller's device array
 * sidecar[n_entries] (8-byte aligned; n_entries from fd_sidecar_layout with
 * the same tuning, else FD_EINVAL).  The workspace is fd_workspace_size_ex's.
 * Statuses: FD_OK, or the errors in the data that a decode would report
 * before EOVERFLOW (EBADDICT, EOFFSETS, EBADCODE, EESCAPE), in the same
 * precedence; then the entries are unspecified.  No output is written. */
fd_status fd_sidecar_build(const fd_dict *dict, const void *codes, int64_t n_codes, const void *code_offsets,
                           int index_bits, int64_t n_strings, int64_t *sidecar, int64_t n_entries, void *workspace,
                           size_t workspace_bytes, int32_t *status, unsigned flags, const fd_tuning *tuning,
                           void *hip_stream);

/* fd_decode_ex with the output positions taken from a sidecar (device,
 * n_entries int64, read only) instead of a scan: every tile starts at once.
 * tuning->tile_codes must be the sidecar's (0 = the automatic choice,
 * as in fd_sidecar_layout) and tuning->mode 0.  Each tile checks its entry
 * against the next (sidecar[k] + tile k's decoded total = sidecar[k + 1], and
 * sidecar[0] = 0); a tile that fails writes no byte, and the call reports
 * FD_ESIDECAR, which ranks after the data errors and before EOVERFLOW and
 * ECAPACITY.  Bytes are never written outside out_bytes[0, out_capacity),
 * whatever the sidecar holds. */
fd_status fd_decode_sidecar(const fd_dict *dict, const void *codes, int64_t n_codes, const void *code_offsets,
                            int index_bits, int64_t n_strings, const int64_t *sidecar, int64_t n_entries,
                            void *out_offsets, uint8_t *out_bytes, int64_t out_capacity, void *workspace,
                            size_t workspace_bytes, int32_t *status, unsigned flags, const fd_tuning *tuning,
                            void *hip_stream);

/* ------------------------------------------------------------------------- */
/* Selective decode (take)                                                    */
/* ------------------------------------------------------------------------- */

/* Dictionary codecs keep every string independently decodable, so a query can
 * decode just the values it needs (the random access the paper's introduction
 * and related-work section give as these codecs' motivation).
 *
 * fd_decode_take decodes the strings rows[0 .. n_rows) of a column, in that
 * order, into a new Arrow string array: out_offsets[0 .. n_rows] (index_bits
 * wide, like code_offsets) and out_bytes.  rows is a DEVICE int64 array (8-byte
 * aligned); rows may repeat and come in any order.  Only the selected
 * strings' codes and code offsets are read: errors in other strings are not
 * seen.  The selected strings' codes are first compacted into the workspace
 * (12-bit codes widened to 16 bits), then decoded by the same kernels as a
 * whole column, so the result equals fd_decode_ex of the column made of the
 * selected strings.
 *   max_codes   an upper bound on the selected strings' total code count,
 *               which sizes the workspace (n_codes when no row repeats);
 *               a selection with more codes reports FD_ENOMEM.  index_bits 32
 *               needs max_codes <= INT32_MAX.
 *   tuning      as fd_decode_ex (mode 0 or 1); the automatic tile size and,
 *               with a NULL tuning, the automatic mode assume the rows have
 *               the column's mean codes per string.
 * Statuses: a row outside [0, n_strings) or a selected string whose code
 * offsets are not ordered inside [0, n_codes] is FD_EOFFSETS; then FD_ENOMEM;
 * then the decode's statuses, the data errors ranked by position in the
 * selection.  n_rows = 0 writes out_offsets[0] = 0. */
fd_status fd_take_workspace_size(fd_codec codec, int64_t n_codes, int64_t n_strings, int64_t n_rows,
                                 int64_t max_codes, const fd_tuning *tuning, size_t *bytes);

fd_status fd_decode_take(const fd_dict *dict, const void *codes, int64_t n_codes, const void *code_offsets,
                         int index_bits, int64_t n_strings, const int64_t *rows, int64_t n_rows, int64_t max_codes,
                         void *out_offsets, uint8_t *out_bytes, int64_t out_capacity, void *workspace,
                         size_t workspace_bytes, int32_t *status, unsigned flags, const fd_tuning *tuning,
                         void *hip_stream);

/* ------------------------------------------------------------------------- */
/* Batched decode                                                              */
/* ------------------------------------------------------------------------- */

/* One column of a batch: the arguments of fd_decode.  dict is a prepared
 * dictionary (its codec is the column's codec); columns may share one. */
typedef struct fd_column {
    const fd_dict *dict;
    const void *codes;
    int64_t n_codes;
    const void *code_offsets;
    int32_t index_bits;
    int64_t n_strings;
    void *out_offsets;
    uint8_t *out_bytes;
    int64_t out_capacity;
} fd_column;

#define FD_GRAPH 2u   /* batch_decode: replay a cached HIP graph of the batch */

/* Workspace bytes for batch_decode of these columns with this tuning (NULL =
 * the autotuner's largest candidate, enough for any tuning it picks). */
fd_status fd_batch_workspace_size(const fd_column *cols, int32_t n_cols, const fd_tuning *tuning, size_t *bytes);

/* Decode n_cols columns of any codecs and offset widths in one stream
 * submission: columns of one codec and offset width form a group, each group
 * runs as one persistent kernel in which every workgroup takes tiles of the
 * group's columns (numbered in column order) from the group's counters, as
 * for fd_tuning's modes (each column keeps its own error word), and a last
 * kernel collects the statuses.  The tile cursors
 * come from a look-back per column (mode 0) or from three phases per group
 * (mode 1: the group's tile totals, one scan over them, then the expand pass).
 * The byte semantics per column are those of fd_decode; out_bytes and
 * out_offsets of different columns must not overlap.
 *   cols, n_cols      host array of column descriptions (0 <= n_cols <= 65536);
 *                     the description is read during the call only.
 *   tuning            NULL: the autotuner's choice for the batch's shape
 *                     (fd_batch_autotune; found by timing the first time a
 *                     shape is seen, then cached); else mode (0 or 1) applies
 *                     to the batch and tile_codes / grid to every column /
 *                     group (0 = automatic).
 *   status            device int32[n_cols + 1] or NULL (required with
 *                     FD_ASYNC): status[c] = the status of column c,
 *                     status[n_cols] = the first non-OK status in column order.
 *   flags             FD_ASYNC as for fd_decode; FD_GRAPH records the whole
 *                     submission as a HIP graph the first time and replays
 *                     the cached graph when the same columns, workspace,
 *                     status pointer and tuning come back (the graph reads the
 *                     column table from library-owned pinned memory).
 * Returns the first non-OK status in column order (or FD_OK with FD_ASYNC).
 * Host-visible errors of any column return FD_EINVAL before anything is
 * enqueued.  Calls sharing a workspace must be ordered. */
fd_status batch_decode(const fd_column *cols, int32_t n_cols, const fd_tuning *tuning, void *workspace,
                       size_t workspace_bytes, int32_t *status, unsigned flags, void *hip_stream);

/* The autotuner behind batch_decode(tuning = NULL) (the paper's performance
 * model and launch-parameter study, Design and Microbenchmarks).  Candidates:
 * mode 0 / 1, tiles of 100, 50 and 25% of the largest, and all or three
 * quarters of the workgroups that fit on the device.  A residency model
 * prunes them first: with R = the workgroups resident at once (set by the
 * kernel's registers and LDS), a smaller tile size is tried only while the
 * larger one leaves some codec group with fewer than 2 R tiles, and fewer
 * workgroups only for mode 0 on groups of at least 2 R tiles.  The rest are
 * timed on the batch (a warm-up and two timed runs each) and the fastest is
 * kept per batch shape (per column: codec, offset width, log2 of its strings
 * and codes) and device type.  With the environment variable
 * FD_AUTOTUNE_CACHE naming a file, choices are appended to it and read back
 * by later processes.
 *
 * fd_batch_autotune returns the choice for a batch (timing it if its shape is
 * new, which decodes the batch into its outputs several times; the workspace
 * is that of fd_batch_workspace_size(tuning = NULL)) and waits for the
 * stream.  source: 0 timed now, 1 cached in this process, 2 read from the
 * file.  fd_debug_autotune_forget clears the process's cache (the file is
 * read again on the next lookup). */
typedef struct fd_batch_choice {
    int32_t mode;                 /* 0 or 1 */
    int32_t tile_scale_pct;       /* tile size, % of the codec's largest */
    int32_t grid_pct;             /* % of the resident workgroups launched */
    int32_t source;
    int32_t candidates_timed;     /* 0 unless timed now */
} fd_batch_choice;

fd_status fd_batch_autotune(const fd_column *cols, int32_t n_cols, void *workspace, size_t workspace_bytes,
                            void *hip_stream, fd_batch_choice *out);
fd_status fd_debug_autotune_forget(void);

/* The FD_GRAPH cache keeps at most 16 graphs, least recently used first out.
 * A cached graph is replayed only for a batch equal to the recorded one in
 * every column's dictionary (compared by a per-handle id, not its address),
 * codec, buffers and sizes, and in workspace, status pointer and tuning;
 * fd_dict_destroy drops (after waiting for the device) every cached graph
 * that reads the destroyed dictionary.
 * Testing hooks: fd_debug_graph_hash_bits keeps only that many bits (0..64)
 * of the cache's hash, so that different batches collide and only the full
 * comparison tells them apart; fd_debug_graph_count is the number of cached
 * graphs. */
fd_status fd_debug_graph_hash_bits(int32_t bits);
int32_t fd_debug_graph_count(void);

/* ------------------------------------------------------------------------- */
/* Kernel timing                                                               */
/* ------------------------------------------------------------------------- */

/* The kernels one decode enqueues, by role (the hot path's stages of the
 * paper's Design section, Decode Stages, as launched here). */
typedef enum fd_prof_kind {
    FD_PROF_RESET = 0,     /* k_reset: workspace words, tile words, status */
    FD_PROF_COARSE = 1,    /* k_coarse: the coarse string index per tile of codes */
    FD_PROF_TOTALS = 2,    /* tile totals (three phases; sidecar build) */
    FD_PROF_SCAN = 3,      /* the scan of tile totals into tile cursors */
    FD_PROF_DECODE = 4,    /* k_decode: expand, single pass, or sidecar decode */
    FD_PROF_PREPARE = 5,   /* one-shot dictionary repack; fd_decode_take's row compaction */
    FD_PROF_KINDS = 6
} fd_prof_kind;

/* fd_profile_begin opens a profile on the current device: from then on, every
 * launch of a kind in kind_mask (bit 1 << fd_prof_kind) made by fsst_decode,
 * onpair_decode, fd_decode(_ex), fd_sidecar_build, fd_decode_sidecar or
 * fd_decode_take on that device is bracketed by two HIP events recorded on
 * the launch's own stream.  The events, 2 * max_launches of them
 * (1..1,048,576), are created here, so the timed calls allocate nothing;
 * launches past the pool are counted as dropped.  batch_decode and the server
 * are not timed.  FD_EINVAL for an empty or unknown mask, a bad size or a
 * profile already open; FD_EHIP if the events cannot be created.
 *
 * fd_profile_end waits for the recorded events and writes, for each of the
 * FD_PROF_KINDS kinds (arrays of that length, each may be NULL), the summed
 * duration in ms, the number of launches timed, and the shortest and longest
 * launch; *dropped (may be NULL) gets the launches not timed.  It closes the
 * profile and frees the events.  FD_EINVAL if no profile is open.
 * Not for use while a stream capture records the calls. */
fd_status fd_profile_begin(uint32_t kind_mask, int32_t max_launches);
fd_status fd_profile_end(double *total_ms, int64_t *launches, double *min_ms, double *max_ms, int64_t *dropped);

/* ------------------------------------------------------------------------- */
/* Served decode (continuous batching)                                         */
/* ------------------------------------------------------------------------- */

/* A decode server on the current device.  Requests are single columns
 * (fd_column: prepared dictionaries, caller-owned device buffers that must stay
 * valid until the request completes).  A scheduler thread owns n_slots streams;
 * whenever a slot is free it admits waiting requests in arrival order while the
 * device bytes they hold (codes, code and Arrow offsets, output capacity,
 * workspace) stay within max_inflight_bytes, up to max_batch per batch, and runs
 * them as one asynchronous batch_decode (three phases, mode 1) on the slot's
 * stream.  Requests that
 * arrive while batches run are admitted as slots and budget free up, so their
 * work overlaps on the device.  Each request's bytes and offsets are those of
 * fd_decode on the same column. */
typedef struct fd_server fd_server;

typedef struct fd_server_config {
    int64_t max_inflight_bytes;   /* HBM budget of admitted requests; 0 = 16 GiB */
    int32_t n_slots;              /* batches on the device at once (1..64); 0 = 4 */
    int32_t max_batch;            /* requests per batch (1..65536); 0 = 64 */
    int64_t queue_timeout_us;     /* a request still waiting for admission this long
                                     after its submission completes with FD_ETIMEOUT
                                     without running; 0 = no deadline */
} fd_server_config;

typedef struct fd_server_stats {
    int64_t submitted, admitted, completed, batches, queued;
    int64_t inflight_bytes, max_inflight_bytes;
    int64_t canceled, timed_out;  /* completed without running */
} fd_server_stats;

/* cfg may be NULL (all defaults).  The server owns its streams, events,
 * status buffers and per-slot workspaces (grown on demand with hipMalloc). */
fd_status fd_server_create(const fd_server_config *cfg, fd_server **out);
/* Queue one request; *ticket identifies it.  Host-visible errors of the column
 * return FD_EINVAL and queue nothing.  Never blocks on the device. */
fd_status fd_server_submit(fd_server *server, const fd_column *request, uint64_t *ticket);
/* Wait for a request: its fd_status and its latency (microseconds from
 * submission to the host seeing its batch complete).  Each ticket is waited
 * for once. */
fd_status fd_server_wait(fd_server *server, uint64_t ticket, int32_t *status, double *latency_us);
/* fd_server_wait with a time limit: FD_ETIMEOUT if the request has not
 * completed within timeout_us microseconds (the ticket stays valid, to be
 * waited for again); a negative timeout waits without limit.  FD_EINVAL for
 * an unknown or already waited ticket. */
fd_status fd_server_wait_for(fd_server *server, uint64_t ticket, int64_t timeout_us, int32_t *status,
                             double *latency_us);
/* Cancel a request that is still waiting for admission: FD_OK, and the
 * request completes with status FD_ECANCELED (its outputs untouched; wait for
 * its ticket as usual).  FD_EBUSY if it was already admitted or has
 * completed (it then completes normally), FD_EINVAL for an unknown or already
 * waited ticket. */
fd_status fd_server_cancel(fd_server *server, uint64_t ticket);
fd_status fd_server_get_stats(fd_server *server, fd_server_stats *out);
/* Completes every queued request, then frees the server. */
fd_status fd_server_destroy(fd_server *server);

#ifdef __cplusplus
}
#endif

#endif /* FASTDECODE_H */
