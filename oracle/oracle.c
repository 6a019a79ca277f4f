/*
 * CPU ORACLE - test infrastructure only.
 *
 * A plain, sequential, obviously-correct decoder for FSST-family string
 * columns.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the library's decode path never calls it.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * What it computes (the decode semantics of the paper's background section on
 * dictionary-compressed strings):
 *   - every fixed-width code indexes a trained dictionary of byte-string tokens;
 *     decoding looks each token up and concatenates the tokens in code order;
 *   - FSST-8 has at most 255 symbols; a byte the table cannot represent is
 *     stored right after the reserved escape code (255 here) and is emitted as
 *     a one-byte literal;
 *   - OnPair-16 (16-bit codes, tokens of up to 16 bytes) has no escapes;
 *   - the output is a byte-packed string array with fixed-width offsets
 *     (the evaluation section's description of the variable-length string
 *     array): out_off[0] = 0, out_off[i+1] - out_off[i] = decoded length of
 *     string i.
 *
 * Precedence of errors (first that applies wins):
 *   EINVAL (arguments) > EBADDICT (token length 0 or > max) > EOFFSETS
 *   (code offsets negative, decreasing or past n_codes) > data errors in stream
 *   order (EBADCODE: code >= dictionary size; EESCAPE: escape as the last code
 *   of a string) > EOVERFLOW (32-bit offsets, total > INT32_MAX) > ECAPACITY
 *   (total > out_capacity; out_off is still complete, bytes past the capacity
 *   are not written).
 *
 * Floating point: none.  All arithmetic is integer.
 */
#include <stdint.h>
#include <string.h>

enum {
    OR_OK = 0,
    OR_EINVAL = 1,
    OR_EBADCODE = 2,
    OR_EESCAPE = 3,
    OR_ECAPACITY = 4,
    OR_EOVERFLOW = 5,
    OR_EBADDICT = 6,
    OR_EOFFSETS = 7,
};

#define OR_FSST_ESCAPE 255
#define OR_FSST_MAX_SYMS 255
#define OR_FSST_MAX_LEN 8
#define OR_ONPAIR_MAX_TOKENS 65536
#define OR_ONPAIR_MAX_LEN 16

/* Checks shared by both codecs: the dictionary lengths and the code offsets. */
static int check_dict(const uint8_t *lens, int32_t n, int32_t max_len) {
    for (int32_t i = 0; i < n; i++)
        if (lens[i] == 0 || lens[i] > max_len) return OR_EBADDICT;
    return OR_OK;
}
static int check_offsets(const int64_t *code_off, int64_t n_strings, int64_t n_codes) {
    if (code_off[0] < 0) return OR_EOFFSETS;
    for (int64_t i = 0; i < n_strings; i++)
        if (code_off[i + 1] < code_off[i]) return OR_EOFFSETS;
    if (code_off[n_strings] > n_codes) return OR_EOFFSETS;
    return OR_OK;
}

/* Append `len` bytes at position *pos of the output, dropping bytes past the
 * capacity (the position still advances). */
static void emit(uint8_t *out, int64_t cap, int64_t *pos, const uint8_t *src, int64_t len) {
    for (int64_t j = 0; j < len; j++) {
        if (*pos + j < cap) out[*pos + j] = src[j];
    }
    *pos += len;
}

static int finish(int index_bits, int64_t total, int64_t out_capacity, int64_t *out_total) {
    *out_total = total;
    if (index_bits == 32 && total > INT32_MAX) return OR_EOVERFLOW;
    if (total > out_capacity) return OR_ECAPACITY;
    return OR_OK;
}

/*
 * FSST-8 decode.
 *   codes[n_codes]            uint8 code stream
 *   code_off[n_strings+1]     string i is codes[code_off[i] .. code_off[i+1])
 *   sym_bytes, sym_lens[n_sym] packed symbol bytes (sum of lens) and lengths
 *   out_off[n_strings+1]      written (int64; index_bits only selects the
 *                             overflow check)
 *   out_bytes[out_capacity]   written up to min(total, capacity)
 *   out_total                 total decoded bytes (when decoding got that far)
 *   err_pos                   code position of a data error, else -1
 */
int oracle_fsst8_decode(const uint8_t *codes, int64_t n_codes, const int64_t *code_off, int64_t n_strings,
                        const uint8_t *sym_bytes, const uint8_t *sym_lens, int32_t n_sym, int index_bits,
                        int64_t *out_off, uint8_t *out_bytes, int64_t out_capacity, int64_t *out_total,
                        int64_t *err_pos) {
    *err_pos = -1;
    *out_total = 0;
    if (n_strings < 0 || n_codes < 0 || out_capacity < 0 || n_sym < 0 || n_sym > OR_FSST_MAX_SYMS ||
        (index_bits != 32 && index_bits != 64))
        return OR_EINVAL;
    int st = check_dict(sym_lens, n_sym, OR_FSST_MAX_LEN);
    if (st) return st;
    st = check_offsets(code_off, n_strings, n_codes);
    if (st) return st;

    /* symbol start positions inside the packed byte array */
    int64_t sym_start[OR_FSST_MAX_SYMS];
    int64_t acc = 0;
    for (int32_t c = 0; c < n_sym; c++) { sym_start[c] = acc; acc += sym_lens[c]; }

    int64_t pos = 0;
    out_off[0] = 0;
    for (int64_t i = 0; i < n_strings; i++) {
        int64_t p = code_off[i], e = code_off[i + 1];
        while (p < e) {
            uint8_t c = codes[p];
            if (c == OR_FSST_ESCAPE) {
                if (p + 1 >= e) { *err_pos = p; return OR_EESCAPE; }
                emit(out_bytes, out_capacity, &pos, &codes[p + 1], 1); /* the literal byte */
                p += 2;
            } else {
                if (c >= n_sym) { *err_pos = p; return OR_EBADCODE; }
                emit(out_bytes, out_capacity, &pos, sym_bytes + sym_start[c], sym_lens[c]);
                p += 1;
            }
        }
        out_off[i + 1] = pos;
    }
    return finish(index_bits, pos, out_capacity, out_total);
}

/*
 * OnPair-16 decode: the same loop with uint16 codes and no escapes.
 */
int oracle_onpair16_decode(const uint16_t *codes, int64_t n_codes, const int64_t *code_off, int64_t n_strings,
                           const uint8_t *tok_bytes, const uint8_t *tok_lens, int32_t n_tok, int index_bits,
                           int64_t *out_off, uint8_t *out_bytes, int64_t out_capacity, int64_t *out_total,
                           int64_t *err_pos, int64_t *tok_start /* scratch: n_tok entries */) {
    *err_pos = -1;
    *out_total = 0;
    if (n_strings < 0 || n_codes < 0 || out_capacity < 0 || n_tok < 0 || n_tok > OR_ONPAIR_MAX_TOKENS ||
        (index_bits != 32 && index_bits != 64))
        return OR_EINVAL;
    int st = check_dict(tok_lens, n_tok, OR_ONPAIR_MAX_LEN);
    if (st) return st;
    st = check_offsets(code_off, n_strings, n_codes);
    if (st) return st;

    int64_t acc = 0;
    for (int32_t c = 0; c < n_tok; c++) { tok_start[c] = acc; acc += tok_lens[c]; }

    int64_t pos = 0;
    out_off[0] = 0;
    for (int64_t i = 0; i < n_strings; i++) {
        for (int64_t p = code_off[i]; p < code_off[i + 1]; p++) {
            uint16_t c = codes[p];
            if (c >= n_tok) { *err_pos = p; return OR_EBADCODE; }
            emit(out_bytes, out_capacity, &pos, tok_bytes + tok_start[c], tok_lens[c]);
        }
        out_off[i + 1] = pos;
    }
    return finish(index_bits, pos, out_capacity, out_total);
}

/*
 * Second formulation of the OnPair decode, after the CPU decoding loop the
 * paper describes for OnPair (background, CPU-based string decoding): each
 * token entry is stored at a fixed 16-byte stride, the loop always copies 16
 * bytes to the cursor and then advances the cursor by the true token length,
 * so the next copy overwrites the excess.  The output buffer needs 16 bytes of
 * slack past the total.  Valid input only (no error checks beyond the code
 * range); used to cross-check oracle_onpair16_decode.
 */
int oracle_onpair16_decode_copy16(const uint16_t *codes, const int64_t *code_off, int64_t n_strings,
                                  const uint8_t *tok_bytes, const uint8_t *tok_lens, int32_t n_tok,
                                  uint8_t *table16 /* scratch: n_tok*16 */, int64_t *out_off,
                                  uint8_t *out_bytes /* total + 16 */) {
    int64_t acc = 0;
    for (int32_t c = 0; c < n_tok; c++) {
        memset(table16 + (int64_t)c * 16, 0, 16);
        memcpy(table16 + (int64_t)c * 16, tok_bytes + acc, tok_lens[c]);
        acc += tok_lens[c];
    }
    uint8_t *cursor = out_bytes;
    out_off[0] = 0;
    for (int64_t i = 0; i < n_strings; i++) {
        for (int64_t p = code_off[i]; p < code_off[i + 1]; p++) {
            uint16_t c = codes[p];
            if (c >= n_tok) return OR_EBADCODE;
            memcpy(cursor, table16 + (int64_t)c * 16, 16);
            cursor += tok_lens[c];
        }
        out_off[i + 1] = cursor - out_bytes;
    }
    return OR_OK;
}
