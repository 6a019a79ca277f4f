/*
 * Seeded synthetic string columns, dictionary builders and greedy encoders.
 *
 * This file produces the inputs that both the CPU oracle and the GPU decoder
 * consume.  It contains no decoding: it only generates text, trains
 * dictionaries and encodes text into code streams (the inverse direction of
 * the method).  Everything is deterministic for a given seed and independent
 * of the number of threads used.
 *
 * Dictionary recipes follow the two training families described in the
 * paper's background section on dictionary-compressed strings:
 *   - FSST-style: a small table (<= 255 symbols of 1..8 bytes, code 255 is the
 *     escape) chosen from a sample by byte coverage (count x length);
 *   - OnPair-style: start from the 256 single-byte tokens and, while scanning a
 *     sample with greedy longest match, append the concatenation of an adjacent
 *     token pair once that pair has been seen `tau` times (<= 16 bytes).
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* RNG: splitmix64 seeding + xoshiro256** streams                             */
/* ------------------------------------------------------------------------- */
typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static void rng_seed(rng_t *r, uint64_t seed, uint64_t stream) {
    uint64_t x = seed * 0x2545F4914F6CDD1DULL + stream * 0x9E3779B97F4A7C15ULL + 0x1234567ULL;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}
static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl64(s[3], 45);
    return result;
}
static inline uint32_t rng_below(rng_t *r, uint32_t n) {
    return (uint32_t)(((rng_next(r) >> 32) * (uint64_t)n) >> 32);
}
static inline double rng_unit(rng_t *r) { return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }
static double rng_normal(rng_t *r) {
    double u1 = rng_unit(r), u2 = rng_unit(r);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
static int lognormal_len(rng_t *r, double median, double sigma, int lo, int hi) {
    double v = exp(log(median) + sigma * rng_normal(r));
    long l = lround(v);
    if (l < lo) l = lo;
    if (l > hi) l = hi;
    return (int)l;
}

/* ------------------------------------------------------------------------- */
/* Column container                                                           */
/* ------------------------------------------------------------------------- */
typedef struct dg_column {
    uint8_t *bytes;
    int64_t *offsets; /* n_strings + 1 */
    int64_t n_strings;
    int64_t n_bytes;
} dg_column;

void dg_column_free(dg_column *c) {
    if (!c) return;
    free(c->bytes);
    free(c->offsets);
    free(c);
}

/* growable per-chunk buffer */
typedef struct {
    uint8_t *b; int64_t nb, cb;
    int64_t *o; int64_t no, co; /* string end offsets (exclusive), relative to chunk */
} chunkbuf;

static void cb_reserve(chunkbuf *c, int64_t extra) {
    if (c->nb + extra > c->cb) {
        int64_t nc = c->cb ? c->cb * 2 : (1 << 20);
        while (nc < c->nb + extra) nc *= 2;
        c->b = (uint8_t *)realloc(c->b, (size_t)nc);
        c->cb = nc;
    }
}
static void cb_push_end(chunkbuf *c) {
    if (c->no == c->co) {
        c->co = c->co ? c->co * 2 : 4096;
        c->o = (int64_t *)realloc(c->o, (size_t)c->co * sizeof(int64_t));
    }
    c->o[c->no++] = c->nb;
}

/* concatenate chunk buffers into one column */
static dg_column *concat_chunks(chunkbuf *cs, int nchunk) {
    dg_column *col = (dg_column *)calloc(1, sizeof(dg_column));
    int64_t nb = 0, ns = 0;
    for (int k = 0; k < nchunk; k++) { nb += cs[k].nb; ns += cs[k].no; }
    col->bytes = (uint8_t *)malloc((size_t)(nb ? nb : 1));
    col->offsets = (int64_t *)malloc((size_t)(ns + 1) * sizeof(int64_t));
    int64_t pb = 0, ps = 0;
    col->offsets[0] = 0;
    for (int k = 0; k < nchunk; k++) {
        if (cs[k].nb) memcpy(col->bytes + pb, cs[k].b, (size_t)cs[k].nb);
        for (int64_t i = 0; i < cs[k].no; i++) col->offsets[ps + 1 + i] = pb + cs[k].o[i];
        pb += cs[k].nb; ps += cs[k].no;
        free(cs[k].b); free(cs[k].o);
    }
    col->n_bytes = nb;
    col->n_strings = ns;
    return col;
}

/* simple parallel-for over chunk indices */
typedef void (*chunk_fn)(void *ctx, int k);
typedef struct { chunk_fn fn; void *ctx; int n; int next; pthread_mutex_t mu; } pool_t;
static void *pool_worker(void *arg) {
    pool_t *p = (pool_t *)arg;
    for (;;) {
        pthread_mutex_lock(&p->mu);
        int k = p->next++;
        pthread_mutex_unlock(&p->mu);
        if (k >= p->n) break;
        p->fn(p->ctx, k);
    }
    return NULL;
}
static void parallel_for(int n, int n_threads, chunk_fn fn, void *ctx) {
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 64) n_threads = 64;
    if (n_threads > n) n_threads = n;
    pool_t p = {fn, ctx, n, 0, PTHREAD_MUTEX_INITIALIZER};
    if (n_threads <= 1) { pool_worker(&p); return; }
    pthread_t th[64];
    for (int i = 0; i < n_threads; i++) pthread_create(&th[i], NULL, pool_worker, &p);
    for (int i = 0; i < n_threads; i++) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------------- */
/* Vocabulary + Zipf sampling                                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n;
    char **w;
    int *len;
    double *cdf;
} vocab_t;

static void vocab_make(vocab_t *v, uint64_t seed, int n, int minl, int maxl, double zipf_s) {
    rng_t r;
    rng_seed(&r, seed, 77);
    v->n = n;
    v->w = (char **)malloc(sizeof(char *) * n);
    v->len = (int *)malloc(sizeof(int) * n);
    v->cdf = (double *)malloc(sizeof(double) * n);
    double tot = 0;
    for (int i = 0; i < n; i++) {
        int l = minl + (int)rng_below(&r, (uint32_t)(maxl - minl + 1));
        v->w[i] = (char *)malloc((size_t)l + 1);
        for (int j = 0; j < l; j++) v->w[i][j] = (char)('a' + rng_below(&r, 26));
        v->w[i][l] = 0;
        v->len[i] = l;
        tot += 1.0 / pow((double)(i + 1), zipf_s);
        v->cdf[i] = tot;
    }
    for (int i = 0; i < n; i++) v->cdf[i] /= tot;
    v->cdf[n - 1] = 1.0;
}
static void vocab_free(vocab_t *v) {
    for (int i = 0; i < v->n; i++) free(v->w[i]);
    free(v->w); free(v->len); free(v->cdf);
}
static int vocab_zipf(const vocab_t *v, rng_t *r) {
    double u = rng_unit(r);
    int lo = 0, hi = v->n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (v->cdf[mid] >= u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static inline void put_str(uint8_t **p, const char *s, int l) { memcpy(*p, s, (size_t)l); *p += l; }
static inline void put_dec(uint8_t **p, uint64_t v, int width) {
    char tmp[24];
    for (int i = width - 1; i >= 0; i--) { tmp[i] = (char)('0' + v % 10); v /= 10; }
    put_str(p, tmp, width);
}
static const char HEX[] = "0123456789abcdef";
static inline void put_hex(uint8_t **p, rng_t *r, int n) {
    for (int i = 0; i < n; i++) *(*p)++ = (uint8_t)HEX[rng_below(r, 16)];
}

/* ------------------------------------------------------------------------- */
/* Config "small": printable ASCII strings, length uniform [min,max]          */
/* ------------------------------------------------------------------------- */
dg_column *dg_gen_printable(uint64_t seed, int64_t n_strings, int min_len, int max_len) {
    rng_t r;
    rng_seed(&r, seed, 1);
    chunkbuf c = {0};
    for (int64_t i = 0; i < n_strings; i++) {
        int l = min_len + (int)rng_below(&r, (uint32_t)(max_len - min_len + 1));
        cb_reserve(&c, l);
        for (int j = 0; j < l; j++) c.b[c.nb + j] = (uint8_t)(0x20 + rng_below(&r, 95));
        c.nb += l;
        cb_push_end(&c);
    }
    return concat_chunks(&c, 1);
}

/* ------------------------------------------------------------------------- */
/* Config "logs": templated log lines                                         */
/*   "YYYY-MM-DD HH:MM:SS.mmm LEVEL <16 hex> word word ..." truncated to a    */
/*   log-normal target length (median 120, sigma 0.5, clamped [32, 2048]).    */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint64_t seed;
    uint64_t stream_base;
    int64_t chunk_target;
    int nchunk;
    const vocab_t *voc;
    chunkbuf *cs;
    int64_t t0_ms;
} logs_ctx;

static void civil_from_days(int64_t z, int *y, int *m, int *d) {
    z += 719468;
    int64_t era = (z >= 0 ? z : z - 146096) / 146097;
    int64_t doe = z - era * 146097;
    int64_t yoe = (doe - doe / 1460 + doe / 36524 - doe / 146096) / 365;
    int64_t yy = yoe + era * 400;
    int64_t doy = doe - (365 * yoe + yoe / 4 - yoe / 100);
    int64_t mp = (5 * doy + 2) / 153;
    int64_t dd = doy - (153 * mp + 2) / 5 + 1;
    int64_t mm = mp < 10 ? mp + 3 : mp - 9;
    *y = (int)(yy + (mm <= 2));
    *m = (int)mm;
    *d = (int)dd;
}

static void logs_chunk(void *vctx, int k) {
    logs_ctx *ctx = (logs_ctx *)vctx;
    rng_t r;
    uint64_t stream = ctx->stream_base + (uint64_t)k;
    rng_seed(&r, ctx->seed, 1000 + stream);
    chunkbuf *c = &ctx->cs[k];
    /* each chunk covers its own time window so timestamps stay monotone */
    int64_t t_ms = ctx->t0_ms + (int64_t)stream * 3600000LL;
    static const char *LV[4] = {"INFO", "DEBUG", "WARN", "ERROR"};
    static const int LVL[4] = {4, 5, 4, 5};
    uint8_t line[4096];
    while (c->nb < ctx->chunk_target) {
        int target = lognormal_len(&r, 120.0, 0.5, 32, 2048);
        uint8_t *p = line;
        t_ms += rng_below(&r, 50);
        int64_t days = t_ms / 86400000LL, rem = t_ms % 86400000LL;
        int y, mo, d;
        civil_from_days(days, &y, &mo, &d);
        put_dec(&p, (uint64_t)y, 4); *p++ = '-';
        put_dec(&p, (uint64_t)mo, 2); *p++ = '-';
        put_dec(&p, (uint64_t)d, 2); *p++ = ' ';
        put_dec(&p, (uint64_t)(rem / 3600000), 2); *p++ = ':';
        put_dec(&p, (uint64_t)(rem / 60000 % 60), 2); *p++ = ':';
        put_dec(&p, (uint64_t)(rem / 1000 % 60), 2); *p++ = '.';
        put_dec(&p, (uint64_t)(rem % 1000), 3); *p++ = ' ';
        uint32_t u = rng_below(&r, 100);
        int lv = u < 70 ? 0 : u < 85 ? 1 : u < 95 ? 2 : 3;
        put_str(&p, LV[lv], LVL[lv]); *p++ = ' ';
        put_hex(&p, &r, 16);
        while (p - line < target) {
            int w = vocab_zipf(ctx->voc, &r);
            *p++ = ' ';
            put_str(&p, ctx->voc->w[w], ctx->voc->len[w]);
        }
        int l = target;
        cb_reserve(c, l);
        memcpy(c->b + c->nb, line, (size_t)l);
        c->nb += l;
        cb_push_end(c);
    }
}

dg_column *dg_gen_logs(uint64_t seed, uint64_t stream_base, int64_t target_bytes, int nchunk, int n_threads) {
    vocab_t voc;
    vocab_make(&voc, seed, 2000, 2, 12, 1.1);
    rng_t r;
    rng_seed(&r, seed, 2);
    logs_ctx ctx;
    ctx.seed = seed;
    ctx.stream_base = stream_base;
    ctx.nchunk = nchunk;
    ctx.chunk_target = (target_bytes + nchunk - 1) / nchunk;
    ctx.voc = &voc;
    ctx.cs = (chunkbuf *)calloc((size_t)nchunk, sizeof(chunkbuf));
    /* seeded base date between 2020-01-01 and ~2027 */
    ctx.t0_ms = (18262LL + rng_below(&r, 2500)) * 86400000LL + rng_below(&r, 86400000);
    parallel_for(nchunk, n_threads, logs_chunk, &ctx);
    dg_column *col = concat_chunks(ctx.cs, nchunk);
    free(ctx.cs);
    vocab_free(&voc);
    return col;
}

/* ------------------------------------------------------------------------- */
/* Config "urls": URL-like (70%) and identifier-like (30%) strings            */
/*   length log-normal (median 30, sigma 0.5, clamped [4, 512]), built then   */
/*   truncated.                                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint64_t seed;
    uint64_t stream_base;
    int64_t chunk_target;
    const vocab_t *words, *hosts, *keys;
    chunkbuf *cs;
} urls_ctx;

static const char *TLD[] = {".com", ".org", ".net", ".io", ".de", ".co.uk", ".fr", ".jp", ".ru", ".edu"};
static const int TLDW[] = {40, 12, 10, 8, 6, 6, 5, 5, 4, 4}; /* weights, sum 100 */

static void urls_chunk(void *vctx, int k) {
    urls_ctx *ctx = (urls_ctx *)vctx;
    rng_t r;
    rng_seed(&r, ctx->seed, 2000 + ctx->stream_base + (uint64_t)k);
    chunkbuf *c = &ctx->cs[k];
    uint8_t buf[2048];
    while (c->nb < ctx->chunk_target) {
        int target = lognormal_len(&r, 30.0, 0.5, 4, 512);
        uint8_t *p = buf;
        if (rng_below(&r, 100) < 70) {
            if (rng_below(&r, 100) < 80) put_str(&p, "https://", 8); else put_str(&p, "http://", 7);
            if (rng_below(&r, 2)) put_str(&p, "www.", 4);
            int h = vocab_zipf(ctx->hosts, &r);
            put_str(&p, ctx->hosts->w[h], ctx->hosts->len[h]);
            if (rng_below(&r, 100) < 20) {
                int h2 = vocab_zipf(ctx->hosts, &r);
                *p++ = '-';
                put_str(&p, ctx->hosts->w[h2], ctx->hosts->len[h2]);
            }
            uint32_t u = rng_below(&r, 100), acc = 0;
            int t = 0;
            for (; t < 9; t++) { acc += (uint32_t)TLDW[t]; if (u < acc) break; }
            put_str(&p, TLD[t], (int)strlen(TLD[t]));
            int segs = 1 + (int)rng_below(&r, 4);
            for (int s = 0; s < segs; s++) {
                int w = vocab_zipf(ctx->words, &r);
                *p++ = '/';
                put_str(&p, ctx->words->w[w], ctx->words->len[w]);
                if (rng_below(&r, 100) < 30) {
                    int w2 = vocab_zipf(ctx->words, &r);
                    *p++ = '-';
                    put_str(&p, ctx->words->w[w2], ctx->words->len[w2]);
                }
                if (rng_below(&r, 100) < 20) { *p++ = '/'; put_dec(&p, rng_below(&r, 1000000), 1 + (int)rng_below(&r, 6)); }
            }
            if (rng_below(&r, 100) < 30) {
                int kk = vocab_zipf(ctx->keys, &r);
                *p++ = '?';
                put_str(&p, ctx->keys->w[kk], ctx->keys->len[kk]);
                *p++ = '=';
                put_dec(&p, rng_below(&r, 100000000), 1 + (int)rng_below(&r, 8));
            }
            while (p - buf < target) {
                if (rng_below(&r, 2)) {
                    int w = vocab_zipf(ctx->words, &r);
                    *p++ = '/';
                    put_str(&p, ctx->words->w[w], ctx->words->len[w]);
                } else {
                    int kk = vocab_zipf(ctx->keys, &r);
                    *p++ = '&';
                    put_str(&p, ctx->keys->w[kk], ctx->keys->len[kk]);
                    *p++ = '=';
                    put_dec(&p, rng_below(&r, 100000), 1 + (int)rng_below(&r, 5));
                }
            }
        } else {
            uint32_t kind = rng_below(&r, 100);
            if (kind < 40) {
                int w = vocab_zipf(ctx->words, &r);
                put_str(&p, ctx->words->w[w], ctx->words->len[w]);
                *p++ = '_';
                put_hex(&p, &r, 8 + (int)rng_below(&r, 9));
            } else if (kind < 70) {
                int w = vocab_zipf(ctx->words, &r);
                put_str(&p, ctx->words->w[w], ctx->words->len[w]);
                *p++ = '-';
                put_dec(&p, rng_next(&r) % 10000000000ULL, 4 + (int)rng_below(&r, 7));
            } else {
                put_hex(&p, &r, 8); *p++ = '-';
                put_hex(&p, &r, 4); *p++ = '-';
                put_hex(&p, &r, 4); *p++ = '-';
                put_hex(&p, &r, 4); *p++ = '-';
                put_hex(&p, &r, 12);
            }
            while (p - buf < target) {
                int w = vocab_zipf(ctx->words, &r);
                *p++ = '_';
                put_str(&p, ctx->words->w[w], ctx->words->len[w]);
            }
        }
        int l = target;
        cb_reserve(c, l);
        memcpy(c->b + c->nb, buf, (size_t)l);
        c->nb += l;
        cb_push_end(c);
    }
}

dg_column *dg_gen_urls(uint64_t seed, uint64_t stream_base, int64_t target_bytes, int nchunk, int n_threads) {
    vocab_t words, hosts, keys;
    vocab_make(&words, seed * 3 + 1, 2000, 2, 12, 1.1);
    vocab_make(&hosts, seed * 3 + 2, 500, 3, 10, 1.2);
    vocab_make(&keys, seed * 3 + 3, 40, 1, 8, 1.3);
    urls_ctx ctx;
    ctx.seed = seed;
    ctx.stream_base = stream_base;
    ctx.chunk_target = (target_bytes + nchunk - 1) / nchunk;
    ctx.words = &words; ctx.hosts = &hosts; ctx.keys = &keys;
    ctx.cs = (chunkbuf *)calloc((size_t)nchunk, sizeof(chunkbuf));
    parallel_for(nchunk, n_threads, urls_chunk, &ctx);
    dg_column *col = concat_chunks(ctx.cs, nchunk);
    free(ctx.cs);
    vocab_free(&words); vocab_free(&hosts); vocab_free(&keys);
    return col;
}

/* ------------------------------------------------------------------------- */
/* FSST-style tables                                                          */
/* ------------------------------------------------------------------------- */

/* Random table for the small printable config: the 95 printable bytes minus
 * `n_excluded` chosen by seed as single-byte symbols, then random multi-byte
 * printable symbols (length uniform [2, 8]) up to n_sym, deduplicated; the code
 * order is shuffled.  Returns n_sym.  out_bytes is packed (sum of lens). */
int dg_fsst_random_table(uint64_t seed, int n_sym, int n_excluded, uint8_t *out_bytes, uint8_t *out_lens) {
    rng_t r;
    rng_seed(&r, seed, 3);
    uint8_t sym[255][8];
    uint8_t len[255];
    int n = 0;
    uint8_t excl[95] = {0};
    for (int e = 0; e < n_excluded;) {
        int b = (int)rng_below(&r, 95);
        if (!excl[b]) { excl[b] = 1; e++; }
    }
    for (int b = 0; b < 95 && n < n_sym; b++)
        if (!excl[b]) { sym[n][0] = (uint8_t)(0x20 + b); len[n] = 1; n++; }
    while (n < n_sym) {
        int l = 2 + (int)rng_below(&r, 7);
        uint8_t s[8];
        for (int j = 0; j < l; j++) s[j] = (uint8_t)(0x20 + rng_below(&r, 95));
        int dup = 0;
        for (int i = 0; i < n && !dup; i++) dup = (len[i] == l && memcmp(sym[i], s, (size_t)l) == 0);
        if (dup) continue;
        memcpy(sym[n], s, (size_t)l);
        len[n] = (uint8_t)l;
        n++;
    }
    int perm[255];
    for (int i = 0; i < n; i++) perm[i] = i;
    for (int i = n - 1; i > 0; i--) {
        int j = (int)rng_below(&r, (uint32_t)(i + 1));
        int t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    int64_t pos = 0;
    for (int i = 0; i < n; i++) {
        memcpy(out_bytes + pos, sym[perm[i]], len[perm[i]]);
        out_lens[i] = len[perm[i]];
        pos += len[perm[i]];
    }
    return n;
}

/* n-gram counting hash table */
typedef struct { uint64_t key; uint32_t cnt; uint8_t len; } ng_ent;

static inline uint64_t mix64(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}

typedef struct { uint64_t key; uint32_t cnt; uint8_t len; double score; } ng_cand;

static int ng_cand_cmp(const void *a, const void *b) {
    const ng_cand *x = (const ng_cand *)a, *y = (const ng_cand *)b;
    if (x->score != y->score) return x->score > y->score ? -1 : 1;
    /* tie: lexicographic byte order, shorter prefix first */
    int ml = x->len < y->len ? x->len : y->len;
    for (int i = 0; i < ml; i++) {
        uint8_t bx = (uint8_t)(x->key >> (8 * i)), by = (uint8_t)(y->key >> (8 * i));
        if (bx != by) return bx < by ? -1 : 1;
    }
    return (int)x->len - (int)y->len;
}

/* Top-`max_syms` 1..8-grams of a sample by count x length (byte coverage).
 * n-grams do not cross string boundaries.  Returns the number of symbols. */
int dg_fsst_ngram_table(const uint8_t *bytes, const int64_t *offsets, int64_t n_strings, int max_syms,
                        uint8_t *out_bytes, uint8_t *out_lens) {
    int64_t total = offsets[n_strings] - offsets[0];
    uint64_t cap = 1;
    while (cap < (uint64_t)(total * 8 * 2 + 1024)) cap <<= 1;
    if (cap > (1ULL << 26)) cap = 1ULL << 26;
    ng_ent *tab = (ng_ent *)calloc(cap, sizeof(ng_ent));
    uint64_t used = 0;
    for (int64_t s = 0; s < n_strings; s++) {
        const uint8_t *p = bytes + offsets[s];
        int64_t L = offsets[s + 1] - offsets[s];
        for (int64_t i = 0; i < L; i++) {
            uint64_t key = 0;
            for (int n = 1; n <= 8 && i + n <= L; n++) {
                key |= (uint64_t)p[i + n - 1] << (8 * (n - 1));
                uint64_t h = mix64(key * 16 + (uint64_t)n) & (cap - 1);
                for (;;) {
                    if (tab[h].len == 0) {
                        if (used * 10 > cap * 7) break; /* table full: drop (never happens at the sizes used) */
                        tab[h].key = key; tab[h].len = (uint8_t)n; tab[h].cnt = 1; used++;
                        break;
                    }
                    if (tab[h].key == key && tab[h].len == n) { tab[h].cnt++; break; }
                    h = (h + 1) & (cap - 1);
                }
            }
        }
    }
    ng_cand *c = (ng_cand *)malloc(sizeof(ng_cand) * (used ? used : 1));
    uint64_t nc = 0;
    for (uint64_t h = 0; h < cap; h++)
        if (tab[h].len) {
            c[nc].key = tab[h].key; c[nc].cnt = tab[h].cnt; c[nc].len = tab[h].len;
            c[nc].score = (double)tab[h].cnt * tab[h].len;
            nc++;
        }
    free(tab);
    qsort(c, nc, sizeof(ng_cand), ng_cand_cmp);
    int n = (int)(nc < (uint64_t)max_syms ? nc : (uint64_t)max_syms);
    int64_t pos = 0;
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < c[i].len; j++) out_bytes[pos + j] = (uint8_t)(c[i].key >> (8 * j));
        out_lens[i] = c[i].len;
        pos += c[i].len;
    }
    free(c);
    return n;
}

/* ------------------------------------------------------------------------- */
/* Trie for greedy longest match                                              */
/*   root children dense, level-1 children dense (256x256), deeper levels in  */
/*   an open-addressing hash keyed by (node, byte).                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t *term;       /* code at node, -1 if none */
    int32_t n_nodes, cap_nodes;
    int32_t root_child[256];
    int32_t *l1_child;   /* [256*256] for depth-1 nodes, indexed by first byte */
    uint64_t *hkey;      /* (node<<8|byte)+1, 0 = empty */
    int32_t *hval;
    uint64_t hcap, hused;
    int max_len;
} trie_t;

static void trie_init(trie_t *t, int expected_nodes, int max_len) {
    memset(t, 0, sizeof(*t));
    t->cap_nodes = expected_nodes + 300;
    t->term = (int32_t *)malloc(sizeof(int32_t) * (size_t)t->cap_nodes);
    t->n_nodes = 1;
    t->term[0] = -1;
    for (int i = 0; i < 256; i++) t->root_child[i] = -1;
    t->l1_child = (int32_t *)malloc(sizeof(int32_t) * 65536);
    for (int i = 0; i < 65536; i++) t->l1_child[i] = -1;
    t->hcap = 1;
    while (t->hcap < (uint64_t)expected_nodes * 2 + 1024) t->hcap <<= 1;
    t->hkey = (uint64_t *)calloc(t->hcap, sizeof(uint64_t));
    t->hval = (int32_t *)malloc(sizeof(int32_t) * t->hcap);
    t->max_len = max_len;
}
static void trie_free(trie_t *t) { free(t->term); free(t->l1_child); free(t->hkey); free(t->hval); }

static inline int32_t trie_hget(const trie_t *t, int32_t node, uint8_t b) {
    uint64_t key = (((uint64_t)node << 8) | b) + 1;
    uint64_t h = mix64(key) & (t->hcap - 1);
    for (;;) {
        uint64_t k = t->hkey[h];
        if (k == key) return t->hval[h];
        if (k == 0) return -1;
        h = (h + 1) & (t->hcap - 1);
    }
}
static void trie_hrehash(trie_t *t) {
    uint64_t oc = t->hcap;
    uint64_t *ok = t->hkey;
    int32_t *ov = t->hval;
    t->hcap = oc * 2;
    t->hkey = (uint64_t *)calloc(t->hcap, sizeof(uint64_t));
    t->hval = (int32_t *)malloc(sizeof(int32_t) * t->hcap);
    for (uint64_t i = 0; i < oc; i++)
        if (ok[i]) {
            uint64_t h = mix64(ok[i]) & (t->hcap - 1);
            while (t->hkey[h]) h = (h + 1) & (t->hcap - 1);
            t->hkey[h] = ok[i]; t->hval[h] = ov[i];
        }
    free(ok); free(ov);
}
static int32_t trie_new_node(trie_t *t) {
    if (t->n_nodes == t->cap_nodes) {
        t->cap_nodes *= 2;
        t->term = (int32_t *)realloc(t->term, sizeof(int32_t) * (size_t)t->cap_nodes);
    }
    t->term[t->n_nodes] = -1;
    return t->n_nodes++;
}
/* child of `node` reached at depth `depth` (0 = root) through byte b; first
 * byte of the path is `b0` (used for the dense level-1 table). */
static inline int32_t trie_child(const trie_t *t, int32_t node, int depth, uint8_t b0, uint8_t b) {
    if (depth == 0) return t->root_child[b];
    if (depth == 1) return t->l1_child[(int)b0 * 256 + b];
    return trie_hget(t, node, b);
}
static void trie_insert(trie_t *t, const uint8_t *s, int l, int32_t code) {
    int32_t node = 0;
    for (int d = 0; d < l; d++) {
        int32_t c = trie_child(t, node, d, s[0], s[d]);
        if (c < 0) {
            c = trie_new_node(t);
            if (d == 0) t->root_child[s[0]] = c;
            else if (d == 1) t->l1_child[(int)s[0] * 256 + s[1]] = c;
            else {
                if ((t->hused + 1) * 2 > t->hcap) trie_hrehash(t);
                uint64_t key = (((uint64_t)node << 8) | s[d]) + 1;
                uint64_t h = mix64(key) & (t->hcap - 1);
                while (t->hkey[h]) h = (h + 1) & (t->hcap - 1);
                t->hkey[h] = key; t->hval[h] = c; t->hused++;
            }
        }
        node = c;
    }
    if (t->term[node] < 0) t->term[node] = code;
}
/* longest match at s[0..rem); returns code (or -1) and writes its length */
static inline int32_t trie_longest(const trie_t *t, const uint8_t *s, int64_t rem, int *out_len) {
    int32_t node = 0, best = -1;
    int bl = 0;
    int lim = rem < t->max_len ? (int)rem : t->max_len;
    for (int d = 0; d < lim; d++) {
        node = trie_child(t, node, d, s[0], s[d]);
        if (node < 0) break;
        if (t->term[node] >= 0) { best = t->term[node]; bl = d + 1; }
    }
    *out_len = bl;
    return best;
}
static int32_t trie_longest_fwd(const trie_t *t, const uint8_t *s, int64_t rem, int *out_len) {
    return trie_longest(t, s, rem, out_len);
}
static int trie_contains(const trie_t *t, const uint8_t *s, int l) {
    int32_t node = 0;
    for (int d = 0; d < l; d++) {
        node = trie_child(t, node, d, s[0], s[d]);
        if (node < 0) return 0;
    }
    return t->term[node] >= 0;
}

/* FSST-style training: several rounds of (greedy parse of the sample with the
 * current table -> count each parsed unit and each adjacent unit pair whose
 * concatenation is <= 8 bytes -> keep the `max_syms` candidates that cover the
 * most sample bytes, gain = count x length).  Unmatched bytes are parsed as
 * single-byte literal units, so frequent bytes enter the table.  Returns the
 * number of symbols; out_bytes packed. */
typedef struct { uint64_t key; uint8_t len; uint64_t cnt; } fc_ent;

static void fc_add(fc_ent *tab, uint64_t cap, uint64_t *used, uint64_t key, int len, uint64_t add) {
    uint64_t h = mix64(key * 16 + (uint64_t)len) & (cap - 1);
    for (;;) {
        if (tab[h].len == 0) {
            if ((*used + 1) * 10 > cap * 7) return;
            tab[h].key = key; tab[h].len = (uint8_t)len; tab[h].cnt = add; (*used)++;
            return;
        }
        if (tab[h].key == key && tab[h].len == len) { tab[h].cnt += add; return; }
        h = (h + 1) & (cap - 1);
    }
}

static void trie_free(trie_t *t);
static void trie_init(trie_t *t, int expected_nodes, int max_len);
static void trie_insert(trie_t *t, const uint8_t *s, int l, int32_t code);
static int32_t trie_longest_fwd(const trie_t *t, const uint8_t *s, int64_t rem, int *out_len);

int dg_fsst_train(const uint8_t *bytes, const int64_t *offsets, int64_t n_strings, int max_syms, int rounds,
                  uint8_t *out_bytes, uint8_t *out_lens) {
    uint64_t syms[255];
    uint8_t slen[255];
    int n = 0;
    uint64_t cap = 1 << 22;
    fc_ent *tab = (fc_ent *)malloc(sizeof(fc_ent) * cap);
    ng_cand *c = (ng_cand *)malloc(sizeof(ng_cand) * cap);
    for (int round = 0; round < rounds; round++) {
        trie_t t;
        trie_init(&t, 4096, 8);
        for (int i = 0; i < n; i++) {
            uint8_t b[8];
            for (int j = 0; j < slen[i]; j++) b[j] = (uint8_t)(syms[i] >> (8 * j));
            trie_insert(&t, b, slen[i], i);
        }
        memset(tab, 0, sizeof(fc_ent) * cap);
        uint64_t used = 0;
        for (int64_t s = 0; s < n_strings; s++) {
            const uint8_t *p = bytes + offsets[s];
            int64_t L = offsets[s + 1] - offsets[s], pos = 0;
            uint64_t pk = 0;
            int pl = 0;
            while (pos < L) {
                int l;
                int32_t code = trie_longest_fwd(&t, p + pos, L - pos, &l);
                uint64_t k;
                if (code < 0) { k = p[pos]; l = 1; } else { k = syms[code]; }
                fc_add(tab, cap, &used, k, l, 1);
                if (pl && pl + l <= 8) fc_add(tab, cap, &used, pk | (k << (8 * pl)), pl + l, 1);
                pk = k; pl = l;
                pos += l;
            }
        }
        trie_free(&t);
        uint64_t nc = 0;
        for (uint64_t h = 0; h < cap; h++)
            if (tab[h].len) {
                c[nc].key = tab[h].key; c[nc].len = tab[h].len; c[nc].cnt = (uint32_t)tab[h].cnt;
                c[nc].score = (double)tab[h].cnt * tab[h].len;
                nc++;
            }
        qsort(c, nc, sizeof(ng_cand), ng_cand_cmp);
        n = (int)(nc < (uint64_t)max_syms ? nc : (uint64_t)max_syms);
        for (int i = 0; i < n; i++) { syms[i] = c[i].key; slen[i] = c[i].len; }
    }
    free(tab); free(c);
    int64_t pos = 0;
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < slen[i]; j++) out_bytes[pos + j] = (uint8_t)(syms[i] >> (8 * j));
        out_lens[i] = slen[i];
        pos += slen[i];
    }
    return n;
}

/* ------------------------------------------------------------------------- */
/* OnPair-style trainer                                                       */
/* ------------------------------------------------------------------------- */
typedef struct { uint64_t *k; uint32_t *v; uint64_t cap, used; } pairmap;
static void pm_init(pairmap *m, uint64_t cap) {
    m->cap = cap; m->used = 0;
    m->k = (uint64_t *)calloc(cap, sizeof(uint64_t));
    m->v = (uint32_t *)calloc(cap, sizeof(uint32_t));
}
static uint32_t *pm_slot(pairmap *m, uint64_t key) {
    key += 1;
    if ((m->used + 1) * 2 > m->cap) {
        uint64_t oc = m->cap;
        uint64_t *ok = m->k;
        uint32_t *ov = m->v;
        m->cap *= 2;
        m->k = (uint64_t *)calloc(m->cap, sizeof(uint64_t));
        m->v = (uint32_t *)calloc(m->cap, sizeof(uint32_t));
        for (uint64_t i = 0; i < oc; i++)
            if (ok[i]) {
                uint64_t h = mix64(ok[i]) & (m->cap - 1);
                while (m->k[h]) h = (h + 1) & (m->cap - 1);
                m->k[h] = ok[i]; m->v[h] = ov[i];
            }
        free(ok); free(ov);
    }
    uint64_t h = mix64(key) & (m->cap - 1);
    for (;;) {
        if (m->k[h] == key) return &m->v[h];
        if (m->k[h] == 0) { m->k[h] = key; m->used++; return &m->v[h]; }
        h = (h + 1) & (m->cap - 1);
    }
}

/* Train on strings of a sample.  Tokens 0..255 are the single bytes (code =
 * byte value).  Returns n_tok; out_bytes packed (capacity max_tokens*max_len). */
int dg_onpair_train(const uint8_t *bytes, const int64_t *offsets, int64_t n_strings, int max_tokens, int tau,
                    int max_len, uint8_t *out_bytes, uint8_t *out_lens) {
    if (max_tokens < 256) return -1;
    uint8_t *tok = (uint8_t *)malloc((size_t)max_tokens * 16);
    uint8_t *tl = (uint8_t *)malloc((size_t)max_tokens);
    trie_t t;
    trie_init(&t, max_tokens * 4, max_len);
    int n = 0;
    for (int b = 0; b < 256; b++) {
        tok[n * 16] = (uint8_t)b; tl[n] = 1;
        trie_insert(&t, &tok[n * 16], 1, n);
        n++;
    }
    pairmap pm;
    pm_init(&pm, 1 << 20);
    for (int pass = 0; pass < 8 && n < max_tokens; pass++) {
        int added = 0;
        for (int64_t s = 0; s < n_strings && n < max_tokens; s++) {
            const uint8_t *p = bytes + offsets[s];
            int64_t L = offsets[s + 1] - offsets[s], pos = 0;
            int32_t prev = -1;
            while (pos < L) {
                int l;
                int32_t c = trie_longest(&t, p + pos, L - pos, &l);
                if (prev >= 0) {
                    uint32_t *cnt = pm_slot(&pm, ((uint64_t)(uint32_t)prev << 32) | (uint32_t)c);
                    (*cnt)++;
                    int nl = tl[prev] + tl[c];
                    if ((int)*cnt >= tau && nl <= max_len && n < max_tokens) {
                        uint8_t cat[32];
                        memcpy(cat, &tok[prev * 16], tl[prev]);
                        memcpy(cat + tl[prev], &tok[c * 16], tl[c]);
                        if (!trie_contains(&t, cat, nl)) {
                            memcpy(&tok[n * 16], cat, (size_t)nl);
                            tl[n] = (uint8_t)nl;
                            trie_insert(&t, cat, nl, n);
                            n++;
                            added++;
                        }
                    }
                }
                prev = c;
                pos += l;
            }
        }
        if (!added) break;
    }
    int64_t pos = 0;
    for (int i = 0; i < n; i++) {
        memcpy(out_bytes + pos, &tok[i * 16], tl[i]);
        out_lens[i] = tl[i];
        pos += tl[i];
    }
    free(pm.k); free(pm.v);
    trie_free(&t);
    free(tok); free(tl);
    return n;
}

/* Random dictionary: n_tok tokens with length uniform [1, max_len] and random
 * bytes (duplicates allowed: decoding does not care). */
int dg_random_dict(uint64_t seed, int n_tok, int max_len, uint8_t *out_bytes, uint8_t *out_lens) {
    rng_t r;
    rng_seed(&r, seed, 5);
    int64_t pos = 0;
    for (int i = 0; i < n_tok; i++) {
        int l = 1 + (int)rng_below(&r, (uint32_t)max_len);
        for (int j = 0; j < l; j++) out_bytes[pos + j] = (uint8_t)rng_below(&r, 256);
        out_lens[i] = (uint8_t)l;
        pos += l;
    }
    return n_tok;
}

/* ------------------------------------------------------------------------- */
/* Greedy longest-match encoders                                              */
/* ------------------------------------------------------------------------- */
typedef struct dg_codes {
    void *codes;
    int64_t n_codes;
    int64_t *code_off; /* n_strings + 1 */
    int64_t n_strings;
    int code_bytes;    /* 1 or 2 */
    int64_t n_escapes;
} dg_codes;

void dg_codes_free(dg_codes *c) {
    if (!c) return;
    free(c->codes);
    free(c->code_off);
    free(c);
}

typedef struct {
    const trie_t *t;
    int escape; /* 1: FSST (code 255 + literal for unmatched bytes) */
    int code_bytes;
    const uint8_t *bytes;
    const int64_t *offsets;
    int64_t n_strings;
    int nchunk;
    /* per chunk outputs */
    uint8_t **cbuf;
    int64_t *cn;      /* codes per chunk */
    int64_t *cesc;
    int64_t *counts;  /* codes per string */
} enc_ctx;

static void enc_chunk(void *vctx, int k) {
    enc_ctx *e = (enc_ctx *)vctx;
    int64_t s0 = e->n_strings * k / e->nchunk, s1 = e->n_strings * (k + 1) / e->nchunk;
    int64_t nbytes = e->offsets[s1] - e->offsets[s0];
    /* worst case: every byte escaped -> 2 codes per byte */
    uint8_t *out = (uint8_t *)malloc((size_t)(nbytes * 2 * e->code_bytes + 16));
    int64_t nc = 0, nesc = 0;
    for (int64_t s = s0; s < s1; s++) {
        const uint8_t *p = e->bytes + e->offsets[s];
        int64_t L = e->offsets[s + 1] - e->offsets[s], pos = 0, before = nc;
        while (pos < L) {
            int l;
            int32_t c = trie_longest(e->t, p + pos, L - pos, &l);
            if (c < 0) {
                /* only reachable with an escape-capable table */
                out[nc++] = 255;
                out[nc++] = p[pos];
                nesc++;
                pos += 1;
                continue;
            }
            if (e->code_bytes == 1) out[nc++] = (uint8_t)c;
            else { uint16_t v = (uint16_t)c; memcpy(out + 2 * nc, &v, 2); nc++; }
            pos += l;
        }
        e->counts[s] = nc - before;
    }
    e->cbuf[k] = out;
    e->cn[k] = nc;
    e->cesc[k] = nesc;
}

static dg_codes *encode_common(const trie_t *t, int escape, int code_bytes, const uint8_t *bytes,
                               const int64_t *offsets, int64_t n_strings, int n_threads) {
    enc_ctx e;
    e.t = t; e.escape = escape; e.code_bytes = code_bytes;
    e.bytes = bytes; e.offsets = offsets; e.n_strings = n_strings;
    e.nchunk = n_strings < 256 ? 1 : 256;
    e.cbuf = (uint8_t **)calloc((size_t)e.nchunk, sizeof(uint8_t *));
    e.cn = (int64_t *)calloc((size_t)e.nchunk, sizeof(int64_t));
    e.cesc = (int64_t *)calloc((size_t)e.nchunk, sizeof(int64_t));
    e.counts = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_strings ? n_strings : 1));
    parallel_for(e.nchunk, n_threads, enc_chunk, &e);
    dg_codes *r = (dg_codes *)calloc(1, sizeof(dg_codes));
    int64_t tot = 0, esc = 0;
    for (int k = 0; k < e.nchunk; k++) { tot += e.cn[k]; esc += e.cesc[k]; }
    r->codes = malloc((size_t)(tot * code_bytes + 16));
    r->code_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_strings + 1));
    r->code_off[0] = 0;
    for (int64_t s = 0; s < n_strings; s++) r->code_off[s + 1] = r->code_off[s] + e.counts[s];
    int64_t pos = 0;
    for (int k = 0; k < e.nchunk; k++) {
        memcpy((uint8_t *)r->codes + pos * code_bytes, e.cbuf[k], (size_t)(e.cn[k] * code_bytes));
        pos += e.cn[k];
        free(e.cbuf[k]);
    }
    r->n_codes = tot;
    r->n_strings = n_strings;
    r->code_bytes = code_bytes;
    r->n_escapes = esc;
    free(e.cbuf); free(e.cn); free(e.cesc); free(e.counts);
    return r;
}

/* FSST-8 greedy encode: longest symbol match, else escape (255) + literal. */
dg_codes *dg_encode_fsst(const uint8_t *sym_bytes, const uint8_t *sym_lens, int n_sym, const uint8_t *bytes,
                         const int64_t *offsets, int64_t n_strings, int n_threads) {
    trie_t t;
    trie_init(&t, 4096, 8);
    int64_t pos = 0;
    for (int i = 0; i < n_sym && i < 255; i++) {
        trie_insert(&t, sym_bytes + pos, sym_lens[i], i);
        pos += sym_lens[i];
    }
    dg_codes *r = encode_common(&t, 1, 1, bytes, offsets, n_strings, n_threads);
    trie_free(&t);
    return r;
}

/* OnPair-16 greedy encode (every byte must be covered by some token). Returns
 * NULL if a byte has no single-byte token. */
dg_codes *dg_encode_onpair(const uint8_t *tok_bytes, const uint8_t *tok_lens, int n_tok, const uint8_t *bytes,
                           const int64_t *offsets, int64_t n_strings, int n_threads) {
    trie_t t;
    trie_init(&t, n_tok * 4 + 1024, 16);
    int64_t pos = 0;
    int have1[256] = {0};
    for (int i = 0; i < n_tok; i++) {
        trie_insert(&t, tok_bytes + pos, tok_lens[i], i);
        if (tok_lens[i] == 1) have1[tok_bytes[pos]] = 1;
        pos += tok_lens[i];
    }
    for (int b = 0; b < 256; b++)
        if (!have1[b]) { trie_free(&t); return NULL; }
    dg_codes *r = encode_common(&t, 0, 2, bytes, offsets, n_strings, n_threads);
    trie_free(&t);
    return r;
}
