/*
 * GPZ CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct C implementation of the GPZ
 * error-bounded particle compressor (arXiv 2508.10305): spatial
 * quantization (Sec. 4.1), in-block sorting by segment ID (Sec. 4.2),
 * run-length + delta + fixed-length encoding (Sec. 4.3) and compaction by
 * a prefix sum of block sizes (Sec. 4.4), plus the reverse (Sec. 3.2:
 * decompression reverses the steps, without un-sorting).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  It shares nothing with the HIP implementation: no
 * headers, no tables, no helpers.  The byte format it writes is the one
 * frozen in the design notes ("stream format v1"); every rule the paper
 * leaves open is fixed there and restated next to the code that applies it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (no contraction, IEEE single/double arithmetic, round-to-nearest-even).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOSPC (-2)
#define OR_ECORRUPT (-3)

#define OR_MAGIC 0x315A5047u /* "GPZ1" little-endian */
#define OR_VERSION 1u
#define OR_HEADER_WORDS 8u
#define OR_SUPER 64u /* blocks per superblock offset entry */
#define OR_QMAX 16777215.0f /* largest grid index: 2^24 - 1 */
#define OR_QMAX_WIDE 9007199254740991.0 /* largest wide grid index: 2^53 - 1 */
#define OR_FLAG_F64 1u  /* stream flag (header word 1, bits 16+): float64 fields */
#define OR_FLAG_WIDE 2u /* stream flag: some record holds a field coded with 64-bit steps */

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

/* Number of significant bits of v (0 for v == 0): the "bit-width" that
 * fixed-length coding uses to drop leading zeros (Sec. 4.3). */
static uint32_t bit_width(uint32_t v) {
    uint32_t w = 0;
    while (v) {
        w++;
        v >>= 1;
    }
    return w;
}

/* The same for 64-bit grid indices (wide blocks). */
static uint32_t bit_width64(uint64_t v) {
    uint32_t w = 0;
    while (v) {
        w++;
        v >>= 1;
    }
    return w;
}

static uint64_t d2u(double d) {
    uint64_t u;
    memcpy(&u, &d, 8);
    return u;
}

static double u2d(uint64_t u) {
    double d;
    memcpy(&d, &u, 8);
    return d;
}

static uint32_t f2u(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static float u2f(uint32_t u) {
    float f;
    memcpy(&f, &u, 4);
    return f;
}

static int eb_valid(float eb) {
    /* 2^-120 <= eb <= 2^120 keeps 2*eb and 1/(2*eb) finite and normal. */
    return isfinite(eb) && eb >= 0x1p-120f && eb <= 0x1p120f;
}

static int block_size_valid(uint32_t B) {
    return B >= 64 && B <= 4096 && (B & (B - 1)) == 0;
}

/* Bit writer for fixed-length coding: value i of an array occupies bits
 * [i*w, i*w + w) of an LSB-first little-endian word stream (Sec. 4.3:
 * every value of an array is written with one uniform bit-width).  Written
 * one bit at a time on purpose. */
static void put_bits(uint32_t *words, uint64_t bitpos, uint32_t value, uint32_t w) {
    for (uint32_t b = 0; b < w; b++) {
        if ((value >> b) & 1u) {
            uint64_t p = bitpos + b;
            words[p / 32] |= 1u << (p % 32);
        }
    }
}

static uint32_t get_bits(const uint32_t *words, uint64_t bitpos, uint32_t w) {
    uint32_t v = 0;
    for (uint32_t b = 0; b < w; b++) {
        uint64_t p = bitpos + b;
        if ((words[p / 32] >> (p % 32)) & 1u) v |= 1u << b;
    }
    return v;
}

/* The same writer and reader for values of up to 64 bits. */
static void put_bits64(uint32_t *words, uint64_t bitpos, uint64_t value, uint32_t w) {
    for (uint32_t b = 0; b < w; b++) {
        if ((value >> b) & 1u) {
            uint64_t p = bitpos + b;
            words[p / 32] |= 1u << (p % 32);
        }
    }
}

static uint64_t get_bits64(const uint32_t *words, uint64_t bitpos, uint32_t w) {
    uint64_t v = 0;
    for (uint32_t b = 0; b < w; b++) {
        uint64_t p = bitpos + b;
        if ((words[p / 32] >> (p % 32)) & 1u) v |= (uint64_t)1 << b;
    }
    return v;
}

static uint32_t words_for(uint64_t count, uint32_t w) {
    return (uint32_t)((count * (uint64_t)w + 31) / 32);
}

/* ------------------------------------------------------------------ */
/* Stage 1: spatial quantization (Sec. 4.1)                             */
/* ------------------------------------------------------------------ */

/* Block boundary minimum (Sec. 4.1: per-axis extrema of the block).  Only
 * finite values take part; a block with no finite value uses 0; a minimum
 * equal to zero is stored as +0.0 so that its bits do not depend on the
 * order in which -0.0 and +0.0 were met. */
float oracle_block_min(const float *x, uint32_t n) {
    int found = 0;
    float lo = 0.0f;
    for (uint32_t i = 0; i < n; i++) {
        if (!isfinite(x[i])) continue;
        if (!found || x[i] < lo) lo = x[i];
        found = 1;
    }
    if (!found || lo == 0.0f) lo = 0.0f;
    return lo;
}

/* Grid index of one value (Sec. 4.1 equation: m*segId + segOffset =
 * (p - min)/(2 eb)).  The division is a multiplication by the reciprocal
 * 1/(2 eb) rounded once to float (Sec. 5.1, division elimination); the
 * result is rounded to the nearest integer, ties to even.  The value is an
 * outlier, to be stored verbatim, when the index falls outside [0, 2^24-1]
 * (32-bit intermediates, Sec. 5.3) or when the float32 reconstruction
 * xr = fma(q, 2 eb, min) (Sec. 5.1, explicit FMA) does not pass the bound
 * test fabsf(xr - x) < eb, evaluated in float32.  Rounding is monotone and
 * eb is a float, so a pass implies that the exact error is below eb: the
 * bound is respected strictly (Sec. 3.2). */
/* The 32-bit steps of the quantizer: grid index (0 when out of range),
 * whether it was in range, and the float32 reconstruction. */
static uint32_t narrow_index(float x, float lo, float eb, int *in_range, float *xr) {
    float twoeb = 2.0f * eb;
    float inv = 1.0f / twoeb;
    float diff = x - lo;
    float t = diff * inv;
    *in_range = (t >= 0.0f) && (t <= OR_QMAX);
    uint32_t q = 0;
    if (*in_range) q = (uint32_t)rintf(t);
    *xr = fmaf((float)q, twoeb, lo);
    return q;
}

uint32_t oracle_quantize(float x, float lo, float eb, int *outlier) {
    int in_range;
    float xr;
    uint32_t q = narrow_index(x, lo, eb, &in_range, &xr);
    float err = xr - x;
    int ok = in_range && (fabsf(err) < eb);
    *outlier = !ok;
    return q;
}

/* Grid index with 64-bit intermediates (Sec. 5.3: 64-bit values when the
 * value range or the precision needs them).  x and lo are a float32 value
 * and block minimum widened exactly, or float64 ones.  The same steps as
 * above in IEEE double: 2 eb exact, its reciprocal rounded once, the index
 * rounded to the nearest integer (ties to even) and kept when it lies in
 * [0, 2^53 - 1] (every such integer is a double); the reconstruction is the
 * double FMA q * 2eb + lo (Sec. 5.1), rounded once more to float32 when the
 * field is float32.  Outlier unless the index is in range and
 * |reconstruction - x| < eb in double: a pass again implies that the exact
 * error is below eb. */
uint64_t oracle_quantize_wide(double x, double lo, float eb, int out_f32, int *outlier) {
    double twoeb = 2.0 * (double)eb;
    double inv = 1.0 / twoeb;
    double t = (x - lo) * inv;
    int in_range = (t >= 0.0) && (t <= OR_QMAX_WIDE);
    uint64_t q = 0;
    if (in_range) q = (uint64_t)rint(t);
    double xr = fma((double)q, twoeb, lo);
    if (out_f32) xr = (double)(float)xr;
    int ok = in_range && (fabs(xr - x) < (double)eb);
    *outlier = !ok;
    return q;
}

/* Block minimum of float64 values, with the same rules as the float32 one:
 * finite values only, 0 when there is none, a zero minimum as +0.0. */
static double block_min64(const double *x, uint32_t n) {
    int found = 0;
    double lo = 0.0;
    for (uint32_t i = 0; i < n; i++) {
        if (!isfinite(x[i])) continue;
        if (!found || x[i] < lo) lo = x[i];
        found = 1;
    }
    if (!found || lo == 0.0) lo = 0.0;
    return lo;
}

/* Value reconstruction used by decompression (Sec. 5.1, FMA). */
static float reconstruct(uint32_t q, float twoeb, float lo) {
    return fmaf((float)q, twoeb, lo);
}

/* Wide reconstruction: the double FMA of the wide quantizer. */
static double reconstruct_wide(uint64_t q, double twoeb, double lo) {
    return fma((double)q, twoeb, lo);
}

/* Segment split of one key axis.  The segment size m is the power of two
 * 2^s with s = max(0, W - K), W the bit-width of the largest grid index of
 * the axis in the block: the occupied range is cut into 2^K segments, a
 * size proportional to max - min (Sec. 4.1), and the power-of-two modulus
 * becomes a bit mask (Sec. 5.1, modulo elimination). */
static uint32_t seg_shift(uint64_t qmax, uint32_t K) {
    uint32_t W = bit_width64(qmax);
    return W > K ? W - K : 0;
}

/* ------------------------------------------------------------------ */
/* Stage 2: in-block sort by segment ID (Sec. 4.2)                      */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t key;
    uint32_t idx;
} key_idx;

static int cmp_key_idx(const void *a, const void *b) {
    const key_idx *x = (const key_idx *)a, *y = (const key_idx *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

/* Stable sort of a block by segment ID: ascending ID, equal IDs keep input
 * order (the radix sort of Sec. 4.2 is stable). perm[p] = input index of
 * the particle placed at position p. */
static void sort_by_segment(const uint32_t *segId, uint32_t n, uint32_t *perm) {
    key_idx *t = (key_idx *)malloc(sizeof(key_idx) * (n ? n : 1));
    for (uint32_t i = 0; i < n; i++) {
        t[i].key = segId[i];
        t[i].idx = i;
    }
    qsort(t, n, sizeof(key_idx), cmp_key_idx);
    for (uint32_t i = 0; i < n; i++) perm[i] = t[i].idx;
    free(t);
}

/* ------------------------------------------------------------------ */
/* Stage 3: run-length + delta encoding (Sec. 4.3)                      */
/* ------------------------------------------------------------------ */

/* Run-length coding of sorted IDs: the distinct IDs in ascending order and
 * how many particles carry each.  Returns the number of runs U. */
static uint32_t run_length(const uint32_t *sorted, uint32_t n, uint32_t *uniq, uint32_t *count) {
    uint32_t U = 0;
    for (uint32_t p = 0; p < n; p++) {
        if (p == 0 || sorted[p] != sorted[p - 1]) {
            uniq[U] = sorted[p];
            count[U] = 0;
            U++;
        }
        count[U - 1]++;
    }
    return U;
}

/* Exposed step (for the worked example of Sec. 4.2): stable sort of n keys
 * followed by run-length and delta coding.  delta[j] = uniq[j] - uniq[j-1]
 * with uniq[-1] taken as 0. */
uint32_t oracle_sort_rle(const uint32_t *keys, uint32_t n, uint32_t *perm, uint32_t *uniq,
                         uint32_t *count, uint32_t *delta) {
    uint32_t *sorted = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    sort_by_segment(keys, n, perm);
    for (uint32_t p = 0; p < n; p++) sorted[p] = keys[perm[p]];
    uint32_t U = run_length(sorted, n, uniq, count);
    for (uint32_t j = 0; j < U; j++) delta[j] = uniq[j] - (j ? uniq[j - 1] : 0);
    free(sorted);
    return U;
}

/* ------------------------------------------------------------------ */
/* One block: stages 1-3 and the record layout                          */
/* ------------------------------------------------------------------ */

/* One block of input: F field pointers of float32 or float64 values. */
typedef struct {
    const float *x32[64];
    const double *x64[64];
    int f64;
} block_in;

/* Everything the encoder derives for one block, kept for inspection. */
typedef struct {
    uint32_t n, F, K, KF, U, f64;
    double lo[64];     /* block minimum (a float32 value unless wide and f64) */
    uint8_t wide[64];  /* field quantized with 64-bit intermediates */
    uint32_t s[3];
    uint32_t w_gap, w_cnt, w[64], nout[64];
    uint64_t *q;       /* F*n grid indices, input order, field-major */
    uint8_t *outlier;  /* F*n flags, input order */
    uint32_t *key;     /* n linearised segment IDs, input order */
    uint32_t *perm;    /* n: position -> input index */
    uint32_t *uniq;    /* U */
    uint32_t *count;   /* U */
    uint32_t coded_words;
} block_state;

static void block_free(block_state *st) {
    free(st->q);
    free(st->outlier);
    free(st->key);
    free(st->perm);
    free(st->uniq);
    free(st->count);
}

/* Words per stored value: 1 for float32 fields, 2 for float64 ones. */
static uint32_t value_words(int f64) { return f64 ? 2u : 1u; }

/* Stage 1 for one field of a float32 block.  The 32-bit quantizer is used
 * unless some finite value's grid index exceeds 2^24 - 1: then the field's
 * value range needs 64-bit intermediates (Sec. 5.3) and the whole field is
 * quantized by the wide steps, about the same block minimum.  Values that
 * miss the bound for any other reason stay outliers of the 32-bit steps. */
static void quantize_field_f32(const float *x, uint32_t n, float eb, block_state *st, uint32_t f) {
    uint64_t *q = st->q + (size_t)f * n;
    uint8_t *o = st->outlier + (size_t)f * n;
    float lo = oracle_block_min(x, n);
    int need_wide = 0;
    for (uint32_t i = 0; i < n; i++) {
        int in_range, outl;
        float xr;
        narrow_index(x[i], lo, eb, &in_range, &xr);
        if (isfinite(x[i]) && !in_range) need_wide = 1;
        q[i] = oracle_quantize(x[i], lo, eb, &outl);
        o[i] = (uint8_t)outl;
    }
    st->lo[f] = (double)lo;
    st->wide[f] = (uint8_t)need_wide;
    if (need_wide) {
        for (uint32_t i = 0; i < n; i++) {
            int outl;
            q[i] = oracle_quantize_wide((double)x[i], (double)lo, eb, 1, &outl);
            o[i] = (uint8_t)outl;
        }
    }
}

/* Stage 1 for one field of a float64 block (Sec. 5.1, floating-point
 * precision: a float64 input is down-cast to float32 when that is enough for
 * the bound).  The values are rounded to float32 and quantized by the 32-bit
 * steps about the block minimum of the rounded values; that is kept when
 * every finite value rounds to a finite float32, gets an in-range index and
 * is reconstructed within the bound of its ORIGINAL float64 value
 * (|y - x| < eb in double).  Otherwise the field is quantized from the
 * float64 values by the wide steps about their own block minimum.
 * Non-finite values are outliers either way. */
static void quantize_field_f64(const double *x, uint32_t n, float eb, block_state *st, uint32_t f) {
    uint64_t *q = st->q + (size_t)f * n;
    uint8_t *o = st->outlier + (size_t)f * n;
    float *xf = (float *)malloc(sizeof(float) * (n ? n : 1));
    int narrow_ok = 1;
    for (uint32_t i = 0; i < n; i++) {
        xf[i] = (float)x[i];
        if (isfinite(x[i]) && !isfinite(xf[i])) narrow_ok = 0;
    }
    float lo = oracle_block_min(xf, n);
    for (uint32_t i = 0; narrow_ok && i < n; i++) {
        if (!isfinite(x[i])) {
            q[i] = 0;
            o[i] = 1;
            continue;
        }
        int in_range;
        float y;
        q[i] = narrow_index(xf[i], lo, eb, &in_range, &y);
        o[i] = 0;
        if (!in_range || !(fabs((double)y - x[i]) < (double)eb)) narrow_ok = 0;
    }
    free(xf);
    st->wide[f] = (uint8_t)!narrow_ok;
    if (narrow_ok) {
        st->lo[f] = (double)lo;
        return;
    }
    double lo64 = block_min64(x, n);
    st->lo[f] = lo64;
    for (uint32_t i = 0; i < n; i++) {
        int outl;
        q[i] = oracle_quantize_wide(x[i], lo64, eb, 0, &outl);
        o[i] = (uint8_t)outl;
    }
}

/* Stages 1-3 for one block of n particles. */
static void analyse_block(const block_in *in, uint32_t n, uint32_t F, const float *eb, uint32_t K,
                          uint32_t KF, block_state *st) {
    memset(st, 0, sizeof(*st));
    st->n = n;
    st->F = F;
    st->K = K;
    st->KF = KF;
    st->f64 = (uint32_t)in->f64;
    st->q = (uint64_t *)calloc((size_t)F * n + 1, sizeof(uint64_t));
    st->outlier = (uint8_t *)calloc((size_t)F * n + 1, 1);
    st->key = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
    st->perm = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
    st->uniq = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
    st->count = (uint32_t *)calloc(n + 1, sizeof(uint32_t));

    /* Stage 1: block minimum and grid index of every value of every field. */
    for (uint32_t f = 0; f < F; f++) {
        if (in->f64) quantize_field_f64(in->x64[f], n, eb[f], st, f);
        else quantize_field_f32(in->x32[f], n, eb[f], st, f);
    }

    /* Stage 1 (cont.): segment ID and offset per key axis; the per-axis
     * segment IDs are linearised into one ID, axis 0 most significant. */
    for (uint32_t a = 0; a < KF; a++) {
        uint64_t qmax = 0;
        for (uint32_t i = 0; i < n; i++)
            if (st->q[(size_t)a * n + i] > qmax) qmax = st->q[(size_t)a * n + i];
        st->s[a] = seg_shift(qmax, K);
    }
    for (uint32_t i = 0; i < n; i++) {
        uint32_t segId = 0;
        for (uint32_t a = 0; a < KF; a++) {
            uint64_t q = st->q[(size_t)a * n + i];
            uint64_t m = (uint64_t)1 << st->s[a];
            uint32_t segId_a = (uint32_t)(q / m); /* same as q >> s (power-of-two m) */
            segId = segId * (1u << K) + segId_a;
        }
        st->key[i] = segId;
    }

    /* Stage 2: stable in-block sort by segment ID. */
    sort_by_segment(st->key, n, st->perm);

    /* Stage 3: run-length coding of the sorted IDs, then delta coding of the
     * distinct IDs.  Consecutive distinct IDs differ by at least one and
     * every run has at least one particle, so "delta - 1" (first ID taken
     * relative to -1) and "count - 1" are stored. */
    uint32_t *sorted = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
    for (uint32_t p = 0; p < n; p++) sorted[p] = st->key[st->perm[p]];
    st->U = run_length(sorted, n, st->uniq, st->count);
    free(sorted);
    uint32_t gmax = 0, cmax = 0;
    for (uint32_t j = 0; j < st->U; j++) {
        uint32_t gap = j == 0 ? st->uniq[0] : st->uniq[j] - st->uniq[j - 1] - 1;
        if (gap > gmax) gmax = gap;
        if (st->count[j] - 1 > cmax) cmax = st->count[j] - 1;
    }
    st->w_gap = bit_width(gmax);
    st->w_cnt = bit_width(cmax);

    /* Fixed-length widths of the per-particle arrays: segment offsets for
     * key axes, whole grid indices for the other fields. */
    uint32_t vw = value_words(in->f64);
    uint32_t words = 2 + words_for(st->U, st->w_gap) + words_for(st->U, st->w_cnt);
    for (uint32_t f = 0; f < F; f++) {
        uint64_t vmax = 0;
        uint32_t nout = 0;
        for (uint32_t i = 0; i < n; i++) {
            uint64_t q = st->q[(size_t)f * n + i];
            uint64_t v = f < KF ? (q & (((uint64_t)1 << st->s[f]) - 1u)) /* q mod m */ : q;
            if (v > vmax) vmax = v;
            nout += st->outlier[(size_t)f * n + i];
        }
        st->w[f] = bit_width64(vmax);
        st->nout[f] = nout;
        words += vw /* lo */ + 1 + words_for(n, st->w[f]) + (1 + vw) * nout;
    }
    st->coded_words = words;
}

/* Record of one block (words).  Coded layout:
 *   h0 = mode 0 | U << 2 | W << 31   (W: some field is wide)
 *   h1 = w_gap | w_cnt << 5 | s0 << 10 | s1 << 15 | s2 << 20 (bits 0-4 of
 *        each s) | (s0 >> 5) << 25 | (s1 >> 5) << 26 | (s2 >> 5) << 27
 *   gaps   : U values of w_gap bits   (uniq[j] - uniq[j-1] - 1, uniq[-1] = -1)
 *   counts : U values of w_cnt bits   (count - 1)
 *   per field f:
 *     lo_f (float32 bits; in float64 streams the double's two words, low first)
 *     field word: w_f | nout_f << 5 (32-bit steps)
 *                 or w_f | nout_f << 6 | 1 << 31 (wide steps; w_f up to 53)
 *     n values of w_f bits in sorted order
 *     nout_f outliers, ascending position: position, then the raw value
 *       (float32 bits, or the float64's two words, low first)
 * Raw layout (when the coded record would not be smaller):
 *   h0 = 1 ; then the F x n input values, field-major, input order (one
 *   word per float32, two per float64, low word first). */
static uint32_t raw_words(uint32_t n, uint32_t F, int f64) { return 1 + F * n * value_words(f64); }

static void put_value(uint32_t *rec, const block_in *in, uint32_t f, uint32_t i) {
    if (in->f64) {
        uint64_t u = d2u(in->x64[f][i]);
        rec[0] = (uint32_t)u;
        rec[1] = (uint32_t)(u >> 32);
    } else {
        rec[0] = f2u(in->x32[f][i]);
    }
}

static uint32_t write_block(const block_in *in, const block_state *st, uint32_t *rec) {
    uint32_t n = st->n, F = st->F, KF = st->KF;
    uint32_t vw = value_words(in->f64);
    uint32_t raw = raw_words(n, F, in->f64);
    if (st->coded_words >= raw) {
        rec[0] = 1;
        for (uint32_t f = 0; f < F; f++)
            for (uint32_t i = 0; i < n; i++) put_value(rec + 1 + (f * n + i) * vw, in, f, i);
        return raw;
    }
    memset(rec, 0, sizeof(uint32_t) * st->coded_words);
    uint32_t any_wide = 0;
    for (uint32_t f = 0; f < F; f++) any_wide |= st->wide[f];
    uint32_t pos = 0;
    rec[pos++] = 0u | (st->U << 2) | (any_wide << 31);
    rec[pos++] = st->w_gap | (st->w_cnt << 5) | ((st->s[0] & 31u) << 10) | ((st->s[1] & 31u) << 15) |
                 ((st->s[2] & 31u) << 20) | ((st->s[0] >> 5) << 25) | ((st->s[1] >> 5) << 26) |
                 ((st->s[2] >> 5) << 27);
    for (uint32_t j = 0; j < st->U; j++) {
        uint32_t gap = j == 0 ? st->uniq[0] : st->uniq[j] - st->uniq[j - 1] - 1;
        put_bits(rec + pos, (uint64_t)j * st->w_gap, gap, st->w_gap);
    }
    pos += words_for(st->U, st->w_gap);
    for (uint32_t j = 0; j < st->U; j++)
        put_bits(rec + pos, (uint64_t)j * st->w_cnt, st->count[j] - 1, st->w_cnt);
    pos += words_for(st->U, st->w_cnt);
    for (uint32_t f = 0; f < F; f++) {
        if (in->f64) {
            uint64_t u = d2u(st->lo[f]);
            rec[pos++] = (uint32_t)u;
            rec[pos++] = (uint32_t)(u >> 32);
        } else {
            rec[pos++] = f2u((float)st->lo[f]);
        }
        if (st->wide[f]) rec[pos++] = st->w[f] | (st->nout[f] << 6) | (1u << 31);
        else rec[pos++] = st->w[f] | (st->nout[f] << 5);
        for (uint32_t p = 0; p < n; p++) {
            uint64_t q = st->q[(size_t)f * n + st->perm[p]];
            uint64_t v = f < KF ? (q & (((uint64_t)1 << st->s[f]) - 1u)) : q;
            put_bits64(rec + pos, (uint64_t)p * st->w[f], v, st->w[f]);
        }
        pos += words_for(n, st->w[f]);
        for (uint32_t p = 0; p < n; p++) {
            uint32_t i = st->perm[p];
            if (st->outlier[(size_t)f * n + i]) {
                rec[pos++] = p;
                put_value(rec + pos, in, f, i);
                pos += vw;
            }
        }
    }
    return pos;
}

/* ------------------------------------------------------------------ */
/* Parameter checks and sizes                                           */
/* ------------------------------------------------------------------ */

static int params_valid(uint32_t F, uint32_t B, uint32_t K, uint32_t KF) {
    if (F < 1 || F > 64) return 0;
    if (!block_size_valid(B)) return 0;
    if (KF < 1 || KF > 3 || KF > F) return 0;
    if (K > 5) return 0;
    return 1;
}

static uint64_t nblocks_of(uint64_t n, uint32_t B) { return (n + B - 1) / B; }
static uint64_t nsuper_of(uint64_t nb) { return (nb + OR_SUPER - 1) / OR_SUPER; }

static uint64_t prefix_words(uint64_t n, uint32_t F, uint32_t B) {
    uint64_t nb = nblocks_of(n, B);
    return OR_HEADER_WORDS + 2 * nsuper_of(nb) + F + nb;
}

/* Largest stream: every block stored raw. */
uint64_t oracle_max_bytes_typed(uint64_t n, uint32_t F, uint32_t B, int f64) {
    if (F < 1 || F > 64 || !block_size_valid(B)) return 0;
    return 4 * (prefix_words(n, F, B) + nblocks_of(n, B) + (uint64_t)F * n * value_words(f64));
}

uint64_t oracle_max_bytes(uint64_t n, uint32_t F, uint32_t B) {
    return oracle_max_bytes_typed(n, F, B, 0);
}

/* ------------------------------------------------------------------ */
/* Stage 4: compaction (Sec. 4.4) -- full compress                       */
/* ------------------------------------------------------------------ */

static int compress_impl(const float *const *f32, const double *const *f64, uint64_t n, uint32_t F,
                         const float *eb, uint32_t B, uint32_t K, uint32_t KF, uint8_t *out,
                         uint64_t cap, uint64_t *out_bytes, uint32_t *perm_out) {
    int is64 = f64 != NULL;
    if (!params_valid(F, B, K, KF)) return OR_EINVAL;
    for (uint32_t f = 0; f < F; f++)
        if (!eb_valid(eb[f])) return OR_EINVAL;
    if (n > 0 && ((f32 == NULL && f64 == NULL) || out == NULL)) return OR_EINVAL;
    for (uint32_t f = 0; n > 0 && f < F; f++)
        if ((is64 ? (const void *)f64[f] : (const void *)f32[f]) == NULL) return OR_EINVAL;

    uint64_t nb = nblocks_of(n, B), ns = nsuper_of(nb);
    uint64_t pre = prefix_words(n, F, B);
    uint32_t *lens = (uint32_t *)calloc(nb + 1, sizeof(uint32_t));
    uint32_t **recs = (uint32_t **)calloc(nb + 1, sizeof(uint32_t *));
    uint64_t total = pre;
    int any_wide = 0;
    for (uint64_t b = 0; b < nb; b++) {
        uint32_t nn = (uint32_t)((b + 1) * B <= n ? B : n - b * B);
        block_in in;
        memset(&in, 0, sizeof(in));
        in.f64 = is64;
        for (uint32_t f = 0; f < F; f++) {
            if (is64) in.x64[f] = f64[f] + b * B;
            else in.x32[f] = f32[f] + b * B;
        }
        block_state st;
        analyse_block(&in, nn, F, eb, K, KF, &st);
        uint32_t rw = raw_words(nn, F, is64);
        uint32_t cap_words = st.coded_words > rw ? st.coded_words : rw;
        recs[b] = (uint32_t *)calloc(cap_words, sizeof(uint32_t));
        lens[b] = write_block(&in, &st, recs[b]);
        if (recs[b][0] >> 31) any_wide = 1;
        if (perm_out) {
            int raw = recs[b][0] == 1u;
            for (uint32_t p = 0; p < nn; p++) perm_out[b * B + p] = (uint32_t)(b * B + (raw ? p : st.perm[p]));
        }
        block_free(&st);
        total += lens[b];
    }
    *out_bytes = 4 * total;
    int rc = OR_OK;
    if (4 * total > cap || (total > 0 && out == NULL)) {
        rc = OR_ENOSPC;
    } else {
        uint32_t *w = (uint32_t *)malloc(4 * total);
        w[0] = OR_MAGIC;
        w[1] = OR_VERSION | (((is64 ? OR_FLAG_F64 : 0u) | (any_wide ? OR_FLAG_WIDE : 0u)) << 16);
        w[2] = (uint32_t)(n & 0xFFFFFFFFu);
        w[3] = (uint32_t)(n >> 32);
        w[4] = F;
        w[5] = B;
        w[6] = K | (KF << 8);
        w[7] = (uint32_t)nb;
        uint32_t *sup = w + OR_HEADER_WORDS;
        uint32_t *ebt = sup + 2 * ns;
        uint32_t *lt = ebt + F;
        uint32_t *rec = lt + nb;
        for (uint32_t f = 0; f < F; f++) ebt[f] = f2u(eb[f]);
        uint64_t off = 0; /* exclusive prefix sum of record lengths */
        for (uint64_t b = 0; b < nb; b++) {
            if (b % OR_SUPER == 0) {
                sup[2 * (b / OR_SUPER)] = (uint32_t)(off & 0xFFFFFFFFu);
                sup[2 * (b / OR_SUPER) + 1] = (uint32_t)(off >> 32);
            }
            lt[b] = lens[b];
            memcpy(rec + off, recs[b], 4 * (size_t)lens[b]);
            off += lens[b];
        }
        memcpy(out, w, 4 * total);
        free(w);
    }
    for (uint64_t b = 0; b < nb; b++) free(recs[b]);
    free(recs);
    free(lens);
    return rc;
}

/* Stream layout (words, little-endian):
 *   0: magic "GPZ1"   1: version 1 | flags << 16 (flag 1: float64 fields;
 *      flag 2: some record has a field coded with the 64-bit steps)
 *   2-3: N (u64)   4: F   5: B   6: K | KF << 8    7: number of blocks
 *   superblock table: one u64 per 64 blocks = word offset of the
 *                     superblock's first record inside the record area
 *   eb table: F float bits
 *   length table: record length in words, one per block
 *   records, in block order.
 * The record offsets are the exclusive prefix sum of the record lengths
 * (Sec. 4.4). */
int oracle_compress(const float *const *fields, uint64_t n, uint32_t F, const float *eb, uint32_t B,
                    uint32_t K, uint32_t KF, uint8_t *out, uint64_t cap, uint64_t *out_bytes,
                    uint32_t *perm_out) {
    if (n > 0 && fields == NULL) return OR_EINVAL;
    return compress_impl(fields, NULL, n, F, eb, B, K, KF, out, cap, out_bytes, perm_out);
}

/* Float64 fields (Sec. 5.1): the same stream with the float64 flag, each
 * field of each block down-cast to float32 where that meets the bound. */
int oracle_compress_f64(const double *const *fields, uint64_t n, uint32_t F, const float *eb,
                        uint32_t B, uint32_t K, uint32_t KF, uint8_t *out, uint64_t cap,
                        uint64_t *out_bytes, uint32_t *perm_out) {
    if (n > 0 && fields == NULL) return OR_EINVAL;
    if (n == 0) {
        static const double *none[64];
        return compress_impl(NULL, none, n, F, eb, B, K, KF, out, cap, out_bytes, perm_out);
    }
    return compress_impl(NULL, fields, n, F, eb, B, K, KF, out, cap, out_bytes, perm_out);
}

/* One block's record alone (for spot checks of large streams). */
int oracle_encode_block(const float *const *x, uint32_t n, uint32_t F, const float *eb, uint32_t K,
                        uint32_t KF, uint32_t *rec, uint32_t cap_words, uint32_t *rec_words,
                        uint32_t *perm_out) {
    if (n == 0 || n > 4096 || F < 1 || F > 64 || KF < 1 || KF > 3 || KF > F || K > 5) return OR_EINVAL;
    for (uint32_t f = 0; f < F; f++)
        if (!eb_valid(eb[f])) return OR_EINVAL;
    block_in in;
    memset(&in, 0, sizeof(in));
    for (uint32_t f = 0; f < F; f++) in.x32[f] = x[f];
    block_state st;
    analyse_block(&in, n, F, eb, K, KF, &st);
    uint32_t need = st.coded_words >= raw_words(n, F, 0) ? raw_words(n, F, 0) : st.coded_words;
    *rec_words = need;
    if (need > cap_words) {
        block_free(&st);
        return OR_ENOSPC;
    }
    uint32_t len = write_block(&in, &st, rec);
    if (perm_out)
        for (uint32_t p = 0; p < n; p++) perm_out[p] = rec[0] == 1u ? p : st.perm[p];
    block_free(&st);
    return (int)(len == need ? OR_OK : OR_EINVAL);
}

/* Inspection of one block: the intermediate results of stages 1-3.
 * Arrays are caller-owned: lo[F], wide[F], s[3], q[F*n], outlier[F*n],
 * key[n], perm[n], uniq[n], count[n]; widths[2+F] = w_gap, w_cnt, w_f...
 * x64 non-NULL: the block is float64 (x ignored). */
int oracle_block_trace(const float *const *x, const double *const *x64, uint32_t n, uint32_t F,
                       const float *eb, uint32_t K, uint32_t KF, double *lo, uint8_t *wide,
                       uint32_t *s, uint64_t *q, uint8_t *outlier, uint32_t *key, uint32_t *perm,
                       uint32_t *uniq, uint32_t *count, uint32_t *widths, uint32_t *U_out,
                       uint32_t *coded_words) {
    if (n == 0 || F < 1 || F > 64 || KF < 1 || KF > 3 || KF > F || K > 5) return OR_EINVAL;
    block_in in;
    memset(&in, 0, sizeof(in));
    in.f64 = x64 != NULL;
    for (uint32_t f = 0; f < F; f++) {
        if (x64) in.x64[f] = x64[f];
        else in.x32[f] = x[f];
    }
    block_state st;
    analyse_block(&in, n, F, eb, K, KF, &st);
    for (uint32_t f = 0; f < F; f++) {
        lo[f] = st.lo[f];
        wide[f] = st.wide[f];
    }
    for (uint32_t a = 0; a < 3; a++) s[a] = st.s[a];
    memcpy(q, st.q, sizeof(uint64_t) * F * n);
    memcpy(outlier, st.outlier, (size_t)F * n);
    memcpy(key, st.key, sizeof(uint32_t) * n);
    memcpy(perm, st.perm, sizeof(uint32_t) * n);
    memcpy(uniq, st.uniq, sizeof(uint32_t) * st.U);
    memcpy(count, st.count, sizeof(uint32_t) * st.U);
    widths[0] = st.w_gap;
    widths[1] = st.w_cnt;
    for (uint32_t f = 0; f < F; f++) widths[2 + f] = st.w[f];
    *U_out = st.U;
    *coded_words = st.coded_words;
    block_free(&st);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Decompression (Sec. 3.2): decode, reconstruct, no un-sorting          */
/* ------------------------------------------------------------------ */

/* Decoded values go to float32 or float64 arrays (one of y32 / y64). */
typedef struct {
    float *const *y32;
    double *const *y64;
} block_out;

static void out_value(const block_out *o, uint32_t f, uint64_t i, double v) {
    if (o->y64) o->y64[f][i] = v;
    else o->y32[f][i] = (float)v;
}

static void out_raw(const block_out *o, uint32_t f, uint64_t i, const uint32_t *w) {
    if (o->y64) o->y64[f][i] = u2d((uint64_t)w[0] | ((uint64_t)w[1] << 32));
    else o->y32[f][i] = u2f(w[0]);
}

static int decode_block(const uint32_t *rec, uint32_t len, uint32_t n, uint32_t F, uint32_t K,
                        uint32_t KF, const float *eb, const block_out *y, uint64_t base,
                        int wide_allowed) {
    int f64 = y->y64 != NULL;
    uint32_t vw = value_words(f64);
    if (len < 1) return OR_ECORRUPT;
    uint32_t mode = rec[0] & 3u;
    if (mode == 1) {
        if (rec[0] != 1u || len != raw_words(n, F, f64)) return OR_ECORRUPT;
        for (uint32_t f = 0; f < F; f++)
            for (uint32_t i = 0; i < n; i++) out_raw(y, f, base + i, rec + 1 + (f * n + i) * vw);
        return OR_OK;
    }
    if (mode != 0 || len < 2) return OR_ECORRUPT;
    uint32_t U = (rec[0] & 0x7FFFFFFFu) >> 2, any_wide = rec[0] >> 31;
    /* a stream announces wide records in its header (decoders may skip the
     * search for them otherwise) */
    if (any_wide && !wide_allowed) return OR_ECORRUPT;
    uint32_t h1 = rec[1];
    uint32_t w_gap = h1 & 31u, w_cnt = (h1 >> 5) & 31u;
    uint32_t s[3];
    for (uint32_t a = 0; a < 3; a++) s[a] = ((h1 >> (10 + 5 * a)) & 31u) | (((h1 >> (25 + a)) & 1u) << 5);
    if ((h1 >> 28) != 0 || U < 1 || U > n || w_gap > 15 || w_cnt > 12) return OR_ECORRUPT;
    for (uint32_t a = 0; a < 3; a++) {
        if (a >= KF && s[a] != 0) return OR_ECORRUPT;
        if (a < KF && s[a] + K > 53) return OR_ECORRUPT;
    }
    uint64_t pos = 2;
    uint64_t need = pos + words_for(U, w_gap) + words_for(U, w_cnt);
    if (need > len) return OR_ECORRUPT;
    const uint32_t *gaps = rec + pos;
    pos += words_for(U, w_gap);
    const uint32_t *cnts = rec + pos;
    pos += words_for(U, w_cnt);

    /* Undo delta and run-length coding: the segment ID of every position. */
    uint32_t *segId = (uint32_t *)malloc(sizeof(uint32_t) * n);
    int64_t id = -1;
    uint64_t p = 0;
    uint64_t idlimit = (uint64_t)1 << (K * KF);
    for (uint32_t j = 0; j < U; j++) {
        id = id + (int64_t)get_bits(gaps, (uint64_t)j * w_gap, w_gap) + 1;
        uint64_t c = (uint64_t)get_bits(cnts, (uint64_t)j * w_cnt, w_cnt) + 1;
        if ((uint64_t)id >= idlimit || p + c > n) {
            free(segId);
            return OR_ECORRUPT;
        }
        for (uint64_t k = 0; k < c; k++) segId[p++] = (uint32_t)id;
    }
    if (p != n) {
        free(segId);
        return OR_ECORRUPT;
    }
    uint32_t seen_wide = 0;
    for (uint32_t f = 0; f < F; f++) {
        if (pos + vw + 1 > len) {
            free(segId);
            return OR_ECORRUPT;
        }
        double lo = f64 ? u2d((uint64_t)rec[pos] | ((uint64_t)rec[pos + 1] << 32))
                        : (double)u2f(rec[pos]);
        uint32_t wword = rec[pos + vw];
        uint32_t wide = wword >> 31;
        uint32_t w = wide ? (wword & 63u) : (wword & 31u);
        uint32_t nout = wide ? ((wword >> 6) & 0x1FFFFFFu) : ((wword >> 5) & 0x3FFFFFFu);
        pos += vw + 1;
        seen_wide |= wide;
        /* 32-bit steps: grid indices below 2^24; wide ones below 2^53 */
        uint32_t qbits = wide ? 53 : 24;
        uint32_t wlimit = f < KF ? s[f] : qbits;
        if ((f < KF && s[f] + K > qbits) || w > wlimit || nout > n ||
            pos + words_for(n, w) + (uint64_t)(1 + vw) * nout > len) {
            free(segId);
            return OR_ECORRUPT;
        }
        float twoeb = 2.0f * eb[f];
        double twoeb64 = 2.0 * (double)eb[f];
        for (uint32_t pp = 0; pp < n; pp++) {
            uint64_t v = get_bits64(rec + pos, (uint64_t)pp * w, w);
            uint64_t q;
            if (f < KF) {
                /* segment ID of axis f, then segId * m + segOffset */
                uint64_t sid = (segId[pp] >> (K * (KF - 1 - f))) & ((1u << K) - 1u);
                q = sid * ((uint64_t)1 << s[f]) + v;
            } else {
                q = v;
            }
            double yv;
            if (wide) {
                yv = reconstruct_wide(q, twoeb64, lo);
                if (!f64) yv = (double)(float)yv;
            } else {
                yv = (double)reconstruct((uint32_t)q, twoeb, (float)lo);
            }
            out_value(y, f, base + pp, yv);
        }
        pos += words_for(n, w);
        int64_t last = -1;
        for (uint32_t k = 0; k < nout; k++) {
            uint32_t op = rec[pos];
            if (op >= n || (int64_t)op <= last) {
                free(segId);
                return OR_ECORRUPT;
            }
            last = op;
            out_raw(y, f, base + op, rec + pos + 1);
            pos += 1 + vw;
        }
    }
    free(segId);
    if (seen_wide != any_wide) return OR_ECORRUPT;
    return pos == len ? OR_OK : OR_ECORRUPT;
}

/* Header fields of a stream (host-side parse). info[0..7] =
 * N, F, B, K, KF, nblocks, total bytes implied by the tables, flags. */
int oracle_inspect(const uint8_t *in, uint64_t bytes, uint64_t *info) {
    if (bytes < 4 * OR_HEADER_WORDS || bytes % 4 != 0) return OR_ECORRUPT;
    const uint32_t *w = (const uint32_t *)in;
    uint32_t flags = w[1] >> 16;
    if (w[0] != OR_MAGIC || (w[1] & 0xFFFFu) != OR_VERSION ||
        (flags & ~(OR_FLAG_F64 | OR_FLAG_WIDE)) != 0)
        return OR_ECORRUPT;
    uint64_t n = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
    uint32_t F = w[4], B = w[5], K = w[6] & 0xFFu, KF = (w[6] >> 8) & 0xFFu;
    if ((w[6] >> 16) != 0 || !params_valid(F, B, K, KF)) return OR_ECORRUPT;
    uint64_t nb = nblocks_of(n, B);
    if (w[7] != (uint32_t)nb || nb > 0xFFFFFFFFull) return OR_ECORRUPT;
    uint64_t pre = prefix_words(n, F, B);
    if (4 * pre > bytes) return OR_ECORRUPT;
    const uint32_t *lt = w + OR_HEADER_WORDS + 2 * nsuper_of(nb) + F;
    uint64_t total = pre;
    for (uint64_t b = 0; b < nb; b++) total += lt[b];
    info[0] = n;
    info[1] = F;
    info[2] = B;
    info[3] = K;
    info[4] = KF;
    info[5] = nb;
    info[6] = 4 * total;
    info[7] = flags;
    return OR_OK;
}

static int decompress_impl(const uint8_t *in, uint64_t bytes, const block_out *out, uint64_t n,
                           uint32_t F) {
    uint64_t info[8];
    if (in == NULL) return OR_EINVAL;
    int rc = oracle_inspect(in, bytes, info);
    if (rc) return rc;
    if (info[0] != n || info[1] != F) return OR_EINVAL;
    /* the caller's value type must be the stream's */
    if ((info[7] & OR_FLAG_F64) != (out->y64 ? OR_FLAG_F64 : 0u)) return OR_EINVAL;
    if (info[6] != bytes) return OR_ECORRUPT;
    const uint32_t *w = (const uint32_t *)in;
    uint32_t B = (uint32_t)info[2], K = (uint32_t)info[3], KF = (uint32_t)info[4];
    uint64_t nb = info[5], ns = nsuper_of(nb);
    const uint32_t *sup = w + OR_HEADER_WORDS;
    const uint32_t *ebt = sup + 2 * ns;
    const uint32_t *lt = ebt + F;
    const uint32_t *rec = lt + nb;
    float eb[64];
    for (uint32_t f = 0; f < F; f++) {
        eb[f] = u2f(ebt[f]);
        if (!eb_valid(eb[f])) return OR_ECORRUPT;
    }
    uint64_t off = 0;
    for (uint64_t b = 0; b < nb; b++) {
        if (b % OR_SUPER == 0) {
            uint64_t so = (uint64_t)sup[2 * (b / OR_SUPER)] | ((uint64_t)sup[2 * (b / OR_SUPER) + 1] << 32);
            if (so != off) return OR_ECORRUPT;
        }
        uint32_t nn = (uint32_t)((b + 1) * B <= n ? B : n - b * B);
        rc = decode_block(rec + off, lt[b], nn, F, K, KF, eb, out, b * B,
                          (info[7] & OR_FLAG_WIDE) != 0);
        if (rc) return rc;
        off += lt[b];
    }
    return OR_OK;
}

int oracle_decompress(const uint8_t *in, uint64_t bytes, float *const *out, uint64_t n, uint32_t F) {
    block_out o = {out, NULL};
    if (n > 0 && out == NULL) return OR_EINVAL;
    return decompress_impl(in, bytes, &o, n, F);
}

int oracle_decompress_f64(const uint8_t *in, uint64_t bytes, double *const *out, uint64_t n,
                          uint32_t F) {
    static double *none[64];
    block_out o = {NULL, out ? out : none};
    if (n > 0 && out == NULL) return OR_EINVAL;
    return decompress_impl(in, bytes, &o, n, F);
}

/* ------------------------------------------------------------------ */
/* Error-bound verification and field ranges                            */
/* ------------------------------------------------------------------ */

/* recon[f][j] is compared with orig[f][perm[j]] (perm NULL: identity).
 * A pair passes when its bits are identical or |recon - orig| <= eb in
 * IEEE double.  max_err is over pairs whose difference is a number.  A
 * permutation entry outside [0, n) names no original value and counts as a
 * violation. */
int oracle_bound_check(const float *const *orig, const float *const *recon, const uint32_t *perm,
                       uint64_t n, uint32_t F, const float *eb, uint64_t *violations,
                       double *max_err) {
    for (uint32_t f = 0; f < F; f++) {
        uint64_t v = 0;
        double m = 0.0;
        for (uint64_t j = 0; j < n; j++) {
            if (perm && perm[j] >= n) {  /* no original to compare with */
                v++;
                continue;
            }
            float x = orig[f][perm ? perm[j] : j];
            float y = recon[f][j];
            double d = fabs((double)y - (double)x);
            if (!isnan(d) && d > m) m = d;
            if (f2u(x) != f2u(y) && !(d <= (double)eb[f])) v++;
        }
        violations[f] = v;
        max_err[f] = m;
    }
    return OR_OK;
}

/* Global minimum and maximum of each field over finite values (0, 0 when a
 * field has none).  A zero extreme is returned as +0.0, so that the result
 * does not depend on whether -0.0 or +0.0 was met first. */
int oracle_field_range(const float *const *fields, uint64_t n, uint32_t F, float *minmax) {
    for (uint32_t f = 0; f < F; f++) {
        int found = 0;
        float lo = 0.0f, hi = 0.0f;
        for (uint64_t i = 0; i < n; i++) {
            float x = fields[f][i];
            if (!isfinite(x)) continue;
            if (!found || x < lo) lo = x;
            if (!found || x > hi) hi = x;
            found = 1;
        }
        if (lo == 0.0f) lo = 0.0f;
        if (hi == 0.0f) hi = 0.0f;
        minmax[2 * f] = lo;
        minmax[2 * f + 1] = hi;
    }
    return OR_OK;
}

/* Rate-distortion statistics of a reconstruction (Sec. 3.1): per field the sum
 * of squared differences recon[f][j] - orig[f][perm[j]] in double, summed in
 * position order over the pairs whose difference is a number (perm entries
 * outside [0, n) are skipped); then the normalized RMSE of every field,
 * sqrt(sum_sq / n) / (max - min) over the original field's finite values,
 * and the aggregate PSNR -20 log10 sqrt(mean over fields of NRMSE^2).  A
 * field with a zero range has NRMSE 0 when it is reconstructed exactly and
 * +inf otherwise. */
int oracle_error_stats(const float *const *orig, const float *const *recon, const uint32_t *perm,
                       uint64_t n, uint32_t F, double *sum_sq, double *nrmse, double *psnr) {
    double mean = 0.0;
    for (uint32_t f = 0; f < F; f++) {
        double ss = 0.0;
        for (uint64_t j = 0; j < n; j++) {
            if (perm && perm[j] >= n) continue;
            double d = (double)recon[f][j] - (double)orig[f][perm ? perm[j] : j];
            if (isnan(d)) continue;
            ss += d * d;
        }
        sum_sq[f] = ss;
        float mm[2];
        const float *one[1] = {orig[f]};
        oracle_field_range(one, n, 1, mm);
        double range = (double)mm[1] - (double)mm[0];
        double rmse = n ? sqrt(ss / (double)n) : 0.0;
        nrmse[f] = range > 0.0 ? rmse / range : (rmse == 0.0 ? 0.0 : INFINITY);
        mean += nrmse[f] * nrmse[f];
    }
    mean /= (double)F;
    *psnr = -20.0 * log10(sqrt(mean));
    return OR_OK;
}

/* Structure statistics of a stream: the outliers stored per field (Sec. 4.3
 * records, counted in coded blocks) and the number of blocks stored raw. */
int oracle_stream_stats(const uint8_t *in, uint64_t bytes, uint64_t n, uint32_t F,
                        uint64_t *outliers, uint64_t *raw_blocks) {
    uint64_t info[8];
    int rc = oracle_inspect(in, bytes, info);
    if (rc) return rc;
    if (info[0] != n || info[1] != F) return OR_EINVAL;
    if (info[6] != bytes) return OR_ECORRUPT;
    uint32_t vw = value_words((info[7] & OR_FLAG_F64) != 0);
    const uint32_t *w = (const uint32_t *)in;
    uint32_t B = (uint32_t)info[2];
    uint64_t nb = info[5];
    const uint32_t *lt = w + OR_HEADER_WORDS + 2 * nsuper_of(nb) + F;
    const uint32_t *rec = lt + nb;
    for (uint32_t f = 0; f < F; f++) outliers[f] = 0;
    *raw_blocks = 0;
    for (uint64_t b = 0; b < nb; b++) {
        uint32_t len = lt[b];
        uint32_t nn = (uint32_t)((b + 1) * B <= n ? B : n - b * B);
        if (len < 1) return OR_ECORRUPT;
        if ((rec[0] & 3u) == 1u) {
            (*raw_blocks)++;
        } else {
            if (len < 2) return OR_ECORRUPT;
            uint32_t U = (rec[0] & 0x7FFFFFFFu) >> 2, h1 = rec[1];
            uint64_t pos = 2 + (uint64_t)words_for(U, h1 & 31u) + words_for(U, (h1 >> 5) & 31u);
            for (uint32_t f = 0; f < F; f++) {
                if (pos + vw + 1 > len) return OR_ECORRUPT;
                uint32_t wn = rec[pos + vw];
                uint32_t wide = wn >> 31;
                uint32_t w_f = wide ? (wn & 63u) : (wn & 31u);
                uint32_t nout = wide ? ((wn >> 6) & 0x1FFFFFFu) : ((wn >> 5) & 0x3FFFFFFu);
                outliers[f] += nout;
                pos += vw + 1 + (uint64_t)words_for(nn, w_f) + (uint64_t)(1 + vw) * nout;
            }
            if (pos != len) return OR_ECORRUPT;
        }
        rec += len;
    }
    return OR_OK;
}

/* Value-range-relative bound -> absolute bound of one field: rel times the
 * field's range, rounded to float; a bound that would fall below 2^-120
 * (a constant field) becomes rel itself, and one above 2^120 is capped. */
float oracle_rel_to_abs(float rel, float lo, float hi) {
    float eb = (float)((double)rel * ((double)hi - (double)lo));
    if (!(eb >= 0x1p-120f)) eb = rel;
    if (eb > 0x1p120f) eb = 0x1p120f;
    return eb;
}
