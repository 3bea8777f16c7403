/* Robustness driver for the oracle's stream readers.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests build it with AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code, gcc) and run it: it compresses
 * seeded random particle sets (float32 ones, float32 ones whose value range
 * needs 64-bit grid indices, and float64 ones), damages the streams (bit
 * flips, truncation, random length-table entries, random header words,
 * random superblock offsets) and hands them to oracle_decompress /
 * oracle_decompress_f64 and oracle_stream_stats.
 * Whatever the bytes, the readers must return a status and never read or
 * write outside their buffers; the sanitizers abort on the first violation.
 *
 * usage: fuzz_decode SEED ITERATIONS      exit 0 when every case was clean
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_compress(const float *const *fields, uint64_t n, uint32_t F, const float *eb, uint32_t B,
                    uint32_t K, uint32_t KF, uint8_t *out, uint64_t cap, uint64_t *out_bytes,
                    uint32_t *perm_out);
int oracle_compress_f64(const double *const *fields, uint64_t n, uint32_t F, const float *eb,
                        uint32_t B, uint32_t K, uint32_t KF, uint8_t *out, uint64_t cap,
                        uint64_t *out_bytes, uint32_t *perm_out);
int oracle_decompress(const uint8_t *in, uint64_t bytes, float *const *out, uint64_t n, uint32_t F);
int oracle_decompress_f64(const uint8_t *in, uint64_t bytes, double *const *out, uint64_t n,
                          uint32_t F);
int oracle_stream_stats(const uint8_t *in, uint64_t bytes, uint64_t n, uint32_t F,
                        uint64_t *outliers, uint64_t *raw_blocks);
uint64_t oracle_max_bytes_typed(uint64_t n, uint32_t F, uint32_t B, int f64);

/* splitmix64: a small, seeded generator for the cases */
static uint64_t state;
static uint64_t next(void) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint32_t below(uint32_t m) { return m ? (uint32_t)(next() % m) : 0; }
static float unit(void) { return (float)((next() >> 40) * (1.0 / 16777216.0)); }

int main(int argc, char **argv) {
    state = argc > 1 ? strtoull(argv[1], NULL, 10) : 1;
    const int iters = argc > 2 ? atoi(argv[2]) : 50;
    const uint32_t Bs[] = {64, 256, 1024, 2048};
    long decoded = 0, rejected = 0;
    for (int it = 0; it < iters; it++) {
        const uint32_t B = Bs[below(4)];
        const uint64_t n = below(3 * B + 9);
        const uint32_t F = 1 + below(6);
        const uint32_t KF = 1 + below(F < 3 ? F : 3);
        const uint32_t K = below(6);
        /* kind 0: float32; 1: float32 over a range wider than 2^24 grid
         * steps (64-bit grid indices); 2: float64 */
        const uint32_t kind = below(3);
        const float scale = kind == 1 ? 1e7f : 1000.0f;
        float eb[64];
        float *x[64];
        float *y[64];
        double *x64[64];
        double *y64[64];
        for (uint32_t f = 0; f < F; f++) {
            eb[f] = powf(10.0f, -1.0f - 5.0f * unit());
            if (kind == 2 && below(2)) eb[f] = 1e-9f;  /* finer than float32 resolves */
            x[f] = (float *)malloc(sizeof(float) * (n ? n : 1));
            y[f] = (float *)malloc(sizeof(float) * (n ? n : 1));
            x64[f] = (double *)malloc(sizeof(double) * (n ? n : 1));
            y64[f] = (double *)malloc(sizeof(double) * (n ? n : 1));
            for (uint64_t i = 0; i < n; i++) {
                float v = unit() * (below(2) ? 1.0f : scale);
                uint32_t r = below(100);
                if (r == 0) v = NAN;
                else if (r == 1) v = INFINITY;
                else if (r == 2) v = -0.0f;
                x[f][i] = v;
                x64[f][i] = (double)v + (double)unit() * 1e-9;
            }
        }
        const uint64_t cap = oracle_max_bytes_typed(n, F, B, kind == 2);
        uint8_t *s = (uint8_t *)malloc(cap);
        uint64_t len = 0;
        int crc = kind == 2
            ? oracle_compress_f64((const double *const *)x64, n, F, eb, B, K, KF, s, cap, &len, NULL)
            : oracle_compress((const float *const *)x, n, F, eb, B, K, KF, s, cap, &len, NULL);
        if (crc != 0) {
            fprintf(stderr, "compress failed (case %d)\n", it);
            return 2;
        }
        uint8_t *d = (uint8_t *)malloc(len ? len : 1);
        uint64_t outl[64], raw;
        for (int m = 0; m < 40; m++) {
            memcpy(d, s, len);
            uint64_t dl = len;
            uint32_t *w = (uint32_t *)d;
            const uint64_t words = len / 4;
            switch (below(5)) {
                case 0:  /* flip a few bits anywhere */
                    for (int k = 0; k < 1 + (int)below(4); k++)
                        d[below((uint32_t)len)] ^= (uint8_t)(1u << below(8));
                    break;
                case 1:  /* truncate */
                    dl = below((uint32_t)len + 1);
                    break;
                case 2: {  /* a random header word */
                    w[below(8)] = (uint32_t)next();
                    break;
                }
                case 3: {  /* a random value in the tables after the header */
                    if (words > 8) w[8 + below((uint32_t)(words - 8))] = (uint32_t)next();
                    break;
                }
                default:  /* a small change to one word (lengths, widths, counts) */
                    if (words) w[below((uint32_t)words)] += (uint32_t)(1 + below(3));
                    break;
            }
            /* the readers see exactly dl bytes: copy into a buffer of that size */
            uint8_t *e = (uint8_t *)malloc(dl ? dl : 1);
            memcpy(e, d, dl);
            const int drc = kind == 2 ? oracle_decompress_f64(e, dl, y64, n, F)
                                      : oracle_decompress(e, dl, y, n, F);
            if (drc == 0) decoded++;
            else rejected++;
            (void)oracle_stream_stats(e, dl, n, F, outl, &raw);
            free(e);
        }
        free(d);
        free(s);
        for (uint32_t f = 0; f < F; f++) {
            free(x[f]);
            free(y[f]);
            free(x64[f]);
            free(y64[f]);
        }
    }
    printf("fuzz_decode: %d cases, %ld damaged streams decoded, %ld rejected\n", iters, decoded,
           rejected);
    return 0;
}
