/* Robustness driver for the host logic of the C ABI.
 *
 * TEST INFRASTRUCTURE ONLY.  tests/test_host_sanitized.py compiles the
 * library's sources for the host alone (no device code) with
 * AddressSanitizer and UBSan, links this driver, and runs it without a GPU.
 * It feeds seeded random and damaged arguments to every entry point whose
 * host part does not need a device: header parsing (gpz_inspect), the size
 * and workspace queries (workspace layout), relative-bound conversion, batch
 * job validation (gpz_batch_workspace_bytes, gpz_batch_create), and the
 * argument checks and launch preparation of compress / decompress with fake
 * device addresses that the host never dereferences (kernel launches fail
 * without a device and the calls return an error status).  Whatever the
 * arguments, every call must return and the sanitizers must stay silent.
 *
 * usage: host_abi_fuzz SEED ITERATIONS    exit 0 when every case was clean
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gpz.h"

static uint64_t state;
static uint64_t next(void) { /* splitmix64 */
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint32_t below(uint32_t m) { return m ? (uint32_t)(next() % m) : 0; }

static float any_float(void) {
    switch (below(8)) {
        case 0: return NAN;
        case 1: return INFINITY;
        case 2: return -1.0f;
        case 3: return 0.0f;
        case 4: return 1e-38f;
        case 5: return 3e38f;
        default: return (float)ldexp(1.0 + (double)below(1000) / 1000.0, (int)below(80) - 40);
    }
}

static gpz_params any_params(uint32_t F) {
    gpz_params p;
    gpz_default_params(&p, F);
    static const uint32_t Bs[] = {0, 32, 64, 100, 128, 256, 512, 1024, 2048, 4096, 8192};
    if (below(2)) p.block_size = Bs[below(11)];
    if (below(3) == 0) p.seg_bits = below(8);
    if (below(3) == 0) p.key_fields = below(5);
    if (below(4) == 0) p.flags = below(4);
    return p;
}

static uint64_t any_n(void) {
    switch (below(5)) {
        case 0: return 0;
        case 1: return below(5000);
        case 2: return (uint64_t)below(1u << 30);
        case 3: return ((uint64_t)1 << 40) + below(7);
        default: return next();
    }
}

int main(int argc, char **argv) {
    state = argc > 1 ? strtoull(argv[1], NULL, 10) : 1;
    const int iters = argc > 2 ? atoi(argv[2]) : 200;
    long calls = 0;
    /* a fake device region: its address is passed, never dereferenced */
    void *fake = (void *)(uintptr_t)0x7f0000000000ull;
    for (int it = 0; it < iters; it++) {
        const uint32_t F = below(70);
        const uint64_t n = any_n();
        gpz_params p = any_params(F ? F : 1);

        /* size and workspace queries (workspace layout) */
        (void)gpz_max_compressed_bytes(n, F, below(2) ? &p : NULL);
        (void)gpz_max_compressed_bytes_f64(n, F, &p);
        (void)gpz_compress_workspace_bytes(n, F, below(2) ? &p : NULL);
        (void)gpz_compress_workspace_bytes_f64(n, F, &p);
        (void)gpz_stats_workspace_bytes(F);
        (void)gpz_rel_to_abs(any_float(), any_float(), any_float());
        calls += 6;

        /* header parsing: valid headers with damaged words, short buffers */
        uint32_t hdr[8] = {0x315A5047u, 1u | (below(4) << 16), (uint32_t)n, (uint32_t)(n >> 32),
                           F, p.block_size, p.seg_bits | (p.key_fields << 8), 0};
        if (p.block_size) hdr[7] = (uint32_t)((n + p.block_size - 1) / p.block_size);
        for (int k = 0; k < (int)below(3); k++) hdr[below(8)] = (uint32_t)next();
        gpz_info info;
        (void)gpz_inspect(hdr, below(4) ? sizeof hdr : below(32), &info);
        (void)gpz_inspect(NULL, 32, &info);
        calls += 2;

        /* batch job validation with random job lists */
        const uint32_t nj = below(6);
        gpz_job jobs[6];
        const float *fl[6][8];
        float ebs[6][8];
        for (uint32_t j = 0; j < nj; j++) {
            const uint32_t Fj = 1 + below(8);
            for (uint32_t f = 0; f < 8; f++) {
                fl[j][f] = below(10) ? (const float *)fake : NULL;
                ebs[j][f] = below(6) ? (float)ldexp(1.0, -(int)below(30)) : any_float();
            }
            memset(&jobs[j], 0, sizeof jobs[j]);
            jobs[j].fields = below(4) ? fl[j] : NULL;
            jobs[j].n = below(3) ? below(200000) : any_n();
            jobs[j].nfields = below(8) ? Fj : below(100);
            jobs[j].eb = below(10) ? ebs[j] : NULL;
            jobs[j].out = below(10) ? fake : NULL;
            jobs[j].out_capacity = below(2) ? next() >> below(64) : (uint64_t)below(1u << 30);
            jobs[j].dec_fields = below(3) ? (float *const *)fl[j] : NULL;
            jobs[j].ws = below(3) ? NULL : fake;
        }
        (void)gpz_batch_workspace_bytes(nj ? jobs : NULL, nj, below(2) ? &p : NULL);
        gpz_batch_config cfg;
        gpz_default_batch_config(&cfg);
        cfg.grid = below(3) ? cfg.grid : 0;
        cfg.tile = below(4);
        cfg.max_blocks = below(2) ? 0 : next() >> below(64);
        gpz_batch *b = NULL;
        /* argument checks run first; without a device the allocation fails */
        (void)gpz_batch_create(&b, nj ? jobs : NULL, nj, &p, &cfg, fake, below(1u << 20));
        if (b) gpz_batch_destroy(b);
        calls += 2;

        /* compress / decompress argument checks and launch preparation */
        const float *cf[70];
        float ceb[70];
        for (uint32_t f = 0; f < 70; f++) {
            cf[f] = below(20) ? (const float *)fake : NULL;
            ceb[f] = below(5) ? 1e-3f : any_float();
        }
        const uint64_t cn = below(3) ? below(100000) : any_n();
        uint64_t out_bytes = 0;
        (void)gpz_compress(below(8) ? cf : NULL, cn, F, below(8) ? ceb : NULL, below(2) ? &p : NULL,
                           below(8) ? fake : NULL, next() >> below(64), &out_bytes, NULL, fake,
                           next() >> below(64), NULL);
        (void)gpz_compress_f64((const double *const *)cf, cn, F, ceb, &p, fake, next(), &out_bytes,
                               NULL, below(2) ? fake : NULL, next() >> below(64), NULL);
        (void)gpz_compress_async(cf, cn, F, ceb, &p, fake, next() >> below(64), (uint64_t *)fake,
                                 NULL, fake, next() >> below(64), NULL);
        (void)gpz_decompress_async(fake, next() >> below(64), (float *const *)cf, cn, F, &p,
                                   (uint32_t *)fake, NULL);
        float mm[140];
        (void)gpz_field_range_async(cf, cn, F, (float *)fake, below(2) ? fake : NULL,
                                    below(4096), NULL);
        (void)gpz_field_range(cf, cn, F, below(8) ? mm : NULL, fake, below(4096), NULL);
        calls += 6;
    }
    (void)gpz_strerror(-99);
    printf("host_abi_fuzz: %d cases, %ld calls\n", iters, calls);
    return 0;
}
