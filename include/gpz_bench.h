/*
 * gpz_bench.h -- achievable-bandwidth probes (libgpzbench.so), the
 * reference the benchmark sets beside the HBM peak.  Not part of the
 * compressor's boundary (gpz.h); nothing in libgpz.so calls them.
 *
 * Both probes stream a device buffer with 16-byte vector accesses: workgroup
 * g of `grid` 256-lane workgroups takes chunks of unroll * 4 KB, g, g + grid,
 * ..., and each lane issues its `unroll` loads (1, 2, 4, 8 or 16) before it
 * uses any.  nt != 0 marks the accesses non-temporal.  Pointers are device
 * pointers, 16-byte aligned; bytes a multiple of 16.  The call only enqueues
 * the kernel on `stream` (a hipStream_t, NULL = default).  Returns 0, -1 for
 * an invalid argument, -4 when the launch fails.
 */
#ifndef GPZ_BENCH_H
#define GPZ_BENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reads every byte of d_x once; d_sink (one uint32) is written only in the
 * practically impossible case that the folded value equals a sentinel. */
int gpzb_read(const void *d_x, uint64_t bytes, uint32_t grid, uint32_t unroll, uint32_t nt,
              uint32_t *d_sink, void *stream);

/* Copies bytes from d_x to d_y (the buffers must not overlap). */
int gpzb_copy(const void *d_x, void *d_y, uint64_t bytes, uint32_t grid, uint32_t unroll,
              uint32_t nt, void *stream);

/* Reads read_bytes from d_x and writes read_bytes * ratio_write /
 * ratio_read to d_y, in the ratio 4:1 (about the encoder's input-to-record
 * traffic) or 1:4 (the decoder's).  read_bytes must be a multiple of 64 KB;
 * d_y must hold the bytes written.  unroll 1, 2 or 4. */
int gpzb_mix(const void *d_x, void *d_y, uint64_t read_bytes, uint32_t ratio_read,
             uint32_t ratio_write, uint32_t grid, uint32_t unroll, uint32_t nt, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GPZ_BENCH_H */
