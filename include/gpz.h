/*
 * gpz.h -- C ABI of the MI355X (gfx950) GPZ particle compressor.
 *
 * GPZ (arXiv 2508.10305) compresses float32 (or float64, Sec. 5.1) particle
 * fields under a per-field absolute error bound: spatial quantization (Sec. 4.1), in-block
 * sort by segment ID (Sec. 4.2), run-length + delta + fixed-length coding
 * (Sec. 4.3) and compaction of the block records by a prefix sum of their
 * sizes (Sec. 4.4).  Decompression reverses the steps without un-sorting
 * (Sec. 3.2).  The byte layout is "stream format v1" (magic "GPZ1").
 *
 * Conventions for every entry point:
 *  - Pointers prefixed d_ are device pointers, h_ are host pointers.  Field
 *    arrays are passed as a HOST array of F device pointers (structure of
 *    arrays, one contiguous float32 array of n values per field).
 *  - The caller owns every buffer; the library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All work is enqueued on it; calls on distinct streams with distinct
 *    workspaces may run concurrently.
 *  - Status codes are returned (gpz_status); nothing throws across the ABI.
 *    On error the contents of output buffers are unspecified, and nothing
 *    outside [d_out, d_out + out_capacity) is written.
 */
#ifndef GPZ_H
#define GPZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GPZ_OK = 0,
    GPZ_EINVAL = -1,      /* bad argument: null pointer, F outside 1..64, bound not a
                             float in [2^-120, 2^120], bad parameters, workspace too small */
    GPZ_ENOSPC = -2,      /* output buffer too small; *h_out_bytes holds the size needed */
    GPZ_ECORRUPT = -3,    /* compressed stream malformed or inconsistent with n / F */
    GPZ_EDEVICE = -4,     /* a HIP runtime call failed */
    GPZ_ENOMEM = -5,      /* the library could not allocate a workspace */
    GPZ_EUNSUPPORTED = -6 /* valid request this build has no kernel for (the single-pass
                             compaction with float64 fields or a block size outside
                             256..2048) */
} gpz_status;

/* Compression parameters.
 * block_size : particles per block B, power of two, 64..4096.  256..2048
 *              run one wave per block; the other sizes (and float64 fields)
 *              run the generic kernels, one 256-lane workgroup per block.
 *              Default 1024 (32 threads x 32 points per block, Sec. 4.2).
 * seg_bits   : K, 0..5: each key axis is cut into 2^K power-of-two segments
 *              (segment size proportional to the block's range, Sec. 4.1).
 *              Default 3.
 * key_fields : KF, 1..3 and <= F: the first KF fields are the spatial
 *              coordinates whose segment IDs form the sort key.  Default
 *              min(F, 3).
 * flags      : 0 (default) or GPZ_FLAG_SINGLE_PASS.  Compression only; the
 *              stream is the same byte for byte either way, except that the
 *              single pass stores raw a block that needs 64-bit grid steps.
 *
 * 64-bit steps (Sec. 5.3: 64-bit intermediates when the value range needs
 * them): a float32 field of a block in which some finite value lies more than
 * 2^24 - 1 grid steps (2 eb each) above the block minimum is quantized in
 * double with grid indices up to 2^53 - 1, its reconstruction rounded to
 * float32; otherwise grid indices stay below 2^24 and the arithmetic is
 * float32.
 */
typedef struct {
    uint32_t block_size;
    uint32_t seg_bits;
    uint32_t key_fields;
    uint32_t flags;
} gpz_params;

/* Default compaction, the paper's design (Sec. 4.4): records to workspace
 * slots, a device scan of their lengths, a copy into the stream.  With this
 * flag the encoder places each record itself after a single-pass look-back
 * over the lengths of the earlier blocks (one launch fewer, no record copy,
 * but every block waits for the blocks before it; slower on MI355X). */
#define GPZ_FLAG_SINGLE_PASS 1u

/* Stream flags (gpz_info.flags; header word 1, bits 16 and up). */
#define GPZ_STREAM_F64 1u  /* the fields are float64 */
#define GPZ_STREAM_WIDE 2u /* some record holds a field coded with 64-bit steps */

/* Fills *p with the defaults for F fields. */
void gpz_default_params(gpz_params *p, uint32_t nfields);

/* Largest stream gpz_compress can produce for (n, F, p): every block raw.
 * Returns 0 for invalid parameters. */
uint64_t gpz_max_compressed_bytes(uint64_t n, uint32_t nfields, const gpz_params *p);

/* Device workspace gpz_compress needs (per-block record slots, lengths,
 * superblock sums and offsets, one look-back word per block): about 4*n*F
 * bytes.  Returns 0 for invalid parameters. */
uint64_t gpz_compress_workspace_bytes(uint64_t n, uint32_t nfields, const gpz_params *p);

/* Device workspace gpz_decompress needs (an error flag). */
uint64_t gpz_decompress_workspace_bytes(void);

/* Compress n particles x F float32 fields (Sec. 4.1-4.4): a clearing
 * kernel, the block encoder, the length scan and the record copy
 * (GPZ_FLAG_SINGLE_PASS: clearing kernel and encoder only).
 *  h_fields     host array of F device pointers, each to n floats.
 *  h_eb         host array of F absolute error bounds (each in [2^-120, 2^120]).
 *  p            parameters (NULL = defaults).
 *  d_out        device buffer of out_capacity bytes for the stream.
 *  h_out_bytes  receives the stream size in bytes (also on GPZ_ENOSPC).
 *  d_perm       nullable device array of n uint32: d_perm[j] = input index of
 *               the particle decompressed at position j (decompression
 *               keeps the in-block sorted order, Sec. 3.2).
 *  d_ws/ws_bytes  workspace of at least gpz_compress_workspace_bytes; d_ws ==
 *               NULL makes the library allocate and free one per call (the
 *               paper's "end-to-end" setting, Sec. 6.2.2).
 * Synchronizes `stream` before returning (the size must reach the host). */
int gpz_compress(const float *const *h_fields, uint64_t n, uint32_t nfields, const float *h_eb,
                 const gpz_params *p, void *d_out, uint64_t out_capacity, uint64_t *h_out_bytes,
                 uint32_t *d_perm, void *d_ws, uint64_t ws_bytes, void *stream);

/* As gpz_compress, without any host synchronization: the stream size is
 * written to the device scalar *d_out_bytes.  Requires out_capacity >=
 * gpz_max_compressed_bytes (so it cannot run out of space) and a caller
 * workspace.  Safe to capture in a HIP graph. */
int gpz_compress_async(const float *const *h_fields, uint64_t n, uint32_t nfields,
                       const float *h_eb, const gpz_params *p, void *d_out, uint64_t out_capacity,
                       uint64_t *d_out_bytes, uint32_t *d_perm, void *d_ws, uint64_t ws_bytes,
                       void *stream);

/* Float64 fields (Sec. 5.1): as gpz_compress, with h_fields an array of F
 * device pointers to n doubles and bounds still float32.  Each field of each
 * block is down-cast to float32 and quantized by the float32 steps when every
 * finite value is then reconstructed strictly within eb of its double
 * (|y - x| < eb in double); otherwise it is quantized from the doubles with
 * 64-bit steps (double arithmetic, grid indices up to 2^53 - 1).  Non-finite
 * values are stored verbatim (64-bit patterns).  The stream carries
 * GPZ_STREAM_F64 and decodes with gpz_decompress_f64 only.  Runs the generic
 * kernels; GPZ_FLAG_SINGLE_PASS gives GPZ_EUNSUPPORTED.  Sizes:
 * gpz_max_compressed_bytes_f64, gpz_compress_workspace_bytes_f64. */
int gpz_compress_f64(const double *const *h_fields, uint64_t n, uint32_t nfields,
                     const float *h_eb, const gpz_params *p, void *d_out, uint64_t out_capacity,
                     uint64_t *h_out_bytes, uint32_t *d_perm, void *d_ws, uint64_t ws_bytes,
                     void *stream);
uint64_t gpz_max_compressed_bytes_f64(uint64_t n, uint32_t nfields, const gpz_params *p);
uint64_t gpz_compress_workspace_bytes_f64(uint64_t n, uint32_t nfields, const gpz_params *p);

/* Decompress a stream of in_bytes bytes (Sec. 3.2) into F device arrays of n
 * floats (h_fields_out: host array of F device pointers).  n and F must
 * match the stream header.  Values come out in in-block sorted order (see
 * d_perm above).  d_ws: at least gpz_decompress_workspace_bytes (NULL: the
 * library allocates).  Synchronizes `stream` (to report corruption).  A
 * float64 stream (GPZ_STREAM_F64) gives GPZ_EINVAL: use gpz_decompress_f64. */
int gpz_decompress(const void *d_in, uint64_t in_bytes, float *const *h_fields_out, uint64_t n,
                   uint32_t nfields, void *d_ws, uint64_t ws_bytes, void *stream);

/* As gpz_decompress for a float64 stream, into F device arrays of n doubles
 * (fields coded with float32 steps are widened exactly).  A float32 stream
 * gives GPZ_EINVAL. */
int gpz_decompress_f64(const void *d_in, uint64_t in_bytes, double *const *h_fields_out,
                       uint64_t n, uint32_t nfields, void *d_ws, uint64_t ws_bytes, void *stream);

/* As gpz_decompress without any host synchronization (graph-capturable):
 * the caller supplies the parameters the stream was written with (they are
 * checked against its header on the device), in_bytes may be any upper
 * bound of the stream size (e.g. the capacity of the compression output
 * buffer), and a malformed stream sets the device flag *d_error (uint32,
 * cleared by this call) instead of returning GPZ_ECORRUPT. */
int gpz_decompress_async(const void *d_in, uint64_t in_bytes, float *const *h_fields_out,
                         uint64_t n, uint32_t nfields, const gpz_params *p, uint32_t *d_error,
                         void *stream);

/* Device workspace of the reporting calls below (gpz_bound_check,
 * gpz_error_stats, gpz_stream_stats, gpz_field_range): 32 bytes per field
 * plus 64, rounded up to 256.  0 for F outside 1..64.  With a workspace these
 * calls allocate nothing; with d_ws == NULL the library allocates and frees
 * one per call (GPZ_ENOMEM if it cannot).  A workspace may be reused by
 * calls that run one after the other on one stream, not by concurrent ones. */
uint64_t gpz_stats_workspace_bytes(uint32_t nfields);

/* Error-bound verification: recon[f][j] against orig[f][perm[j]] (d_perm
 * NULL: identity).  A pair passes when the float bits are equal or
 * |recon - orig| <= eb in IEEE double.  h_violations[F] receives the failing
 * pair count, h_max_abs_err[F] the largest |recon - orig| over pairs whose
 * difference is a number.  A perm entry outside [0, n) counts as a violation
 * and is not read.  Synchronizes `stream`. */
int gpz_bound_check(const float *const *h_orig, const float *const *h_recon,
                    const uint32_t *d_perm, uint64_t n, uint32_t nfields, const float *h_eb,
                    uint64_t *h_violations, double *h_max_abs_err, void *d_ws, uint64_t ws_bytes,
                    void *stream);

/* Per-field result of gpz_error_stats. */
typedef struct {
    uint64_t violations;  /* pairs outside the bound (as gpz_bound_check) */
    double max_abs_err;   /* largest |recon - orig| over pairs whose difference is a number */
    double sum_sq_err;    /* sum of (recon - orig)^2 over those pairs, in double; the
                             summation order is not fixed (may differ from a sequential
                             sum in the last bits) */
    double nrmse;         /* sqrt(sum_sq_err / n) / (max - min); for a zero range 0 when
                             sum_sq_err is 0, else +inf */
    float min, max;       /* range of the original field's finite values (0, 0: none) */
} gpz_field_error;

/* Rate-distortion figures of a reconstruction (Sec. 3.1): the bound check of
 * every field, its sum of squared errors and normalized RMSE over the
 * original field's value range (h_out[F]), and the aggregate PSNR
 * -20 log10 sqrt(mean over fields of NRMSE^2) in dB (*h_psnr, nullable).
 * Reads orig twice (errors, then its range).  Synchronizes `stream`. */
int gpz_error_stats(const float *const *h_orig, const float *const *h_recon,
                    const uint32_t *d_perm, uint64_t n, uint32_t nfields, const float *h_eb,
                    gpz_field_error *h_out, double *h_psnr, void *d_ws, uint64_t ws_bytes,
                    void *stream);

/* Structure statistics of a stream of n particles x F fields in device
 * memory (in_bytes: at least the stream length): h_outliers[F] receives the
 * number of values each field stores verbatim in coded blocks (Sec. 4.1
 * outliers), *h_raw_blocks the number of blocks stored raw.  GPZ_ECORRUPT
 * on a malformed header or record structure, GPZ_EINVAL when n or F differ
 * from the header.  Synchronizes `stream`. */
int gpz_stream_stats(const void *d_in, uint64_t in_bytes, uint64_t n, uint32_t nfields,
                     uint64_t *h_outliers, uint64_t *h_raw_blocks, void *d_ws, uint64_t ws_bytes,
                     void *stream);

/* Per-field minimum and maximum over finite values (h_minmax[2F]: min, max;
 * 0, 0 for a field with none; a zero extreme is returned as +0.0), used to
 * turn the value-range-relative bounds of the paper's tables into absolute
 * ones.  Synchronizes `stream`. */
int gpz_field_range(const float *const *h_fields, uint64_t n, uint32_t nfields, float *h_minmax,
                    void *d_ws, uint64_t ws_bytes, void *stream);

/* As gpz_field_range without any host synchronization (graph-capturable):
 * the 2F results (as gpz_field_range returns them) land in the device array
 * d_minmax; d_ws (required) holds at least gpz_stats_workspace_bytes(F)
 * bytes.  A serving loop can queue it with a copy of d_minmax to host memory
 * and learn the relative bound of a request when that copy completes. */
int gpz_field_range_async(const float *const *h_fields, uint64_t n, uint32_t nfields,
                          float *d_minmax, void *d_ws, uint64_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code that sets up HIP graph
 * captures, tight serving loops, harnesses that forbid hipMalloc):
 * gpz_field_range with no workspace argument and no allocation of any kind.
 * Its scratch is a library-owned device array of 2 * 64 int keys (512
 * bytes; at most 64 fields, GPZ_EINVAL beyond), one per GPU, held until the
 * process ends and reset by the call itself.  Every call on one GPU shares
 * that GPU's array, so calls that overlap on one GPU (from other host
 * threads or on other streams) race: the caller serializes them.
 * Synchronizes `stream`. */
int gpz_field_range_noalloc(const float *const *h_fields, uint64_t n, uint32_t nfields,
                            float *h_minmax, void *stream);

/* Relative bound -> absolute bound of one field: (float)(rel * (hi - lo))
 * computed in double; below 2^-120 (constant field) it is rel itself; above
 * 2^120 it is capped. */
float gpz_rel_to_abs(float rel, float lo, float hi);

/* Header fields parsed from a host copy of the first bytes of a stream.
 * Returns GPZ_ECORRUPT on a bad magic/version/parameters; needs only the 32
 * header bytes. */
typedef struct {
    uint64_t n;
    uint32_t nfields, block_size, seg_bits, key_fields;
    uint64_t nblocks;
    uint32_t flags; /* GPZ_STREAM_F64 | GPZ_STREAM_WIDE */
} gpz_info;
int gpz_inspect(const void *h_prefix, uint64_t bytes, gpz_info *out);

/* ---------------------------------------------------------------- batches
 * Batched form: many snapshots of uneven sizes, compressed or decompressed by
 * persistent kernels that take blocks from a device work queue (one launch
 * per stage for the whole batch), optionally captured once into a HIP graph
 * and replayed.  Each job's stream is byte-identical to gpz_compress of that
 * snapshot alone.  The batch owns small device tables (allocated once by
 * gpz_batch_create); the caller owns inputs, outputs and the workspace. */

typedef struct {
    const float *const *fields; /* host array of F device pointers: compression input
                                   (NULL for a job that is only decompressed) */
    uint64_t n;                 /* particles */
    uint32_t nfields;           /* F, 1..64 */
    const float *eb;            /* host array of F absolute bounds (as for gpz_compress) */
    void *out;                  /* device stream buffer: written by compression, read by
                                   decompression */
    uint64_t out_capacity;      /* bytes; >= gpz_max_compressed_bytes(n, F, p) for a job
                                   that compresses; any upper bound of the stream size for
                                   a job that only decompresses */
    float *const *dec_fields;   /* host array of F device pointers: decompression output
                                   (NULL for a job that is only compressed) */
    void *ws;                   /* device record-slot workspace of this job (at least
                                   gpz_compress_workspace_bytes(n, F, p) bytes), or NULL to
                                   carve it from the batch workspace */
} gpz_job;

typedef struct {
    uint32_t grid;       /* persistent workgroups (one wave each); default 8 per CU;
                            0: one workgroup per block of the capacity instead */
    uint32_t tile;       /* consecutive blocks taken per work-queue grab; default 1 */
    uint32_t use_graph;  /* 1: capture the kernel sequence once, then replay it */
    uint32_t max_jobs;   /* capacity for gpz_batch_rebind (0: the creation job count) */
    uint64_t max_blocks; /* capacity in blocks over all jobs (0: at creation); at most
                            2^30, and at most 2^26 when grid is 0 (GPZ_EINVAL beyond) */
} gpz_batch_config;

typedef struct gpz_batch gpz_batch;

/* Fills *c with the defaults (queries the current device's CU count). */
void gpz_default_batch_config(gpz_batch_config *c);

/* Device workspace for a job list (record slots of every block of the jobs
 * that compress without their own `ws`); 0 on invalid jobs.  All jobs share the parameters p
 * (NULL = defaults).  A batch may be created with no jobs (njobs = 0) and
 * capacities in cfg, then bound with gpz_batch_rebind. */
uint64_t gpz_batch_workspace_bytes(const gpz_job *jobs, uint32_t njobs, const gpz_params *p);

/* Creates a batch bound to `jobs` and the caller's workspace d_ws (device,
 * >= gpz_batch_workspace_bytes).  Allocates the batch's device tables, a
 * pinned host image of them and a private non-blocking stream used for graph
 * capture; the tables are on the device when it returns.  *out = NULL on
 * error. */
int gpz_batch_create(gpz_batch **out, const gpz_job *jobs, uint32_t njobs, const gpz_params *p,
                     const gpz_batch_config *cfg, void *d_ws, uint64_t ws_bytes);

/* Binds the batch to a new job list within its capacities, without device
 * allocation and without invalidating captured graphs.  Synchronizes
 * `stream` first (earlier work of this batch must have finished), then
 * queues the new tables on `stream` with one copy from pinned memory and
 * returns without waiting for it: the batch's next gpz_batch_compress /
 * gpz_batch_decompress must be issued on the same stream (or on one that
 * waits for it). */
int gpz_batch_rebind(gpz_batch *b, const gpz_job *jobs, uint32_t njobs, void *d_ws,
                     uint64_t ws_bytes, void *stream);

/* Enqueues compression of every job on `stream` (no host synchronization).
 * Stream sizes land in the device array gpz_batch_sizes(b)[job].  Every job
 * must have input fields. */
int gpz_batch_compress(gpz_batch *b, void *stream);

/* Enqueues decompression of every job's `out` stream into its dec_fields
 * (no host synchronization).  A malformed stream sets
 * gpz_batch_errors(b)[job] (device uint32) nonzero. */
int gpz_batch_decompress(gpz_batch *b, void *stream);

/* Device arrays owned by the batch, one entry per bound job: stream sizes in
 * bytes (written by gpz_batch_compress) and decode error flags (written by
 * gpz_batch_decompress).  Valid until gpz_batch_destroy; NULL for b == NULL. */
const uint64_t *gpz_batch_sizes(const gpz_batch *b);
const uint32_t *gpz_batch_errors(const gpz_batch *b);

/* Releases the batch (graphs, tables, its capture stream).  Waits for the
 * device first, so a launch still queued on any stream is not left with
 * freed tables.  NULL is a no-op. */
int gpz_batch_destroy(gpz_batch *b);

/* Optional kernel timing with HIP events recorded on the launch stream.
 * While enabled (per host thread), every compress / decompress call records
 * an event pair around each of its kernels.  gpz_timing_collect waits for
 * the recorded events, adds up the durations per kernel kind into
 * total_ms[kind] with launch counts[kind] (kind 0 encode, 1 workspace
 * clearing, 2 decode, 3 length scan, 4 record copy, 5 the generic kernels;
 * arrays of nkinds entries) and clears the log. */
int gpz_set_timing(int enable);
int gpz_timing_collect(double *total_ms, uint32_t *counts, int nkinds);

/* Like gpz_set_timing, for a subset of the kernel kinds: bit k of mask times
 * kind k (0 turns timing off; 0x3F is every kind).  Each timed kernel costs
 * an event pair on its stream, so timing only the kernels of interest keeps
 * the others' launches unchanged.  GPZ_EINVAL for bits beyond kind 5. */
int gpz_set_timing_kinds(uint32_t mask);

const char *gpz_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* GPZ_H */
