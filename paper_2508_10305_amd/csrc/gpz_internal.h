// Internal declarations of the gfx950 GPZ library: kernel argument blocks,
// wave64 primitives and the launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpz {

constexpr uint32_t kMagic = 0x315A5047u;  // "GPZ1"
constexpr uint32_t kVersion = 1u;
constexpr uint32_t kHeaderWords = 8u;
constexpr uint32_t kSuper = 64u;          // blocks per superblock offset entry
constexpr uint32_t kMaxFields = 64u;
constexpr float kQMax = 16777215.0f;      // largest grid index, 2^24 - 1

// ------------------------------------------------------------ stream geometry

__host__ __device__ inline uint64_t nblocks_of(uint64_t n, uint32_t B) { return (n + B - 1) / B; }
__host__ __device__ inline uint64_t nsuper_of(uint64_t nb) { return (nb + kSuper - 1) / kSuper; }
// Words before the first record: header, superblock table, eb table, length table.
__host__ __device__ inline uint64_t prefix_words(uint64_t n, uint32_t F, uint32_t B) {
    uint64_t nb = nblocks_of(n, B);
    return kHeaderWords + 2 * nsuper_of(nb) + F + nb;
}
__host__ __device__ inline uint32_t words_for(uint32_t count, uint32_t w) {
    return (uint32_t)(((uint64_t)count * w + 31) / 32);
}
__host__ __device__ inline uint32_t bit_width(uint32_t v) { return v ? 32u - (uint32_t)__builtin_clz(v) : 0u; }

// ------------------------------------------------------------ kernel arguments

struct EncodeArgs {
    const float* x[kMaxFields];  // float32 fields, or float64 ones (f64: read as double*)
    float eb[kMaxFields];
    float twoeb[kMaxFields];
    float inv[kMaxFields];
    uint64_t n;
    uint32_t F, K, KF, B;
    uint32_t nblocks;
    uint32_t slot_words;   // record slot stride in the workspace (>= 1 + F*B)
    uint32_t* temp;        // nblocks record slots
    uint64_t* state;       // single pass: nblocks look-back words, zero before the launch
    uint32_t* ticket;      // single pass: block ticket counter, zero before the launch
    uint32_t* perm;        // nullable: n global input indices
    // three-step compaction: lengths for the scan and copy kernels
    uint32_t* lens;        // record length (words) per block
    uint32_t* supsum;      // per 64-block superblock: sum of record lengths (zeroed before)
    // single-pass compaction: records go straight to their final offsets
    uint32_t* out;
    uint64_t capacity;     // bytes of out
    uint64_t prefix;       // words before the record area
    uint64_t* total_bytes; // stream size, written by the last block
    uint64_t* ext_bytes;   // nullable second destination of the size
    uint32_t f64;          // the fields are float64
    // blocks whose grid needs 64-bit steps, left by the wave-per-block
    // encoder to the generic one (three-step compaction only)
    uint32_t* defer;       // nblocks entries
    uint32_t* defer_count; // zeroed before the launch
    uint32_t* wide_flag;   // set when a record codes a field with 64-bit steps (zeroed before)
};

// Three-step compaction (Sec. 4.4): scan of the superblock sums, then the copy.
struct ScanArgs {
    const uint32_t* supsum; // record words per superblock
    uint64_t* supoff;       // exclusive prefix of supsum (words, inside the record area)
    uint64_t* total_bytes;  // whole stream size in bytes
    uint64_t* ext_bytes;    // nullable second destination of the size (async API)
    uint32_t nsuper;
    uint64_t prefix;        // words before the record area
    // stream header, written here when the stream fits the output buffer
    uint32_t* out;
    uint64_t capacity;      // bytes
    uint64_t n;
    uint32_t F, B, K, KF, nblocks;
    uint32_t eb_bits[kMaxFields];
    uint32_t f64;               // header flag 1: float64 fields
    const uint32_t* wide_flag;  // nonzero: header flag 2 (a record has a wide field)
};

struct CopyArgs {
    const uint32_t* temp;
    const uint32_t* lens;
    const uint64_t* supoff;
    const uint64_t* total_bytes;
    uint32_t* out;
    uint64_t capacity;     // bytes
    uint32_t slot_words;
    uint32_t nblocks;
    uint32_t F;
};

struct DecodeArgs {
    const uint32_t* in;
    uint64_t in_words;
    float* y[kMaxFields];
    uint64_t n;
    uint32_t F, K, KF, B;
    uint32_t nblocks;
    uint64_t prefix;       // words before the record area
    uint32_t* err;         // set nonzero on a malformed record
    uint32_t exact;        // in_words is the exact stream length (else an upper bound)
    uint32_t f64;          // float64 stream: y[f] are double* (generic decoder only)
};

// ------------------------------------------------------------ wave64 primitives
// Cross-lane traffic uses DPP (no LDS round trip): quad_perm / row mirrors
// inside 16-lane rows, row_shr / row_bcast for scans, and v_readlane to
// combine the four rows into a wave-uniform (SGPR) result.  Callers keep all
// 64 lanes active.

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// Orders LDS accesses between the lanes of one wave, for workgroups of a
// single wave.  A wave's LDS operations execute in the order they are
// issued, so no wait is needed (a workgroup barrier would wait for every
// outstanding LDS operation); the wavefront-scope fences and the wave
// barrier only keep the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
constexpr int kQuadSwap1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowShl1 = 0x101;  // lane i receives lane i+1 of its row
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// Reduce within 16-lane rows (every lane of a row gets the row result), then
// across the four rows through readlane.
#define GPZ_WAVE_REDUCE(NAME, T, OP, TOBITS, FROMBITS)                         \
    __device__ __forceinline__ T NAME(T v) {                                   \
        v = OP(v, FROMBITS(dpp<kQuadSwap1>(TOBITS(v))));                       \
        v = OP(v, FROMBITS(dpp<kQuadSwap2>(TOBITS(v))));                       \
        v = OP(v, FROMBITS(dpp<kRowHalfMirror>(TOBITS(v))));                   \
        v = OP(v, FROMBITS(dpp<kRowMirror>(TOBITS(v))));                       \
        T r0 = FROMBITS(readlane(TOBITS(v), 0)), r1 = FROMBITS(readlane(TOBITS(v), 16)); \
        T r2 = FROMBITS(readlane(TOBITS(v), 32)), r3 = FROMBITS(readlane(TOBITS(v), 48)); \
        return OP(OP(r0, r1), OP(r2, r3));                                     \
    }

__device__ __forceinline__ uint32_t op_max(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t op_min(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t op_or(uint32_t a, uint32_t b) { return a | b; }
__device__ __forceinline__ uint32_t op_add(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ uint32_t id_u32(uint32_t v) { return v; }

GPZ_WAVE_REDUCE(wave_max_u32, uint32_t, op_max, id_u32, id_u32)
GPZ_WAVE_REDUCE(wave_min_u32, uint32_t, op_min, id_u32, id_u32)
GPZ_WAVE_REDUCE(wave_or_u32, uint32_t, op_or, id_u32, id_u32)
GPZ_WAVE_REDUCE(wave_sum_u32, uint32_t, op_add, id_u32, id_u32)
#undef GPZ_WAVE_REDUCE

// Minimum of non-NaN floats across the wave.  The float is mapped to an
// unsigned key with the same order (sign bit flipped for positive values,
// all bits flipped for negative ones), so the reduction runs on integer
// minimums, which fuse with their DPP lane moves; a float minimum would also
// quiet its operands at every step.  -0 orders below +0.
__device__ __forceinline__ float wave_min_f32(float v) {
    const uint32_t u = __float_as_uint(v);
    const uint32_t k = u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
    const uint32_t m = wave_min_u32(k);
    return __uint_as_float(m ^ (((m >> 31) - 1u) | 0x80000000u));
}

// Inclusive prefix sum across the wave (lane order).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const uint32_t lane = lane_id(), rl = lane & 15u;
    uint32_t t;
    t = dpp<kRowShr1>(v);
    v += rl >= 1 ? t : 0u;
    t = dpp<kRowShr2>(v);
    v += rl >= 2 ? t : 0u;
    t = dpp<kRowShr4>(v);
    v += rl >= 4 ? t : 0u;
    t = dpp<kRowShr8>(v);
    v += rl >= 8 ? t : 0u;
    t = dpp<kRowBcast15>(v);
    v += (lane & 16u) ? t : 0u;
    t = dpp<kRowBcast31>(v);
    v += lane >= 32 ? t : 0u;
    return v;
}

// Inclusive prefix maximum across the wave (lane order).
__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
    const uint32_t lane = lane_id(), rl = lane & 15u;
    uint32_t t;
    t = dpp<kRowShr1>(v);
    v = rl >= 1 ? max(v, t) : v;
    t = dpp<kRowShr2>(v);
    v = rl >= 2 ? max(v, t) : v;
    t = dpp<kRowShr4>(v);
    v = rl >= 4 ? max(v, t) : v;
    t = dpp<kRowShr8>(v);
    v = rl >= 8 ? max(v, t) : v;
    t = dpp<kRowBcast15>(v);
    v = (lane & 16u) ? max(v, t) : v;
    t = dpp<kRowBcast31>(v);
    v = lane >= 32 ? max(v, t) : v;
    return v;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t f2u(float f) { return __float_as_uint(f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __uint_as_float(u); }

// Exclusive scan of the per-superblock record sizes (Sec. 4.4) by one
// workgroup of T lanes (there are only ceil(nblocks / 64) superblocks):
// thread t sums a contiguous chunk, the
// chunk totals are scanned in LDS, then each thread writes its offsets.  The
// last thread publishes the stream size; when the stream fits the output
// buffer the workgroup also writes the header and the eb table.
template <uint32_t T>
__device__ __forceinline__ void scan_superblocks(const ScanArgs& a, uint64_t* part) {
    const uint32_t t = threadIdx.x;
    const uint32_t ns = a.nsuper;
    const uint32_t chunk = (ns + T - 1) / T;
    const uint32_t lo = t * chunk;
    const uint32_t hi = lo + chunk < ns ? lo + chunk : ns;
    uint64_t sum = 0;
    for (uint32_t i = lo; i < hi; i++) sum += a.supsum[i];
    part[t] = sum;
    __syncthreads();
    for (uint32_t o = 1; o < T; o <<= 1) {
        uint64_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint64_t run = part[t] - sum;
    for (uint32_t i = lo; i < hi; i++) {
        a.supoff[i] = run;
        run += a.supsum[i];
    }
    const uint64_t bytes = 4 * (a.prefix + part[T - 1]);
    if (t == T - 1) {
        *a.total_bytes = bytes;
        if (a.ext_bytes) *a.ext_bytes = bytes;
    }
    if (bytes <= a.capacity) {
        if (t == 0) {
            a.out[0] = kMagic;
            // flags: 1 float64 fields, 2 some record has a wide field
            const uint32_t wide = a.wide_flag && *a.wide_flag ? 2u : 0u;
            a.out[1] = kVersion | (((a.f64 ? 1u : 0u) | wide) << 16);
            a.out[2] = (uint32_t)(a.n & 0xFFFFFFFFu);
            a.out[3] = (uint32_t)(a.n >> 32);
            a.out[4] = a.F;
            a.out[5] = a.B;
            a.out[6] = a.K | (a.KF << 8);
            a.out[7] = a.nblocks;
        }
        uint32_t* ebt = a.out + kHeaderWords + 2 * nsuper_of(a.nblocks);
        for (uint32_t f = t; f < a.F; f += T) ebt[f] = a.eb_bits[f];
    }
}

// ------------------------------------------------------------ launchers

// single_pass: one launch that also places the records (look-back);
// otherwise records and lengths for launch_scan / launch_copy.
hipError_t launch_encode(const EncodeArgs& a, bool single_pass, hipStream_t s);
hipError_t launch_scan(const ScanArgs& a, hipStream_t s);
hipError_t launch_copy(const CopyArgs& a, hipStream_t s);
hipError_t launch_decode(const DecodeArgs& a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s);
hipError_t launch_bound_check(const float* const* orig, const float* const* recon,
                              const uint32_t* perm, uint64_t n, uint32_t F, const float* eb,
                              unsigned long long* viol, unsigned long long* maxerr_bits,
                              double* sumsq, hipStream_t s);
hipError_t launch_stream_stats(const uint32_t* in, uint64_t in_words, uint64_t n, uint32_t F,
                               uint32_t B, unsigned long long* outliers, unsigned long long* raw,
                               uint32_t* err, hipStream_t s);
hipError_t launch_field_range(const float* const* x, uint64_t n, uint32_t F, int* keys,
                              hipStream_t s);
// The same with an explicit launch shape: workgroups per CU and 16-byte
// loads in flight per lane (2, 4, 8 or 16).
hipError_t launch_field_range_shape(const float* const* x, uint64_t n, uint32_t F, int* keys,
                                    uint32_t groups_per_cu, uint32_t unroll, hipStream_t s);
// Generic 256-lane-per-block kernels (float64 fields, fields needing 64-bit
// grid steps, any block size).  deferred_only: the blocks the wave-per-block
// encoder left on its list; otherwise every block.  The decoder takes every
// block (the wave-per-block decoder decodes records with a wide field
// itself).
hipError_t launch_encode_generic(const EncodeArgs& a, bool deferred_only, hipStream_t s);
// The deferred blocks, then the length scan in the same launch (the last
// workgroup to finish its share scans; *done is zero before the launch).
hipError_t launch_encode_deferred_then_scan(const EncodeArgs& a, const ScanArgs& sa,
                                            uint32_t* done, hipStream_t s);
hipError_t launch_decode_generic(const DecodeArgs& a, hipStream_t s);
// The range keys as floats in device memory (min, max per field).
hipError_t launch_range_to_floats(const int* keys, uint32_t F, float* out, hipStream_t s);
// Compute units of the current device (queried once per device, 256 if the
// query fails).
uint32_t device_cu_count();

// ------------------------------------------------------------ batched form
// Many snapshots in one launch per stage.  Job tables live in device memory;
// block g of the flattened list belongs to the job j with
// prefix[j] <= g < prefix[j+1] (found by a uniform binary search).

// g must be wave-uniform; the result is returned through readfirstlane so
// the compiler keeps it (and the job arguments it indexes) in scalar registers.
__device__ __forceinline__ uint32_t find_job(const uint32_t* __restrict__ prefix, uint32_t njobs,
                                             uint32_t g) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
}

// Launch descriptor of a batch, kept in device memory so that a captured
// graph stays valid when the job table is rebound (counts change, pointers
// and launch shapes do not).
struct BatchLaunch {
    uint32_t njobs;
    uint32_t total_full;    // full blocks over all jobs
    uint32_t total_blocks;  // all blocks over all jobs
    uint32_t ntail;         // jobs whose last block is partial
    uint32_t tile;          // consecutive blocks taken per work-queue grab
    const uint32_t* full_prefix;   // njobs + 1
    const uint32_t* block_prefix;  // njobs + 1
    const uint32_t* tail_jobs;     // ntail job indices
    uint32_t* counter;             // [0] encode queue head, [1] decode queue head
};

// Launch shapes of the batched kernels (fixed for the life of a batch).
struct BatchShape {
    uint32_t B;
    uint32_t grid;        // persistent encode / decode workgroups (one wave each);
                          // 0: one workgroup per block instead (direct_grid of them)
    uint32_t direct_grid; // block capacity of the batch (direct launches)
    uint32_t scan_grid;   // workgroups striding over jobs for the scans
    uint32_t copy_grid;   // 4-wave workgroups striding over blocks for the copies
    uint32_t tail_grid;   // workgroups striding over the partial tail blocks
};

hipError_t launch_encode_batch(const EncodeArgs* jobs, const BatchLaunch* L, const BatchShape& S,
                               hipStream_t s);
hipError_t launch_scan_batch(const ScanArgs* jobs, const BatchLaunch* L, const BatchShape& S,
                             hipStream_t s);
hipError_t launch_copy_batch(const CopyArgs* jobs, const BatchLaunch* L, const BatchShape& S,
                             hipStream_t s);
// Batched form of the deferred-block encoder: a fixed grid that walks every
// job's list (max_blocks: the batch's block capacity).
hipError_t launch_encode_generic_batch(const EncodeArgs* jobs, const BatchLaunch* L, uint32_t B,
                                       uint32_t max_blocks, hipStream_t s);
hipError_t launch_decode_batch(const DecodeArgs* jobs, const BatchLaunch* L,
                               const BatchShape& S, hipStream_t s);

}  // namespace gpz
