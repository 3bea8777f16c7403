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
    const float* x[kMaxFields];
    float eb[kMaxFields];
    float twoeb[kMaxFields];
    float inv[kMaxFields];
    uint64_t n;
    uint32_t F, K, KF, B;
    uint32_t nblocks;
    uint32_t slot_words;  // record slot stride in the workspace (>= 1 + F*B)
    uint32_t* temp;       // nblocks record slots
    uint32_t* lens;       // record length (words) per block
    uint32_t* perm;       // nullable: n global input indices
};

struct ScanArgs {
    const uint32_t* lens;
    uint64_t* offs;        // exclusive prefix of lens (words, inside the record area)
    uint64_t* total_bytes; // whole stream size in bytes
    uint64_t* ext_bytes;   // nullable second destination of the size (async API)
    uint32_t nblocks;
    uint64_t prefix;       // words before the record area
};

struct CopyArgs {
    const uint32_t* temp;
    const uint32_t* lens;
    const uint64_t* offs;
    const uint64_t* total_bytes;
    uint32_t* out;
    uint64_t capacity;     // bytes
    uint32_t slot_words;
    uint32_t nblocks;
    uint64_t n;
    uint32_t F, B, K, KF;
    uint32_t eb_bits[kMaxFields];
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
};

// ------------------------------------------------------------ wave64 primitives

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= (uint32_t)__shfl_xor((int)v, o);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
    return v;
}

__device__ __forceinline__ float wave_min_f32(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}

// Inclusive prefix sum across the wave (lane order).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)v, o);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Inclusive prefix maximum across the wave (lane order).
__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)v, o);
        if (lane >= (uint32_t)o) v = max(v, t);
    }
    return v;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t f2u(float f) { return __float_as_uint(f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __uint_as_float(u); }

// ------------------------------------------------------------ launchers

hipError_t launch_encode(const EncodeArgs& a, hipStream_t s);
hipError_t launch_scan(const ScanArgs& a, hipStream_t s);
hipError_t launch_copy(const CopyArgs& a, hipStream_t s);
hipError_t launch_decode(const DecodeArgs& a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s);
hipError_t launch_bound_check(const float* const* orig, const float* const* recon,
                              const uint32_t* perm, uint64_t n, uint32_t F, const float* eb,
                              unsigned long long* viol, unsigned long long* maxerr_bits,
                              hipStream_t s);
hipError_t launch_field_range(const float* const* x, uint64_t n, uint32_t F, int* keys,
                              hipStream_t s);

}  // namespace gpz
