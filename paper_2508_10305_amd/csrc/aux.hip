// Compaction (Sec. 4.4, steps two and three): a device-level exclusive scan
// of the block record lengths, then a copy of every record to its final
// offset together with the stream header and tables.  Also: a fill kernel
// (used instead of hipMemset so the sequence stays graph-capturable), the
// error-bound check and the per-field range reduction.
#include "gpz_internal.h"

namespace gpz {
namespace {

constexpr uint32_t kScanThreads = 1024;

// Exclusive scan of the per-superblock record sizes (one workgroup; there
// are only ceil(nblocks / 64) of them): thread t sums a contiguous chunk, the
// chunk totals are scanned in LDS, then each thread writes its offsets.  The
// last thread publishes the stream size; when the stream fits the output
// buffer the workgroup also writes the header and the eb table.
__device__ __forceinline__ void scan_body(const ScanArgs& a, uint64_t* part) {
    const uint32_t t = threadIdx.x;
    const uint32_t ns = a.nsuper;
    const uint32_t chunk = (ns + kScanThreads - 1) / kScanThreads;
    const uint32_t lo = t * chunk;
    const uint32_t hi = lo + chunk < ns ? lo + chunk : ns;
    uint64_t sum = 0;
    for (uint32_t i = lo; i < hi; i++) sum += a.supsum[i];
    part[t] = sum;
    __syncthreads();
    for (uint32_t o = 1; o < kScanThreads; o <<= 1) {
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
    const uint64_t bytes = 4 * (a.prefix + part[kScanThreads - 1]);
    if (t == kScanThreads - 1) {
        *a.total_bytes = bytes;
        if (a.ext_bytes) *a.ext_bytes = bytes;
    }
    if (bytes <= a.capacity) {
        if (t == 0) {
            a.out[0] = kMagic;
            a.out[1] = kVersion;
            a.out[2] = (uint32_t)(a.n & 0xFFFFFFFFu);
            a.out[3] = (uint32_t)(a.n >> 32);
            a.out[4] = a.F;
            a.out[5] = a.B;
            a.out[6] = a.K | (a.KF << 8);
            a.out[7] = a.nblocks;
        }
        uint32_t* ebt = a.out + kHeaderWords + 2 * nsuper_of(a.nblocks);
        for (uint32_t f = t; f < a.F; f += kScanThreads) ebt[f] = a.eb_bits[f];
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_lengths(ScanArgs a) {
    __shared__ uint64_t part[kScanThreads];
    scan_body(a, part);
}

__global__ __launch_bounds__(kScanThreads) void scan_lengths_batch(const ScanArgs* jobs,
                                                                    const BatchLaunch* L) {
    __shared__ uint64_t part[kScanThreads];
    const uint32_t njobs = L->njobs;
    for (uint32_t j = blockIdx.x; j < njobs; j += gridDim.x) {
        scan_body(jobs[j], part);
        __syncthreads();
    }
}

// One wave per block record: copy it from its slot to its final offset
// (superblock offset + lengths of the earlier blocks of the superblock), and
// write its length-table entry (and the superblock entry every 64 blocks).
// Nothing is written when the stream does not fit the output buffer.
__device__ __forceinline__ void copy_body(const CopyArgs& a, uint32_t b, uint32_t lane) {
    const uint64_t total = *a.total_bytes;
    if (total > a.capacity) return;
    const uint64_t nsup = nsuper_of(a.nblocks);
    uint32_t* sup = a.out + kHeaderWords;
    uint32_t* lt = sup + 2 * nsup + a.F;
    uint32_t* recs = lt + a.nblocks;
    const uint32_t sb = b / kSuper, first = sb * kSuper;
    const uint32_t before = wave_sum_u32(first + lane < b ? a.lens[first + lane] : 0u);
    const uint32_t len = a.lens[b];
    const uint64_t off = a.supoff[sb] + before;
    if (lane == 0) {
        lt[b] = len;
        if (b % kSuper == 0) {
            sup[2 * sb] = (uint32_t)(off & 0xFFFFFFFFu);
            sup[2 * sb + 1] = (uint32_t)(off >> 32);
        }
    }
    const uint32_t* src = a.temp + (uint64_t)b * a.slot_words;
    uint32_t* dst = recs + off;
    for (uint32_t k = lane; k < len; k += 64) dst[k] = src[k];
}

__global__ __launch_bounds__(256) void copy_records(CopyArgs a) {
    const uint32_t b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= a.nblocks) return;
    copy_body(a, b, threadIdx.x & 63u);
}

__global__ __launch_bounds__(256) void copy_records_batch(const CopyArgs* jobs,
                                                          const BatchLaunch* L) {
    const uint32_t total = L->total_blocks, njobs = L->njobs;
    const uint32_t* prefix = L->block_prefix;
    for (uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6); g < total; g += gridDim.x * 4) {
        const uint32_t j = find_job(prefix, njobs, g);
        copy_body(jobs[j], g - prefix[j], threadIdx.x & 63u);
    }
}

__global__ void fill_u32(uint32_t* p, uint32_t value, uint64_t count) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

struct BoundArgs {
    const float* orig[kMaxFields];
    const float* recon[kMaxFields];
    float eb[kMaxFields];
    const uint32_t* perm;
    uint64_t n;
    unsigned long long* viol;
    unsigned long long* maxerr_bits;
};

// Grid-stride over positions, field = blockIdx.y.  A pair passes when its
// bits match or |recon - orig| <= eb in double.
__global__ __launch_bounds__(256) void bound_check_kernel(BoundArgs a) {
    __shared__ unsigned long long sv[4], sm[4];
    const uint32_t f = blockIdx.y;
    const float* x = a.orig[f];
    const float* y = a.recon[f];
    const double eb = (double)a.eb[f];
    unsigned long long v = 0;
    double m = 0.0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n;
         j += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t src = a.perm ? a.perm[j] : j;
        if (src >= a.n) {  // not a permutation of [0, n): count, do not read
            v++;
            continue;
        }
        float xo = x[src];
        float yr = y[j];
        double d = __builtin_fabs((double)yr - (double)xo);
        if (!__builtin_isnan(d) && d > m) m = d;
        if (f2u(xo) != f2u(yr) && !(d <= eb)) v++;
    }
    unsigned long long mb = (unsigned long long)__double_as_longlong(m);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_xor(v, o);
        mb = max(mb, (unsigned long long)__shfl_xor(mb, o));
    }
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) {
        sv[w] = v;
        sm[w] = mb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tv = 0, tm = 0;
        for (int i = 0; i < 4; i++) {
            tv += sv[i];
            tm = max(tm, sm[i]);
        }
        if (tv) atomicAdd(&a.viol[f], tv);
        atomicMax(&a.maxerr_bits[f], tm);
    }
}

struct RangeArgs {
    const float* x[kMaxFields];
    uint64_t n;
    uint32_t F;
    int* keys;  // order-preserving integer keys: [0, F) minima, [F, 2F) maxima
};

// Order-preserving map of float bits to signed integers (-0 < +0).
__device__ __forceinline__ int order_key(float v) {
    int i = __float_as_int(v);
    return i ^ ((i >> 31) & 0x7FFFFFFF);
}

__global__ __launch_bounds__(256) void field_range_kernel(RangeArgs a) {
    __shared__ int smin[4], smax[4];
    const uint32_t f = blockIdx.y;
    const float* x = a.x[f];
    int mn = 0x7FFFFFFF, mx = (int)0x80000000;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n;
         j += (uint64_t)gridDim.x * blockDim.x) {
        float v = x[j];
        if (__builtin_isfinite(v)) {
            int k = order_key(v);
            mn = min(mn, k);
            mx = max(mx, k);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o));
        mx = max(mx, __shfl_xor(mx, o));
    }
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) {
        smin[w] = mn;
        smax[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; i++) {
            mn = min(mn, smin[i]);
            mx = max(mx, smax[i]);
        }
        atomicMin(&a.keys[f], mn);
        atomicMax(&a.keys[a.F + f], mx);
    }
}

}  // namespace

hipError_t launch_scan(const ScanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(scan_lengths, dim3(1), dim3(kScanThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy(const CopyArgs& a, hipStream_t s) {
    if (a.nblocks == 0) return hipSuccess;
    const uint32_t groups = (a.nblocks + 3) / 4;
    hipLaunchKernelGGL(copy_records, dim3(groups), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scan_batch(const ScanArgs* jobs, const BatchLaunch* L, const BatchShape& S,
                             hipStream_t s) {
    hipLaunchKernelGGL(scan_lengths_batch, dim3(S.scan_grid), dim3(kScanThreads), 0, s, jobs, L);
    return hipGetLastError();
}

hipError_t launch_copy_batch(const CopyArgs* jobs, const BatchLaunch* L, const BatchShape& S,
                             hipStream_t s) {
    hipLaunchKernelGGL(copy_records_batch, dim3(S.copy_grid), dim3(256), 0, s, jobs, L);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_bound_check(const float* const* orig, const float* const* recon,
                              const uint32_t* perm, uint64_t n, uint32_t F, const float* eb,
                              unsigned long long* viol, unsigned long long* maxerr_bits,
                              hipStream_t s) {
    BoundArgs a{};
    for (uint32_t f = 0; f < F; f++) {
        a.orig[f] = orig[f];
        a.recon[f] = recon[f];
        a.eb[f] = eb[f];
    }
    a.perm = perm;
    a.n = n;
    a.viol = viol;
    a.maxerr_bits = maxerr_bits;
    uint64_t groups = (n + 255) / 256;
    if (groups > 4096) groups = 4096;
    if (groups == 0) groups = 1;
    hipLaunchKernelGGL(bound_check_kernel, dim3((uint32_t)groups, F), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_field_range(const float* const* x, uint64_t n, uint32_t F, int* keys,
                              hipStream_t s) {
    RangeArgs a{};
    for (uint32_t f = 0; f < F; f++) a.x[f] = x[f];
    a.n = n;
    a.F = F;
    a.keys = keys;
    uint64_t groups = (n + 255) / 256;
    if (groups > 4096) groups = 4096;
    if (groups == 0) groups = 1;
    hipLaunchKernelGGL(field_range_kernel, dim3((uint32_t)groups, F), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gpz
