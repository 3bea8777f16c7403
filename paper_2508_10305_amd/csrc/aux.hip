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
    // 16 loads in flight per lane (4 KB per wave) before the stores; whole
    // 1024-word steps run without per-word predicates, at 32-bit offsets
    // from the scalar bases, and only the last step is predicated.
    constexpr int U = 16;
    const uint8_t* sb8 = reinterpret_cast<const uint8_t*>(src);
    uint8_t* db8 = reinterpret_cast<uint8_t*>(dst);
    const uint32_t whole = len & ~(64u * U - 1u);
    for (uint32_t k0 = 0; k0 < whole; k0 += 64 * U) {
        uint32_t v[U];
#pragma unroll
        for (int i = 0; i < U; i++)
            v[i] = __builtin_nontemporal_load(
                reinterpret_cast<const uint32_t*>(sb8 + 4u * (k0 + 64u * i + lane)));
#pragma unroll
        for (int i = 0; i < U; i++)
            *reinterpret_cast<uint32_t*>(db8 + 4u * (k0 + 64u * i + lane)) = v[i];
    }
    if (whole < len) {
        uint32_t v[U];
#pragma unroll
        for (int i = 0; i < U; i++) {
            const uint32_t k = whole + 64 * i + lane;
            v[i] = k < len ? __builtin_nontemporal_load(src + k) : 0u;
        }
#pragma unroll
        for (int i = 0; i < U; i++) {
            const uint32_t k = whole + 64 * i + lane;
            if (k < len) dst[k] = v[i];
        }
    }
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
    uint32_t F;
    unsigned long long* viol;
    unsigned long long* maxerr_bits;
    double* sumsq;  // nullable: sum of squared differences per field
};

constexpr uint32_t kCheckChunk = 1024;  // positions per workgroup step

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    return v;
}

// Error-bound verification.  A 256-lane workgroup takes chunks of 1024
// positions (lane t: positions 4t..4t+3), reads the permutation once per
// chunk for all fields, the reconstructed values contiguously and the
// originals by gather -- block-local for GPZ permutations, so each chunk's
// originals come from one 4 KB window per field.  A pair passes when its bits
// match or |recon - orig| <= eb in double; a permutation entry >= n counts
// as a violation and is not read.  Per-field counts and maxima gather in LDS
// (one slot per wave) and leave with one atomic per field per workgroup.
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void bound_check_kernel(BoundArgs a) {
    __shared__ unsigned long long sv[4][kMaxFields], sm[4][kMaxFields];
    __shared__ double ss[4][kMaxFields];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < 4 * kMaxFields; i += 256) {
        (&sv[0][0])[i] = 0;
        (&sm[0][0])[i] = 0;
        (&ss[0][0])[i] = 0.0;
    }
    __syncthreads();
    const uint64_t nchunks = (a.n + kCheckChunk - 1) / kCheckChunk;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t j0 = c * kCheckChunk + 4 * threadIdx.x;
        uint32_t src[4];
        bool in[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            in[i] = j0 + i < a.n;
            src[i] = in[i] ? (a.perm ? a.perm[j0 + i] : (uint32_t)(j0 + i)) : 0u;
        }
        for (uint32_t f = 0; f < a.F; f++) {
            const float* x = a.orig[f];
            const float* y = a.recon[f];
            const double eb = (double)a.eb[f];
            float yr[4], xo[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                yr[i] = in[i] ? y[j0 + i] : 0.0f;
                xo[i] = in[i] && src[i] < a.n ? x[src[i]] : 0.0f;
            }
            unsigned long long v = 0;
            double m = 0.0, q = 0.0;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                if (!in[i]) continue;
                if (src[i] >= a.n) {  // not a permutation of [0, n)
                    v++;
                    continue;
                }
                const double d = __builtin_fabs((double)yr[i] - (double)xo[i]);
                if (!__builtin_isnan(d)) {
                    if (d > m) m = d;
                    q += d * d;
                }
                if (f2u(xo[i]) != f2u(yr[i]) && !(d <= eb)) v++;
            }
            v = wave_sum_u64(v);
            const unsigned long long mb =
                wave_max_u64((unsigned long long)__double_as_longlong(m));
            if (a.sumsq) q = wave_sum_f64(q);
            if (lane == 0) {
                sv[w][f] += v;
                if (mb > sm[w][f]) sm[w][f] = mb;
                ss[w][f] += q;
            }
        }
    }
    __syncthreads();
    for (uint32_t f = threadIdx.x; f < a.F; f += 256) {
        unsigned long long tv = 0, tm = 0;
        for (int i = 0; i < 4; i++) {
            tv += sv[i][f];
            tm = sm[i][f] > tm ? sm[i][f] : tm;
        }
        if (tv) atomicAdd(&a.viol[f], tv);
        if (tm) atomicMax(&a.maxerr_bits[f], tm);
        if (a.sumsq) {
            const double tq = ss[0][f] + ss[1][f] + ss[2][f] + ss[3][f];
            if (tq != 0.0) atomicAdd(&a.sumsq[f], tq);
        }
    }
}

// Structure statistics of a stream: outliers per field (coded blocks) and
// raw blocks.  One lane per block: the record offset comes from the
// superblock table plus the lengths before the block in its superblock; the
// lane walks the record's array headers.  Malformed structure sets *err.
struct StatsArgs {
    const uint32_t* in;
    uint64_t in_words;
    uint64_t n;
    uint32_t F, B, nblocks;
    uint64_t prefix;
    unsigned long long* outliers;  // F
    unsigned long long* raw;
    uint32_t* err;
};

__global__ __launch_bounds__(256) void stream_stats_kernel(StatsArgs a) {
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    const bool live = b < a.nblocks;
    const uint64_t nsup = nsuper_of(a.nblocks);
    const uint32_t* sup = a.in + kHeaderWords;
    const uint32_t* lt = sup + 2 * nsup + a.F;
    const uint64_t rec_total = a.in_words - a.prefix;
    bool bad = false, raw = false;
    uint64_t off = 0, pos = 0;
    uint32_t len = 0, nn = 0;
    const uint32_t* rec = a.in + a.prefix;
    if (live) {
        // superblock entry checked before use, lengths summed in 64 bits (at
        // most 63 of them): no sum wraps, an accepted record lies inside the
        // record area
        const uint32_t sb = b / kSuper;
        const uint64_t sup_off = (uint64_t)sup[2 * sb] | ((uint64_t)sup[2 * sb + 1] << 32);
        off = sup_off;
        for (uint32_t k = sb * kSuper; k < b; k++) off += lt[k];
        len = lt[b];
        nn = (uint32_t)((uint64_t)(b + 1) * a.B <= a.n ? a.B : a.n - (uint64_t)b * a.B);
        bad = len < 1 || sup_off > rec_total || off > rec_total || (uint64_t)len > rec_total - off;
        if (!bad) {
            rec += off;
            raw = (rec[0] & 3u) == 1u;
            if (raw) {
                bad = len != 1 + a.F * nn;
            } else {
                bad = len < 2;
                if (!bad) {
                    const uint32_t U = rec[0] >> 2, h1 = rec[1];
                    pos = 2 + (uint64_t)words_for(U, h1 & 31u) + words_for(U, (h1 >> 5) & 31u);
                }
            }
        }
    }
    const bool walk = live && !bad && !raw;
    for (uint32_t f = 0; f < a.F; f++) {
        uint32_t nout = 0;
        if (walk && !bad) {
            if (pos + 2 > len) {
                bad = true;
            } else {
                const uint32_t wn = rec[pos + 1];
                nout = wn >> 5;
                pos += 2 + (uint64_t)words_for(nn, wn & 31u) + 2 * (uint64_t)nout;
            }
        }
        const uint32_t tot = wave_sum_u32(nout);
        if ((threadIdx.x & 63u) == 0 && tot) atomicAdd(&a.outliers[f], (unsigned long long)tot);
    }
    if (walk && !bad && pos != len) bad = true;
    const uint32_t nraw = wave_sum_u32(live && !bad && raw ? 1u : 0u);
    if ((threadIdx.x & 63u) == 0 && nraw) atomicAdd(a.raw, (unsigned long long)nraw);
    if (live && bad) *a.err = 1u;
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

__device__ __forceinline__ void range_take(float v, int& mn, int& mx) {
    if (__builtin_isfinite(v)) {
        const int k = order_key(v);
        mn = min(mn, k);
        mx = max(mx, k);
    }
}

// Field range over finite values, field = blockIdx.y: grid-stride over
// 16-byte vectors, four of them in flight per lane; the unaligned head and
// the tail are done element by element by workgroup 0.
__global__ __launch_bounds__(256) void field_range_kernel(RangeArgs a) {
    __shared__ int smin[4], smax[4];
    const uint32_t f = blockIdx.y;
    const float* x = a.x[f];
    int mn = 0x7FFFFFFF, mx = (int)0x80000000;
    // elements before the first 16-byte boundary
    const uint64_t head = ((16u - (reinterpret_cast<uintptr_t>(x) & 15u)) & 15u) / 4u;
    const uint64_t h = head < a.n ? head : a.n;
    const uint64_t nv = (a.n - h) / 4;  // whole vectors
    const f32x4* xv = reinterpret_cast<const f32x4*>(x + h);
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < nv; i += 4 * stride) {
        f32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; k++) v[k] = __builtin_nontemporal_load(xv + i + k * stride);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            range_take(v[k].x, mn, mx);
            range_take(v[k].y, mn, mx);
            range_take(v[k].z, mn, mx);
            range_take(v[k].w, mn, mx);
        }
    }
    for (; i < nv; i += stride) {
        const f32x4 v = __builtin_nontemporal_load(xv + i);
        range_take(v.x, mn, mx);
        range_take(v.y, mn, mx);
        range_take(v.z, mn, mx);
        range_take(v.w, mn, mx);
    }
    if (blockIdx.x == 0) {
        for (uint64_t j = threadIdx.x; j < h; j += 256) range_take(x[j], mn, mx);
        for (uint64_t j = h + 4 * nv + threadIdx.x; j < a.n; j += 256) range_take(x[j], mn, mx);
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
        for (int k = 1; k < 4; k++) {
            mn = min(mn, smin[k]);
            mx = max(mx, smax[k]);
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

hipError_t launch_stream_stats(const uint32_t* in, uint64_t in_words, uint64_t n, uint32_t F,
                               uint32_t B, unsigned long long* outliers, unsigned long long* raw,
                               uint32_t* err, hipStream_t s) {
    StatsArgs a{};
    a.in = in;
    a.in_words = in_words;
    a.n = n;
    a.F = F;
    a.B = B;
    a.nblocks = (uint32_t)nblocks_of(n, B);
    a.prefix = prefix_words(n, F, B);
    a.outliers = outliers;
    a.raw = raw;
    a.err = err;
    if (a.nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(stream_stats_kernel, dim3((a.nblocks + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bound_check(const float* const* orig, const float* const* recon,
                              const uint32_t* perm, uint64_t n, uint32_t F, const float* eb,
                              unsigned long long* viol, unsigned long long* maxerr_bits,
                              double* sumsq, hipStream_t s) {
    BoundArgs a{};
    for (uint32_t f = 0; f < F; f++) {
        a.orig[f] = orig[f];
        a.recon[f] = recon[f];
        a.eb[f] = eb[f];
    }
    a.perm = perm;
    a.n = n;
    a.F = F;
    a.viol = viol;
    a.maxerr_bits = maxerr_bits;
    a.sumsq = sumsq;
    uint64_t groups = (n + kCheckChunk - 1) / kCheckChunk;
    if (groups > 8192) groups = 8192;
    if (groups == 0) groups = 1;
    hipLaunchKernelGGL(bound_check_kernel, dim3((uint32_t)groups), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_field_range(const float* const* x, uint64_t n, uint32_t F, int* keys,
                              hipStream_t s) {
    RangeArgs a{};
    for (uint32_t f = 0; f < F; f++) a.x[f] = x[f];
    a.n = n;
    a.F = F;
    a.keys = keys;
    // about two 4-vector sweeps per lane at full size; at least one workgroup
    uint64_t groups = (n / 4 + 4095) / 4096;
    if (groups > 2048) groups = 2048;
    if (groups == 0) groups = 1;
    hipLaunchKernelGGL(field_range_kernel, dim3((uint32_t)groups, F), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gpz
