// Compaction (Sec. 4.4, steps two and three): a device-level exclusive scan
// of the block record lengths, then a copy of every record to its final
// offset together with the stream header and tables.  Also: a fill kernel
// (used instead of hipMemset so the sequence stays graph-capturable), the
// error-bound check and the per-field range reduction.
#include <atomic>

#include "gpz_internal.h"

namespace gpz {
namespace {

constexpr uint32_t kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void scan_lengths(ScanArgs a) {
    __shared__ uint64_t part[kScanThreads];
    scan_superblocks<kScanThreads>(a, part);
}

__global__ __launch_bounds__(kScanThreads) void scan_lengths_batch(const ScanArgs* jobs,
                                                                    const BatchLaunch* L) {
    __shared__ uint64_t part[kScanThreads];
    const uint32_t njobs = L->njobs;
    for (uint32_t j = blockIdx.x; j < njobs; j += gridDim.x) {
        scan_superblocks<kScanThreads>(jobs[j], part);
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

// Direct form: one wave per block of the batch's capacity (4 per
// workgroup), as the plain copy; waves past the bound jobs' blocks exit.
__global__ __launch_bounds__(256) void copy_records_batch_direct(const CopyArgs* jobs,
                                                                 const BatchLaunch* L) {
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= L->total_blocks) return;
    const uint32_t* prefix = L->block_prefix;
    const uint32_t j = find_job(prefix, L->njobs, g);
    copy_body(jobs[j], g - prefix[j], threadIdx.x & 63u);
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
    const uint32_t vw = (a.in[1] >> 16) & 1u ? 2u : 1u;  // words per value (float64 stream: 2)
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
                bad = len != 1 + a.F * nn * vw;
            } else {
                bad = len < 2;
                if (!bad) {
                    const uint32_t U = (rec[0] & 0x7FFFFFFFu) >> 2, h1 = rec[1];
                    pos = 2 + (uint64_t)words_for(U, h1 & 31u) + words_for(U, (h1 >> 5) & 31u);
                }
            }
        }
    }
    const bool walk = live && !bad && !raw;
    for (uint32_t f = 0; f < a.F; f++) {
        uint32_t nout = 0;
        if (walk && !bad) {
            if (pos + vw + 1 > len) {
                bad = true;
            } else {
                // field word: w | nout << 5, or w | nout << 6 | 1 << 31 (wide)
                const uint32_t wn = rec[pos + vw];
                const bool wide = (wn >> 31) != 0;
                const uint32_t w = wide ? (wn & 63u) : (wn & 31u);
                nout = wide ? ((wn >> 6) & 0x1FFFFFFu) : ((wn >> 5) & 0x3FFFFFFu);
                pos += vw + 1 + (uint64_t)words_for(nn, w) + (uint64_t)(1 + vw) * nout;
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
    uint64_t cpf;  // chunks per field: ceil((n / 4) / (U * 256))
    int* keys;     // order-preserving integer keys: [0, F) minima, [F, 2F) maxima
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

__device__ __forceinline__ void range_take4(const f32x4& v, int& mn, int& mx) {
    range_take(v.x, mn, mx);
    range_take(v.y, mn, mx);
    range_take(v.z, mn, mx);
    range_take(v.w, mn, mx);
}

// Workgroup minimum / maximum of the keys, then one atomic pair per
// workgroup (atomics of many waves on the same few words serialize).  Every
// lane calls it (a change of field is workgroup-uniform).
__device__ __forceinline__ void range_flush(const RangeArgs& a, uint32_t f, int mn, int mx,
                                            int* smin, int* smax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o));
        mx = max(mx, __shfl_xor(mx, o));
    }
    if ((threadIdx.x & 63u) == 0) {
        smin[threadIdx.x >> 6] = mn;
        smax[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; k++) {
            mn = min(mn, smin[k]);
            mx = max(mx, smax[k]);
        }
        if (mn != 0x7FFFFFFF) atomicMin(&a.keys[f], mn);
        if (mx != (int)0x80000000) atomicMax(&a.keys[a.F + f], mx);
    }
    __syncthreads();
}

// Chunk c of the flattened (field, chunk) space: its field, the 16-byte
// vectors of that field past its unaligned head, and the chunk's first vector.
struct RangeChunk {
    uint32_t f;
    const f32x4* xv;
    uint64_t nv, v0;
};

__device__ __forceinline__ RangeChunk range_chunk(const RangeArgs& a, uint64_t c, uint64_t chunk) {
    RangeChunk r;
    r.f = (uint32_t)(c / a.cpf);
    const float* x = a.x[r.f];
    const uint64_t head = ((16u - (reinterpret_cast<uintptr_t>(x) & 15u)) & 15u) / 4u;
    const uint64_t h = head < a.n ? head : a.n;
    r.nv = (a.n - h) / 4;
    r.xv = reinterpret_cast<const f32x4*>(x + h);
    r.v0 = (c - (uint64_t)r.f * a.cpf) * chunk;
    return r;
}

template <int U>
__device__ __forceinline__ void range_load(const RangeChunk& r, uint64_t chunk, f32x4 (&v)[U]) {
    const uint64_t i0 = r.v0 + threadIdx.x;
    if (r.v0 + chunk <= r.nv) {
#pragma unroll
        for (int k = 0; k < U; k++) v[k] = __builtin_nontemporal_load(r.xv + i0 + 256 * k);
    } else {
        const f32x4 nan4 = {__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""),
                            __builtin_nanf("")};
#pragma unroll
        for (int k = 0; k < U; k++)
            v[k] = i0 + 256 * k < r.nv ? __builtin_nontemporal_load(r.xv + i0 + 256 * k) : nan4;
    }
}

// Field range over finite values.  The 16-byte vectors of every field are cut
// into chunks of U * 256 vectors (chunk c belongs to field c / cpf);
// workgroup g takes chunks g, g + gridDim.x, ...  The loads of the next chunk
// are issued before the current one is reduced (two register buffers), so
// the memory stays busy while a wave computes.  Positions past a field's
// last whole vector load as NaN, which the finite test skips.  Every wave
// follows the same chunk sequence, so a change of field is
// workgroup-uniform: the running extrema are then folded into the field's
// keys.  The elements before a field's first 16-byte boundary and after its
// last whole vector (at most 3 + 3) are taken by workgroup 0, each lane
// with its own atomics.
template <int U>
__global__ __launch_bounds__(256) void field_range_kernel(RangeArgs a) {
    __shared__ int smin[4], smax[4];
    const uint64_t chunk = (uint64_t)U * 256;
    const uint64_t total = a.cpf * a.F;
    int mn = 0x7FFFFFFF, mx = (int)0x80000000;
    uint64_t c = blockIdx.x;
    if (c < total) {
        uint32_t cur = 0xFFFFFFFFu;
        RangeChunk r = range_chunk(a, c, chunk);
        f32x4 v[U];
        range_load<U>(r, chunk, v);
        for (;;) {
            const uint64_t cn = c + gridDim.x;
            RangeChunk rn = r;
            f32x4 w[U];
            if (cn < total) {
                rn = range_chunk(a, cn, chunk);
                range_load<U>(rn, chunk, w);
            }
            if (r.f != cur) {
                if (cur != 0xFFFFFFFFu) range_flush(a, cur, mn, mx, smin, smax);
                mn = 0x7FFFFFFF;
                mx = (int)0x80000000;
                cur = r.f;
            }
#pragma unroll
            for (int k = 0; k < U; k++) range_take4(v[k], mn, mx);
            if (cn >= total) break;
            c = cn;
            r = rn;
#pragma unroll
            for (int k = 0; k < U; k++) v[k] = w[k];
        }
        range_flush(a, cur, mn, mx, smin, smax);
    }
    if (blockIdx.x == 0) {
        // thread t < 8F: slot t % 8 of field t / 8 (slots 0-3 the head, 4-7 the tail)
        for (uint32_t t = threadIdx.x; t < 8u * a.F; t += 256) {
            const uint32_t f = t >> 3, j = t & 7u;
            const float* xf = a.x[f];
            const uint64_t head = ((16u - (reinterpret_cast<uintptr_t>(xf) & 15u)) & 15u) / 4u;
            const uint64_t h = head < a.n ? head : a.n;
            const uint64_t tail0 = h + 4 * ((a.n - h) / 4);
            const uint64_t i = j < 4 ? (uint64_t)j : tail0 + (j - 4);
            const bool live = j < 4 ? i < h : i < a.n;
            if (live && __builtin_isfinite(xf[i])) {
                const int k = order_key(xf[i]);
                atomicMin(&a.keys[f], k);
                atomicMax(&a.keys[a.F + f], k);
            }
        }
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
    if (S.grid)
        hipLaunchKernelGGL(copy_records_batch, dim3(S.copy_grid), dim3(256), 0, s, jobs, L);
    else
        hipLaunchKernelGGL(copy_records_batch_direct, dim3((S.direct_grid + 3) / 4), dim3(256), 0,
                           s, jobs, L);
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

namespace {

// The 2F range keys as floats in out[2F] (min, max per field): 0, 0 for a
// field with no finite value, a zero extreme as +0.0.
__global__ __launch_bounds__(64) void range_keys_to_floats(const int* __restrict__ keys, uint32_t F,
                                                           float* __restrict__ out) {
    for (uint32_t f = threadIdx.x; f < F; f += 64) {
        const int mn = keys[f], mx = keys[F + f];
        float lo = 0.0f, hi = 0.0f;
        if (mn <= mx) {
            lo = __int_as_float(mn ^ ((mn >> 31) & 0x7FFFFFFF));
            hi = __int_as_float(mx ^ ((mx >> 31) & 0x7FFFFFFF));
            if (lo == 0.0f) lo = 0.0f;
            if (hi == 0.0f) hi = 0.0f;
        }
        out[2 * f] = lo;
        out[2 * f + 1] = hi;
    }
}

}  // namespace

hipError_t launch_range_to_floats(const int* keys, uint32_t F, float* out, hipStream_t s) {
    hipLaunchKernelGGL(range_keys_to_floats, dim3(1), dim3(64), 0, s, keys, F, out);
    return hipGetLastError();
}

uint32_t device_cu_count() {
    constexpr int kDevices = 64;
    static std::atomic<int> cached[kDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) return 256;
    int c = cached[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            c = 256;
        cached[dev].store(c, std::memory_order_relaxed);
    }
    return (uint32_t)c;
}

hipError_t launch_field_range_shape(const float* const* x, uint64_t n, uint32_t F, int* keys,
                                    uint32_t groups_per_cu, uint32_t unroll, hipStream_t s) {
    RangeArgs a{};
    for (uint32_t f = 0; f < F; f++) a.x[f] = x[f];
    a.n = n;
    a.F = F;
    a.keys = keys;
    const uint64_t chunk = (uint64_t)unroll * 256;
    a.cpf = (n / 4 + chunk - 1) / chunk;
    if (a.cpf == 0) a.cpf = 1;  // workgroup 0 still takes the loose elements
    uint64_t groups = (uint64_t)groups_per_cu * device_cu_count();
    if (groups > a.cpf * F) groups = a.cpf * F;  // never more than the chunks
    if (groups == 0) groups = 1;
    const dim3 g((uint32_t)groups), b(256);
    switch (unroll) {
        case 2: hipLaunchKernelGGL(field_range_kernel<2>, g, b, 0, s, a); break;
        case 4: hipLaunchKernelGGL(field_range_kernel<4>, g, b, 0, s, a); break;
        case 8: hipLaunchKernelGGL(field_range_kernel<8>, g, b, 0, s, a); break;
        case 16: hipLaunchKernelGGL(field_range_kernel<16>, g, b, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_field_range(const float* const* x, uint64_t n, uint32_t F, int* keys,
                              hipStream_t s) {
    // two workgroups per CU, four 16-byte loads in flight per lane: the best
    // shape of a sweep over 1-16 workgroups per CU and 2-16 loads (64M x 6)
    return launch_field_range_shape(x, n, F, keys, 2, 4, s);
}

}  // namespace gpz
