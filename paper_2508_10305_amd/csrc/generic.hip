// Generic block kernels: the cases the wave-per-block kernels leave out.
//  - float64 fields (Sec. 5.1: each field of each block is down-cast to
//    float32 when that meets the bound, else quantized in double);
//  - fields of a block whose grid needs more than 24 bits (Sec. 5.3: 64-bit
//    intermediates when the value range needs them): the fast encoder
//    leaves such blocks on a list for the encoder here (the fast decoder
//    decodes their records with the record decoder of generic_block.h);
//  - block sizes outside 256..2048 (the format allows 64..4096).
// One workgroup of 256 lanes per block.  Lane t owns the IPT = CB/256
// consecutive positions [t*IPT, t*IPT + IPT) of a block of capacity CB
// ("blocked"), which is what keeps the LDS radix sort stable.  The block's
// codes, flags, sort buffers and run tables live in LDS; every value is read
// from global memory again where a later phase needs it.
#include "generic_block.h"

namespace gpz {
namespace {

constexpr uint32_t kT = 256;                       // lanes per workgroup
constexpr uint32_t kDigit = 4;                     // radix sort digit bits
template <uint32_t CB>
struct GenEncodeSmem {
    static constexpr uint32_t IPT = CB / kT;
    uint16_t idxA[CB], idxB[CB];  // sort buffers: particle indices in block order
    uint16_t key[CB];             // linearised segment ID of each particle (K*KF <= 15 bits)
    union {
        uint16_t cnt[(1u << kDigit) * kT];      // radix counters, digit-major
        struct {
            uint64_t q[CB];                     // grid indices of one field
            uint8_t out[CB];                    // its outlier flags
        } f;
        struct {
            uint32_t uniq[CB];                  // distinct IDs, ascending
            uint32_t start[CB + 1];             // first sorted position of each run
        } r;
    } u;
    Scratch s;
};

// One field of a block after quantization.
struct GenField {
    uint64_t lo_bits;  // float32 bits (float32 stream) or float64 bits (float64 stream)
    uint64_t qmax;
    uint32_t nout;
    bool wide;
};

// Stage 1 (Sec. 4.1) for field f of the block at `base`: block minimum, grid
// index and outlier flag of every value, into sm.u.f.  The 32-bit steps
// unless the field needs 64-bit ones (float32: a finite value beyond 2^24 - 1
// grid steps; float64: some finite value the float32 down-cast does not
// reconstruct within the bound of the double).
template <uint32_t CB>
__device__ GenField quantize_field(const EncodeArgs& a, uint32_t f, uint64_t base, uint32_t nb,
                                   GenEncodeSmem<CB>& sm) {
    constexpr uint32_t IPT = CB / kT;
    const uint32_t t0 = threadIdx.x * IPT;
    const float eb = a.eb[f], twoeb = a.twoeb[f], inv = a.inv[f];
    const double twoeb64 = 2.0 * (double)eb;
    const double inv64 = 1.0 / twoeb64;
    GenField r{0, 0, 0, false};
    if (!a.f64) {
        const float* x = a.x[f] + base;
        float v[IPT];
        uint32_t mk = 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t j = 0; j < IPT; j++) {
            const uint32_t i = t0 + j;
            v[j] = i < nb ? x[i] : 0.0f;
            if (i < nb && __builtin_isfinite(v[j])) mk = min(mk, okey32(v[j]));
        }
        const uint64_t m = block_min_u64(mk, sm.s);
        float lo = m == 0xFFFFFFFFull ? 0.0f : from_okey32((uint32_t)m);
        if (lo == 0.0f) lo = 0.0f;
        bool need = false;
#pragma unroll
        for (uint32_t j = 0; j < IPT; j++) {
            const uint32_t i = t0 + j;
            if (i >= nb) continue;
            const float tt = (v[j] - lo) * inv;
            const bool in = (tt >= 0.0f) && (tt <= kQMax);
            const uint32_t q = in ? (uint32_t)__builtin_rintf(tt) : 0u;
            const float xr = __builtin_fmaf((float)q, twoeb, lo);
            sm.u.f.q[i] = q;
            sm.u.f.out[i] = (in && __builtin_fabsf(xr - v[j]) < eb) ? 0 : 1;
            if (__builtin_isfinite(v[j]) && !in) need = true;
        }
        r.wide = block_any(need, sm.s);
        r.lo_bits = f2u(lo);
        if (r.wide) {
            const double lo64 = (double)lo;
#pragma unroll
            for (uint32_t j = 0; j < IPT; j++) {
                const uint32_t i = t0 + j;
                if (i >= nb) continue;
                const double x64 = (double)v[j];
                const double tt = (x64 - lo64) * inv64;
                const bool in = (tt >= 0.0) && (tt <= kQMaxWide);
                const uint64_t q = in ? (uint64_t)__builtin_rint(tt) : 0ull;
                const double xr = (double)(float)__builtin_fma((double)q, twoeb64, lo64);
                sm.u.f.q[i] = q;
                sm.u.f.out[i] = (in && __builtin_fabs(xr - x64) < (double)eb) ? 0 : 1;
            }
        }
    } else {
        const double* x = reinterpret_cast<const double*>(a.x[f]) + base;
        double v[IPT];
        uint32_t mk = 0xFFFFFFFFu;
        bool bad = false;
#pragma unroll
        for (uint32_t j = 0; j < IPT; j++) {
            const uint32_t i = t0 + j;
            v[j] = i < nb ? x[i] : 0.0;
            const float xf = (float)v[j];
            if (i < nb && __builtin_isfinite(v[j]) && !__builtin_isfinite(xf)) bad = true;
            if (i < nb && __builtin_isfinite(xf)) mk = min(mk, okey32(xf));
        }
        const uint64_t m = block_min_u64(mk, sm.s);
        float lo = m == 0xFFFFFFFFull ? 0.0f : from_okey32((uint32_t)m);
        if (lo == 0.0f) lo = 0.0f;
#pragma unroll
        for (uint32_t j = 0; j < IPT; j++) {
            const uint32_t i = t0 + j;
            if (i >= nb) continue;
            if (!__builtin_isfinite(v[j])) {
                sm.u.f.q[i] = 0;
                sm.u.f.out[i] = 1;
                continue;
            }
            const float xf = (float)v[j];
            const float tt = (xf - lo) * inv;
            const bool in = (tt >= 0.0f) && (tt <= kQMax);
            const uint32_t q = in ? (uint32_t)__builtin_rintf(tt) : 0u;
            const float y = __builtin_fmaf((float)q, twoeb, lo);
            sm.u.f.q[i] = q;
            sm.u.f.out[i] = 0;
            if (!in || !(__builtin_fabs((double)y - v[j]) < (double)eb)) bad = true;
        }
        r.wide = block_any(bad, sm.s);
        r.lo_bits = d2u((double)lo);
        if (r.wide) {
            uint64_t mk64 = ~0ull;
#pragma unroll
            for (uint32_t j = 0; j < IPT; j++)
                if (t0 + j < nb && __builtin_isfinite(v[j])) mk64 = min(mk64, okey64(v[j]));
            const uint64_t m64 = block_min_u64(mk64, sm.s);
            double lo64 = m64 == ~0ull ? 0.0 : from_okey64(m64);
            if (lo64 == 0.0) lo64 = 0.0;
            r.lo_bits = d2u(lo64);
#pragma unroll
            for (uint32_t j = 0; j < IPT; j++) {
                const uint32_t i = t0 + j;
                if (i >= nb) continue;
                const double tt = (v[j] - lo64) * inv64;
                const bool in = (tt >= 0.0) && (tt <= kQMaxWide);
                const uint64_t q = in ? (uint64_t)__builtin_rint(tt) : 0ull;
                const double xr = __builtin_fma((double)q, twoeb64, lo64);
                sm.u.f.q[i] = q;
                sm.u.f.out[i] = (in && __builtin_fabs(xr - v[j]) < (double)eb) ? 0 : 1;
            }
        }
    }
    __syncthreads();
    uint64_t qm = 0;
    uint32_t no = 0;
#pragma unroll
    for (uint32_t j = 0; j < IPT; j++) {
        const uint32_t i = t0 + j;
        if (i < nb) {
            qm = sm.u.f.q[i] > qm ? sm.u.f.q[i] : qm;
            no += sm.u.f.out[i];
        }
    }
    r.qmax = block_max_u64(qm, sm.s);
    r.nout = block_sum_u32(no, sm.s);
    return r;
}

// One radix pass of the stable in-block sort (Sec. 4.2) over the 4-bit
// digit of the IDs at bit `sh`: per-lane digit counts, an exclusive scan in
// digit-major order, then each lane scatters its positions in order.
template <uint32_t CB>
__device__ void radix_pass(const uint16_t* __restrict__ in, uint16_t* __restrict__ out,
                           uint32_t sh, uint32_t nb, GenEncodeSmem<CB>& sm) {
    constexpr uint32_t IPT = CB / kT;
    constexpr uint32_t D = 1u << kDigit;
    const uint32_t t = threadIdx.x, t0 = t * IPT;
    __syncthreads();  // the counters share LDS with the previous phase
#pragma unroll
    for (uint32_t d = 0; d < D; d++) sm.u.cnt[d * kT + t] = 0;
#pragma unroll
    for (uint32_t j = 0; j < IPT; j++)
        if (t0 + j < nb) sm.u.cnt[((sm.key[in[t0 + j]] >> sh) & (D - 1)) * kT + t]++;
    __syncthreads();
    // lane t scans the 16 consecutive counters [16t, 16t + 16) of the
    // digit-major order
    uint32_t c[D], sum = 0;
#pragma unroll
    for (uint32_t e = 0; e < D; e++) {
        c[e] = sm.u.cnt[D * t + e];
        sum += c[e];
    }
    uint32_t total;
    uint32_t run = block_excl_scan_u32(sum, sm.s, &total);
#pragma unroll
    for (uint32_t e = 0; e < D; e++) {
        sm.u.cnt[D * t + e] = (uint16_t)run;
        run += c[e];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < IPT; j++) {
        if (t0 + j < nb) {
            const uint16_t i = in[t0 + j];
            const uint32_t slot = ((sm.key[i] >> sh) & (D - 1)) * kT + t;
            out[sm.u.cnt[slot]++] = i;
        }
    }
    __syncthreads();
}

// Stages 1-3 (Sec. 4.1-4.3) of block b into its workspace slot, then its
// length and superblock sum (first compaction step, Sec. 4.4).
template <uint32_t CB>
__device__ void gen_encode_block(const EncodeArgs& a, uint32_t b, GenEncodeSmem<CB>& sm) {
    constexpr uint32_t IPT = CB / kT;
    const uint32_t t = threadIdx.x, t0 = t * IPT;
    const uint64_t base = (uint64_t)b * a.B;
    const uint32_t nb = (uint32_t)((a.n - base) < a.B ? (a.n - base) : a.B);
    const uint32_t F = a.F, K = a.K, KF = a.KF;
    const uint32_t vw = a.f64 ? 2u : 1u;
    const uint32_t cap = 1 + F * nb * vw;  // raw record length
    uint32_t* __restrict__ rec = a.temp + (uint64_t)b * a.slot_words;

    // ---- Stage 1: key axes, linearised segment ID (axis 0 most significant)
#pragma unroll
    for (uint32_t j = 0; j < IPT; j++) sm.key[t0 + j] = 0;
    uint32_t s[3] = {0, 0, 0};
    for (uint32_t ax = 0; ax < KF; ax++) {
        const GenField g = quantize_field<CB>(a, ax, base, nb, sm);
        const uint32_t W = bit_width64(g.qmax);
        s[ax] = W > K ? W - K : 0;
#pragma unroll
        for (uint32_t j = 0; j < IPT; j++)
            if (t0 + j < nb)
                sm.key[t0 + j] = (uint16_t)((sm.key[t0 + j] << K) | (uint32_t)(sm.u.f.q[t0 + j] >> s[ax]));
        __syncthreads();
    }
    // OR of every ID: a digit pass only where some ID has a nonzero digit
    uint32_t kor = 0;
#pragma unroll
    for (uint32_t j = 0; j < IPT; j++) {
        sm.idxA[t0 + j] = (uint16_t)(t0 + j);
        if (t0 + j < nb) kor |= sm.key[t0 + j];
    }
    const uint32_t korr = block_or_u32(kor, sm.s);  // its barriers also publish idxA

    // ---- Stage 2: stable in-block sort by segment ID
    uint16_t* cur = sm.idxA;
    uint16_t* nxt = sm.idxB;
    for (uint32_t sh = 0; sh < K * KF; sh += kDigit) {
        if (((korr >> sh) & ((1u << kDigit) - 1u)) == 0) continue;  // identity pass
        radix_pass<CB>(cur, nxt, sh, nb, sm);
        uint16_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    __syncthreads();

    // ---- Stage 3: run-length coding of the sorted IDs
    uint32_t nflag = 0;
    bool flag[IPT];
#pragma unroll
    for (uint32_t j = 0; j < IPT; j++) {
        const uint32_t p = t0 + j;
        flag[j] = p < nb && (p == 0 || sm.key[cur[p]] != sm.key[cur[p - 1]]);
        nflag += flag[j];
    }
    uint32_t U;
    uint32_t rank = block_excl_scan_u32(nflag, sm.s, &U);
#pragma unroll
    for (uint32_t j = 0; j < IPT; j++) {
        if (flag[j]) {
            sm.u.r.uniq[rank] = sm.key[cur[t0 + j]];
            sm.u.r.start[rank] = t0 + j;
            rank++;
        }
    }
    if (t == 0) sm.u.r.start[U] = nb;
    __syncthreads();
    uint64_t gmax = 0, cmax = 0;
    for (uint32_t jj = t; jj < U; jj += kT) {
        const uint32_t g = jj == 0 ? sm.u.r.uniq[0] : sm.u.r.uniq[jj] - sm.u.r.uniq[jj - 1] - 1u;
        const uint32_t c = sm.u.r.start[jj + 1] - sm.u.r.start[jj] - 1u;
        gmax = g > gmax ? g : gmax;
        cmax = c > cmax ? c : cmax;
    }
    const uint32_t w_gap = bit_width64(block_max_u64(gmax, sm.s));
    const uint32_t w_cnt = bit_width64(block_max_u64(cmax, sm.s));
    uint32_t pos = 2;
    bool over = pos + words_for(U, w_gap) + words_for(U, w_cnt) > cap;
    if (!over) {
        pack_seq<kT>(rec + pos, U, w_gap, [&](uint32_t jj) -> uint64_t {
            return jj == 0 ? sm.u.r.uniq[0] : sm.u.r.uniq[jj] - sm.u.r.uniq[jj - 1] - 1u;
        });
        pos += words_for(U, w_gap);
        pack_seq<kT>(rec + pos, U, w_cnt, [&](uint32_t jj) -> uint64_t {
            return sm.u.r.start[jj + 1] - sm.u.r.start[jj] - 1u;
        });
        pos += words_for(U, w_cnt);
    }
    __syncthreads();  // the run tables are read; their LDS is reused

    // ---- per field: lo, field word, payload in sorted order, outliers
    bool any_wide = false;
    for (uint32_t f = 0; f < F && !over; f++) {
        const GenField g = quantize_field<CB>(a, f, base, nb, sm);
        const bool key = f < KF;
        const uint64_t mask = key ? low_mask64(s[f]) : ~0ull;
        uint64_t vmax = 0;
#pragma unroll
        for (uint32_t j = 0; j < IPT; j++) {
            if (t0 + j < nb) {
                const uint64_t v = sm.u.f.q[t0 + j] & mask;
                vmax = v > vmax ? v : vmax;
            }
        }
        const uint32_t w = bit_width64(block_max_u64(vmax, sm.s));
        const uint32_t pw = words_for(nb, w);
        if ((uint64_t)pos + vw + 1 + pw + (uint64_t)(1 + vw) * g.nout > cap) {
            over = true;
            break;
        }
        if (t == 0) {
            rec[pos] = (uint32_t)g.lo_bits;
            if (vw == 2) rec[pos + 1] = (uint32_t)(g.lo_bits >> 32);
            rec[pos + vw] = g.wide ? (w | (g.nout << 6) | (1u << 31)) : (w | (g.nout << 5));
        }
        pos += vw + 1;
        pack_seq<kT>(rec + pos, nb, w, [&](uint32_t p) -> uint64_t { return sm.u.f.q[cur[p]] & mask; });
        pos += pw;
        if (g.nout) {
            uint32_t c = 0;
#pragma unroll
            for (uint32_t j = 0; j < IPT; j++)
                if (t0 + j < nb) c += sm.u.f.out[cur[t0 + j]];
            uint32_t tot;
            uint32_t k = block_excl_scan_u32(c, sm.s, &tot);
            uint32_t* ol = rec + pos;
#pragma unroll
            for (uint32_t j = 0; j < IPT; j++) {
                const uint32_t p = t0 + j;
                if (p < nb && sm.u.f.out[cur[p]]) {
                    const uint32_t i = cur[p];
                    ol[(1 + vw) * k] = p;
                    if (vw == 2) {
                        const uint64_t u = d2u(reinterpret_cast<const double*>(a.x[f])[base + i]);
                        ol[(1 + vw) * k + 1] = (uint32_t)u;
                        ol[(1 + vw) * k + 2] = (uint32_t)(u >> 32);
                    } else {
                        ol[2 * k + 1] = f2u(a.x[f][base + i]);
                    }
                    k++;
                }
            }
            pos += (1 + vw) * g.nout;
        }
        any_wide = any_wide || g.wide;
        __syncthreads();  // the field's codes are read before the next field's
    }

    const bool raw = over || pos >= cap;
    if (raw) {
        // raw form: the block's values verbatim, field-major, input order;
        // the barrier orders these stores after the coded ones they replace
        __syncthreads();
        if (t == 0) rec[0] = 1u;
        for (uint32_t f = 0; f < F; f++) {
            uint32_t* dst = rec + 1 + f * nb * vw;
            if (vw == 2) {
                const uint64_t* xf = reinterpret_cast<const uint64_t*>(a.x[f]) + base;
                for (uint32_t i = t; i < nb; i += kT) {
                    const uint64_t u = xf[i];
                    dst[2 * i] = (uint32_t)u;
                    dst[2 * i + 1] = (uint32_t)(u >> 32);
                }
            } else {
                const float* xf = a.x[f] + base;
                for (uint32_t i = t; i < nb; i += kT) dst[i] = f2u(xf[i]);
            }
        }
    } else if (t == 0) {
        rec[0] = (U << 2) | (any_wide ? (1u << 31) : 0u);
        rec[1] = w_gap | (w_cnt << 5) | ((s[0] & 31u) << 10) | ((s[1] & 31u) << 15) |
                 ((s[2] & 31u) << 20) | ((s[0] >> 5) << 25) | ((s[1] >> 5) << 26) |
                 ((s[2] >> 5) << 27);
    }
    if (t == 0) {
        const uint32_t len = raw ? cap : pos;
        a.lens[b] = len;
        atomicAdd(&a.supsum[b / kSuper], len);
        if (!raw && any_wide) atomicOr(a.wide_flag, 1u);
    }
    if (a.perm) {
#pragma unroll
        for (uint32_t j = 0; j < IPT; j++) {
            const uint32_t p = t0 + j;
            if (p < nb) a.perm[base + p] = (uint32_t)(base + (raw ? p : cur[p]));
        }
    }
}

// Every block of a snapshot, one workgroup each.
template <uint32_t CB>
__global__ __launch_bounds__(256) void gen_encode_all(EncodeArgs a) {
    __shared__ __align__(16) GenEncodeSmem<CB> sm;
    gen_encode_block<CB>(a, blockIdx.x, sm);
}

// The blocks the fast encoder left on the deferred list (their grid needs
// 64-bit steps); a fixed grid walks the list, whose length is only known on
// the device.
template <uint32_t CB>
__global__ __launch_bounds__(256) void gen_encode_deferred(EncodeArgs a) {
    __shared__ __align__(16) GenEncodeSmem<CB> sm;
    const uint32_t count = *a.defer_count;
    for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
        gen_encode_block<CB>(a, a.defer[k], sm);
        __syncthreads();
    }
}

// The deferred blocks, then the length scan (second compaction step,
// Sec. 4.4) in the same launch.  Workgroup g < min(count, grid) walks its
// share of the list; the last of those to finish (counted in *done) scans
// the superblock sums, which by then hold every block's length.  With no
// deferred block, workgroup 0 scans at once and no counter is touched (an
// atomic per workgroup on one word would serialize).  One dependent launch
// fewer than a walk followed by the scan kernel.
template <uint32_t CB>
__global__ __launch_bounds__(256) void gen_encode_deferred_then_scan(EncodeArgs a, ScanArgs sa,
                                                                     uint32_t* done) {
    __shared__ __align__(16) union {
        GenEncodeSmem<CB> enc;
        uint64_t part[kT];
    } sm;
    __shared__ uint32_t last;
    const uint32_t count = *a.defer_count;
    const uint32_t workers = count < gridDim.x ? count : gridDim.x;
    if (workers == 0) {
        if (blockIdx.x == 0) scan_superblocks<kT>(sa, sm.part);
        return;
    }
    if (blockIdx.x >= workers) return;
    for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
        gen_encode_block<CB>(a, a.defer[k], sm.enc);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's records, lengths and sums first
        last = atomicAdd(done, 1u) == workers - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // every other worker's writes are visible past here
    scan_superblocks<kT>(sa, sm.part);
}

// The same over the deferred lists of every job of a batch.
template <uint32_t CB>
__global__ __launch_bounds__(256) void gen_encode_deferred_batch(const EncodeArgs* __restrict__ jobs,
                                                                 const BatchLaunch* __restrict__ L) {
    __shared__ __align__(16) GenEncodeSmem<CB> sm;
    __shared__ uint32_t counts[kT];
    const uint32_t njobs = L->njobs;
    for (uint32_t j0 = 0; j0 < njobs; j0 += kT) {
        // the deferred counts of kT jobs at once, one job per thread: when
        // nothing is deferred (the common case) the walk costs one memory
        // round trip per kT jobs instead of one per job
        const uint32_t jt = j0 + threadIdx.x;
        const uint32_t c = jt < njobs ? *jobs[jt].defer_count : 0u;
        counts[threadIdx.x] = c;
        __syncthreads();  // every count is in LDS before any thread reads them
        if (!__syncthreads_or(c != 0u)) continue;
        const uint32_t jn = njobs - j0 < kT ? njobs - j0 : kT;
        for (uint32_t i = 0; i < jn; i++) {
            const uint32_t count = counts[i];
            const EncodeArgs& a = jobs[j0 + i];
            for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
                gen_encode_block<CB>(a, a.defer[k], sm);
                __syncthreads();
            }
        }
        __syncthreads();  // counts[] is read before the next group replaces it
    }
}

// ------------------------------------------------------------ decoder

// Decompression of block b (Sec. 3.2) by one 256-lane workgroup: locate the
// record through the superblock table and check it against the stream (as
// the wave-per-block decoder does), then decode it.
template <uint32_t CB>
__device__ void gen_decode_block(const DecodeArgs& a, uint32_t b, GenDecodeSmem<CB>& sm) {
    constexpr uint32_t IPT = CB / kT;
    const uint32_t t = threadIdx.x, t0 = t * IPT;
    const bool f64 = a.f64 != 0;
    const uint32_t vw = f64 ? 2u : 1u;
    const uint64_t base = (uint64_t)b * a.B;
    const uint32_t nb = (uint32_t)((a.n - base) < a.B ? (a.n - base) : a.B);
    const uint32_t F = a.F, K = a.K, KF = a.KF;
    const uint64_t nsup = nsuper_of(a.nblocks);
    const uint32_t* sup = a.in + kHeaderWords;
    const uint32_t* ebt = sup + 2 * nsup;
    const uint32_t* lens = ebt + F;
    const uint32_t* recs = a.in + a.prefix;
    const uint64_t rec_total = a.in_words - a.prefix;

    // ---- locate the record (wave 0): superblock offset + lengths before it,
    // every sum in 64 bits and every offset checked against the record area
    if (t < 64) {
        const uint32_t sb = b / kSuper, first = sb * kSuper;
        const uint64_t sup_off = (uint64_t)sup[2 * sb] | ((uint64_t)sup[2 * sb + 1] << 32);
        uint64_t mine = (first + t < b) ? (uint64_t)lens[first + t] : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
        const uint64_t off = sup_off + mine;
        const uint32_t len = lens[b];
        bool bad = sup_off > rec_total || off > rec_total || (uint64_t)len > rec_total - off;
        if (b == 0 && (sup[0] | sup[1]) != 0u) bad = true;
        if (a.exact && b + 1 == a.nblocks && off + len != rec_total) bad = true;
        // header: magic, version and flags (float64 as the caller says, the
        // wide-record flag free), N, F, B, K | KF << 8, block count; eb table
        if (t < kHeaderWords) {
            const uint32_t h = a.in[t];
            bool ok;
            switch (t) {
                case 0: ok = h == kMagic; break;
                case 1: ok = (h & 0xFFFFu) == kVersion && ((h >> 16) & ~2u) == (f64 ? 1u : 0u); break;
                case 2: ok = h == (uint32_t)(a.n & 0xFFFFFFFFu); break;
                case 3: ok = h == (uint32_t)(a.n >> 32); break;
                case 4: ok = h == a.F; break;
                case 5: ok = h == a.B; break;
                case 6: ok = h == (a.K | (a.KF << 8)); break;
                default: ok = h == a.nblocks; break;
            }
            if (!ok) bad = true;
        }
        for (uint32_t f = t; f < F; f += 64)
            if (!eb_in_range(u2f(ebt[f]))) bad = true;
        if (b == first && sb > 0) {
            uint64_t pl = lens[first - kSuper + t];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) pl += __shfl_xor(pl, o);
            const uint64_t prev = (uint64_t)sup[2 * sb - 2] | ((uint64_t)sup[2 * sb - 1] << 32);
            if (prev > rec_total || prev + pl != off) bad = true;
        }
        const bool any = __any(bad);
        if (t == 0) {
            sm.off = off;
            sm.bad = any ? 1u : 0u;
        }
    }
    __syncthreads();
    if (sm.bad) {
        if (t == 0) *a.err = 1u;
        return;
    }
    gen_decode_record<CB, kT>(a, b, recs + sm.off, lens[b], sm);
}

template <uint32_t CB>
__global__ __launch_bounds__(256) void gen_decode_all(DecodeArgs a) {
    __shared__ __align__(16) GenDecodeSmem<CB> sm;
    gen_decode_block<CB>(a, blockIdx.x, sm);
}

// Workgroups of the fixed grids: enough to keep every CU busy when a whole
// snapshot is wide, and few enough that an empty walk costs little.
uint32_t walk_grid(uint32_t nblocks) {
    const uint32_t g = 4u * device_cu_count();
    return nblocks < g ? (nblocks ? nblocks : 1u) : g;
}

}  // namespace

hipError_t launch_encode_generic(const EncodeArgs& a, bool deferred_only, hipStream_t s) {
    if (a.nblocks == 0) return hipSuccess;
    const dim3 block(kT);
    if (deferred_only) {
        const dim3 grid(walk_grid(a.nblocks));
        if (a.B <= 1024) hipLaunchKernelGGL(gen_encode_deferred<1024>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(gen_encode_deferred<4096>, grid, block, 0, s, a);
    } else {
        const dim3 grid(a.nblocks);
        if (a.B <= 256) hipLaunchKernelGGL(gen_encode_all<256>, grid, block, 0, s, a);
        else if (a.B <= 1024) hipLaunchKernelGGL(gen_encode_all<1024>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(gen_encode_all<4096>, grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_encode_deferred_then_scan(const EncodeArgs& a, const ScanArgs& sa,
                                            uint32_t* done, hipStream_t s) {
    // two workgroups per CU: few empty workgroups when nothing is deferred
    const uint32_t g = 2u * device_cu_count();
    const dim3 grid(a.nblocks < g ? (a.nblocks ? a.nblocks : 1u) : g), block(kT);
    if (a.B <= 1024)
        hipLaunchKernelGGL(gen_encode_deferred_then_scan<1024>, grid, block, 0, s, a, sa, done);
    else
        hipLaunchKernelGGL(gen_encode_deferred_then_scan<4096>, grid, block, 0, s, a, sa, done);
    return hipGetLastError();
}

hipError_t launch_decode_generic(const DecodeArgs& a, hipStream_t s) {
    if (a.nblocks == 0) return hipSuccess;
    const dim3 grid(a.nblocks), block(kT);
    if (a.B <= 256) hipLaunchKernelGGL(gen_decode_all<256>, grid, block, 0, s, a);
    else if (a.B <= 1024) hipLaunchKernelGGL(gen_decode_all<1024>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(gen_decode_all<4096>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_encode_generic_batch(const EncodeArgs* jobs, const BatchLaunch* L, uint32_t B,
                                       uint32_t max_blocks, hipStream_t s) {
    const dim3 grid(walk_grid(max_blocks)), block(kT);
    if (B <= 1024) hipLaunchKernelGGL(gen_encode_deferred_batch<1024>, grid, block, 0, s, jobs, L);
    else hipLaunchKernelGGL(gen_encode_deferred_batch<4096>, grid, block, 0, s, jobs, L);
    return hipGetLastError();
}


}  // namespace gpz
