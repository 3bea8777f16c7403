// Shared pieces of the generic block kernels (float64 fields, fields coded
// with 64-bit grid steps, any block size): workgroup-wide primitives for
// workgroups of one to four waves, fixed-length packing and unpacking of
// values up to 53 bits, and the record decoder, which the wave-per-block
// decoder also calls for a record with a wide field.
#pragma once

#include "gpz_internal.h"

namespace gpz {

constexpr double kQMaxWide = 9007199254740991.0;   // largest wide grid index, 2^53 - 1

__device__ __forceinline__ uint32_t bit_width64(uint64_t v) {
    return v ? 64u - (uint32_t)__builtin_clzll(v) : 0u;
}
__device__ __forceinline__ uint64_t low_mask64(uint32_t w) {
    return w >= 64u ? ~0ull : ((1ull << w) - 1ull);
}
__device__ __forceinline__ uint64_t d2u(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ double u2d(uint64_t u) { return __longlong_as_double((long long)u); }

// Order-preserving unsigned keys (-0 below +0); callers exclude NaN.
__device__ __forceinline__ uint32_t okey32(float v) {
    const uint32_t u = __float_as_uint(v);
    return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}
__device__ __forceinline__ float from_okey32(uint32_t k) {
    return __uint_as_float(k ^ (((k >> 31) - 1u) | 0x80000000u));
}
__device__ __forceinline__ uint64_t okey64(double v) {
    const uint64_t u = d2u(v);
    return u ^ ((uint64_t)((int64_t)u >> 63) | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_okey64(uint64_t k) {
    return u2d(k ^ (((k >> 63) - 1ull) | 0x8000000000000000ull));
}

// ---- workgroup-wide reductions and scans for workgroups of 1-4 waves.
// Every lane of the workgroup calls them (no lane has left); the leading
// barrier lets the scratch be reused.
struct Scratch {
    uint64_t w64[4];
    uint32_t w32[4];
};

__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, Scratch& s) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) s.w64[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t r = s.w64[0];
    for (uint32_t k = 1; k < (blockDim.x >> 6); k++) r = s.w64[k] > r ? s.w64[k] : r;
    return r;
}

__device__ __forceinline__ uint64_t block_min_u64(uint64_t v, Scratch& s) {
    return ~block_max_u64(~v, s);
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, Scratch& s) {
    v = wave_sum_u32(v);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) s.w32[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = 0;
    for (uint32_t k = 0; k < (blockDim.x >> 6); k++) r += s.w32[k];
    return r;
}

__device__ __forceinline__ bool block_any(bool v, Scratch& s) { return block_sum_u32(v ? 1u : 0u, s) != 0; }

__device__ __forceinline__ uint32_t block_or_u32(uint32_t v, Scratch& s) {
    v = wave_or_u32(v);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) s.w32[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = 0;
    for (uint32_t k = 0; k < (blockDim.x >> 6); k++) r |= s.w32[k];
    return r;
}

// Exclusive prefix sum over the lanes in workgroup order; *total = the sum.
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, Scratch& s, uint32_t* total) {
    const uint32_t incl = wave_incl_scan_u32(v);
    __syncthreads();
    if ((threadIdx.x & 63u) == 63u) s.w32[threadIdx.x >> 6] = incl;
    __syncthreads();
    const uint32_t w = threadIdx.x >> 6;
    uint32_t off = 0, tot = 0;
    for (uint32_t k = 0; k < (blockDim.x >> 6); k++) {
        off += k < w ? s.w32[k] : 0u;
        tot += s.w32[k];
    }
    *total = tot;
    return off + incl - v;
}

// Maximum over the lanes before this one, in workgroup order (0 for lane 0).
__device__ __forceinline__ uint32_t block_excl_max_u32(uint32_t v, Scratch& s) {
    const uint32_t incl = wave_incl_max_u32(v);
    uint32_t x = (uint32_t)__shfl_up((int)incl, 1);
    if ((threadIdx.x & 63u) == 0) x = 0;
    __syncthreads();
    if ((threadIdx.x & 63u) == 63u) s.w32[threadIdx.x >> 6] = incl;
    __syncthreads();
    const uint32_t w = threadIdx.x >> 6;
    for (uint32_t k = 0; k < w; k++) x = max(x, s.w32[k]);
    return x;
}

// Fixed-length coding (Sec. 4.3): value i of width w at bits [i*w, i*w + w)
// of an LSB-first word stream.  Lane t builds words t, t + LANES, ...; each
// word ORs in the (at most 33) values that overlap it, so every word is
// written once and its padding bits are zero.  w <= 53.
template <uint32_t LANES, class Get>
__device__ __forceinline__ void pack_seq(uint32_t* __restrict__ dst, uint32_t count, uint32_t w,
                                         Get get) {
    if (w == 0 || count == 0) return;
    const uint32_t words = words_for(count, w);
    for (uint32_t j = threadIdx.x; j < words; j += LANES) {
        const uint32_t b0 = 32u * j;
        uint32_t i = b0 / w;
        const uint32_t iend = min(count, (b0 + 32u + w - 1u) / w);
        uint32_t word = 0;
        for (; i < iend; i++) {
            const uint32_t vb = i * w;
            const uint64_t v = get(i);
            word |= vb >= b0 ? (uint32_t)(v << (vb - b0)) : (uint32_t)(v >> (b0 - vb));
        }
        dst[j] = word;
    }
}

// Value i of width w (<= 53) of a fixed-length array in global memory whose
// bit length is at least (i + 1) * w (so every word read is inside it).
__device__ __forceinline__ uint64_t get_bits64(const uint32_t* __restrict__ src, uint32_t i,
                                               uint32_t w) {
    if (w == 0) return 0;
    const uint32_t bit = i * w, wd = bit >> 5, sh = bit & 31u;
    const uint32_t last = (bit + w - 1u) >> 5;
    uint64_t v = (uint64_t)src[wd] >> sh;
    if (last > wd) v |= (uint64_t)src[wd + 1] << (32u - sh);
    if (last > wd + 1) v |= (uint64_t)src[wd + 2] << (64u - sh);
    return v & low_mask64(w);
}

// ------------------------------------------------------------ decoder

template <uint32_t CB>
struct GenDecodeSmem {
    uint32_t keyat[CB];  // segment ID + 1 at each run start, then every position's ID
    uint64_t off;        // the record's word offset in the record area
    uint32_t bad;
    Scratch s;
};

__device__ __forceinline__ bool eb_in_range(float eb) {
    return __builtin_isfinite(eb) && eb >= 0x1p-120f && eb <= 0x1p120f;
}

__device__ __forceinline__ void put_out(const DecodeArgs& a, uint32_t f, uint64_t i, double v,
                                        bool f64) {
    if (f64) reinterpret_cast<double*>(a.y[f])[i] = v;
    else a.y[f][i] = (float)v;
}

__device__ __forceinline__ void put_raw(const DecodeArgs& a, uint32_t f, uint64_t i,
                                        const uint32_t* w, bool f64) {
    if (f64) reinterpret_cast<uint64_t*>(a.y[f])[i] = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    else a.y[f][i] = u2f(w[0]);
}

// Decoding of block b's record (Sec. 3.2) of len words at rec, already
// located and checked against the stream, by one workgroup of LANES lanes:
// undo the run-length and delta coding, rebuild every value with the FMA of
// its field's steps (float32, or double for wide fields), patch the
// outliers, store in sorted order.  A malformed record sets *a.err.
// MAY_F64 false: a float32 stream only (the wave-per-block decoder's case,
// compiled without the float64 paths).
template <uint32_t CB, uint32_t LANES, bool MAY_F64 = true>
__device__ void gen_decode_record(const DecodeArgs& a, uint32_t b, const uint32_t* __restrict__ rec,
                                  uint32_t len, GenDecodeSmem<CB>& sm) {
    constexpr uint32_t IPT = CB / LANES;
    const uint32_t t = threadIdx.x, t0 = t * IPT;
    const bool f64 = MAY_F64 && a.f64 != 0;
    const uint32_t vw = f64 ? 2u : 1u;
    const uint64_t base = (uint64_t)b * a.B;
    const uint32_t nb = (uint32_t)((a.n - base) < a.B ? (a.n - base) : a.B);
    const uint32_t F = a.F, K = a.K, KF = a.KF;
    const uint32_t* ebt = a.in + kHeaderWords + 2 * nsuper_of(a.nblocks);
    const uint32_t h0 = len ? rec[0] : 0u;
    const uint32_t mode = h0 & 3u;
    if (len == 0 || mode > 1) {
        if (t == 0) *a.err = 1u;
        return;
    }
    if (mode == 1) {
        if (h0 != 1u || len != 1 + F * nb * vw) {
            if (t == 0) *a.err = 1u;
            return;
        }
        for (uint32_t f = 0; f < F; f++)
            for (uint32_t i = t; i < nb; i += LANES) put_raw(a, f, base + i, rec + 1 + (f * nb + i) * vw, f64);
        return;
    }
    const uint32_t U = (h0 & 0x7FFFFFFFu) >> 2, any_wide = h0 >> 31;
    const uint32_t h1 = len > 1 ? rec[1] : 0xFFFFFFFFu;
    const uint32_t w_gap = h1 & 31u, w_cnt = (h1 >> 5) & 31u;
    uint32_t s[3];
#pragma unroll
    for (uint32_t ax = 0; ax < 3; ax++)
        s[ax] = ((h1 >> (10 + 5 * ax)) & 31u) | (((h1 >> (25 + ax)) & 1u) << 5);
    bool bad = len < 2 || (h1 >> 28) != 0u || U < 1 || U > nb || w_gap > 15 || w_cnt > 12;
    // a wide record in a stream whose header does not announce one
    if (any_wide && !((a.in[1] >> 17) & 1u)) bad = true;
#pragma unroll
    for (uint32_t ax = 0; ax < 3; ax++) {
        if (ax >= KF && s[ax] != 0) bad = true;
        if (ax < KF && s[ax] + K > 53) bad = true;
    }
    const uint32_t gw = words_for(U, w_gap), cw = words_for(U, w_cnt);
    if ((uint64_t)2 + gw + cw > len) bad = true;
    if (bad) {
        if (t == 0) *a.err = 1u;
        return;
    }
    // ---- undo delta and run-length coding: lane t takes runs [t*IPT, ...)
    const uint32_t* gaps = rec + 2;
    const uint32_t* cnts = rec + 2 + gw;
    // (loops over a lane's positions are not unrolled: the wave-per-block
    // decoder runs this with 64 lanes and its register budget)
    uint32_t gsum = 0, csum = 0;
#pragma unroll 1
    for (uint32_t j = 0; j < IPT; j++) {
        const uint32_t r = t0 + j;
        if (r < U) {
            gsum += (uint32_t)get_bits64(gaps, r, w_gap) + 1u;
            csum += (uint32_t)get_bits64(cnts, r, w_cnt) + 1u;
        }
    }
    uint32_t gtot, ctot;
    uint32_t gx = block_excl_scan_u32(gsum, sm.s, &gtot);
    uint32_t cx = block_excl_scan_u32(csum, sm.s, &ctot);
    // the largest ID must fit K*KF bits and the runs must cover the block
    if (ctot != nb || gtot - 1u >= (1u << (K * KF))) {
        if (t == 0) *a.err = 1u;
        return;
    }
#pragma unroll 1
    for (uint32_t j = 0; j < IPT; j++) sm.keyat[t0 + j] = 0;
    __syncthreads();
#pragma unroll 1
    for (uint32_t j = 0; j < IPT; j++) {
        const uint32_t r = t0 + j;
        if (r < U) {
            gx += (uint32_t)get_bits64(gaps, r, w_gap) + 1u;
            sm.keyat[cx] = gx;  // ID + 1 at the run's first position
            cx += (uint32_t)get_bits64(cnts, r, w_cnt) + 1u;
        }
    }
    __syncthreads();
    // IDs increase with position: a prefix maximum gives every position the
    // ID (+1) of its run, left in keyat (lane t's positions in place)
    uint32_t run = 0;
#pragma unroll 1
    for (uint32_t j = 0; j < IPT; j++) {
        run = max(run, sm.keyat[t0 + j]);
        sm.keyat[t0 + j] = run;
    }
    const uint32_t prevmax = block_excl_max_u32(run, sm.s);
#pragma unroll 1
    for (uint32_t j = 0; j < IPT; j++) sm.keyat[t0 + j] = max(sm.keyat[t0 + j], prevmax) - 1u;

    // ---- fields
    uint64_t pos = 2 + gw + cw;
    uint32_t seen_wide = 0;
    for (uint32_t f = 0; f < F; f++) {
        if (pos + vw + 1 > len) {
            bad = true;
            break;
        }
        const uint64_t lob = vw == 2 ? ((uint64_t)rec[pos] | ((uint64_t)rec[pos + 1] << 32))
                                     : (uint64_t)rec[pos];
        const uint32_t wword = rec[pos + vw];
        const bool wide = (wword >> 31) != 0;
        const uint32_t w = wide ? (wword & 63u) : (wword & 31u);
        const uint32_t nout = wide ? ((wword >> 6) & 0x1FFFFFFu) : ((wword >> 5) & 0x3FFFFFFu);
        pos += vw + 1;
        seen_wide |= wide ? 1u : 0u;
        const uint32_t qbits = wide ? 53u : 24u;
        const uint32_t wlim = f < KF ? s[f] : qbits;
        const uint32_t pw = words_for(nb, w);
        if ((f < KF && s[f] + K > qbits) || w > wlim || nout > nb ||
            pos + pw + (uint64_t)(1 + vw) * nout > len) {
            bad = true;
            break;
        }
        const double lo64 = f64 ? u2d(lob) : (double)u2f((uint32_t)lob);
        const float lo32 = f64 ? (float)u2d(lob) : u2f((uint32_t)lob);
        const float eb = u2f(ebt[f]);
        const float twoeb = 2.0f * eb;
        const double twoeb64 = 2.0 * (double)eb;
        const uint32_t shift = f < KF ? K * (KF - 1 - f) : 0u;
        const uint32_t* pay = rec + pos;
#pragma unroll 1
        for (uint32_t j = 0; j < IPT; j++) {
            const uint32_t p = t0 + j;
            if (p >= nb) continue;
            const uint64_t v = get_bits64(pay, p, w);
            uint64_t q = v;
            if (f < KF) q = ((uint64_t)((sm.keyat[p] >> shift) & ((1u << K) - 1u)) << s[f]) + v;
            double y;
            if (wide) {
                y = __builtin_fma((double)q, twoeb64, lo64);
                if (!f64) y = (double)(float)y;
            } else {
                y = (double)__builtin_fmaf((float)(uint32_t)q, twoeb, lo32);
            }
            put_out(a, f, base + p, y, f64);
        }
        pos += pw;
        if (nout) {
            // the outliers overwrite values other lanes stored: the barrier
            // orders those stores first
            __syncthreads();
            const uint32_t* ol = rec + pos;
            bool obad = false;
            for (uint32_t k = t; k < nout; k += LANES) {
                const uint32_t op = ol[(1 + vw) * k];
                const uint32_t prevp = k ? ol[(1 + vw) * (k - 1)] : 0u;
                if (op >= nb || (k && prevp >= op)) obad = true;
                else put_raw(a, f, base + op, ol + (1 + vw) * k + 1, f64);
            }
            if (block_any(obad, sm.s)) {
                bad = true;
                break;
            }
            pos += (uint64_t)(1 + vw) * nout;
        }
    }
    if (bad || pos != len || seen_wide != any_wide) {
        if (t == 0) *a.err = 1u;
    }
}


}  // namespace gpz
