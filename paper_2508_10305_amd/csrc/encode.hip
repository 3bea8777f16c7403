// Block encoder: GPZ stages 1-3 (Sec. 4.1 quantization, Sec. 4.2 in-block
// sort, Sec. 4.3 run-length / delta / fixed-length coding) for one block of
// B particles per wave64, writing the block's record into its workspace slot
// (first step of the Sec. 4.4 compaction).
//
// Lane layout: lane l owns the ITEMS = B/64 consecutive particles
// [l*ITEMS, (l+1)*ITEMS) of its block ("blocked"), so per-lane sequential
// order followed by lane order is input order; that is what makes the LDS
// radix sort stable.  One wave per workgroup: __syncthreads() only orders LDS
// traffic, it never waits for another wave.
#include "gpz_internal.h"

namespace gpz {
namespace {

constexpr uint32_t kDigitBits = 5;
constexpr uint32_t kDigits = 1u << kDigitBits;
// Digit counters, digit-major: (d, lane) at d*64 + lane, with 4 pad words per
// 32 so that the raking scan reads 16-byte chunks without bank conflicts.
constexpr uint32_t kCounterWords = kDigits * 64 + kDigits * 64 / 8;

__device__ __forceinline__ uint32_t counter_addr(uint32_t d, uint32_t lane) {
    uint32_t f = d * 64 + lane;
    return f + 4 * (f >> 5);
}

// Padded blocked layout: position p of a block lives at p + 4*(p / ITEMS), so
// lane l's ITEMS consecutive positions start at l*(ITEMS+4) (16-byte aligned,
// spread over the banks).
template <int ITEMS>
__device__ __forceinline__ uint32_t pad_addr(uint32_t p) {
    return p + 4 * (p / ITEMS);
}

// Exact copy of the quantizer rule: t = (x - lo) * inv (two IEEE float ops),
// q = rint(t) when t lies in [0, 2^24-1] (else 0), outlier when out of range
// or when fma(q, 2eb, lo) misses x by more than eb (tested in double).
__device__ __forceinline__ uint32_t quantize(float x, float lo, float inv, float twoeb, float eb,
                                             bool& outlier) {
    float t = (x - lo) * inv;
    bool in = (t >= 0.0f) && (t <= kQMax);
    uint32_t q = in ? (uint32_t)__builtin_rintf(t) : 0u;
    float xr = __builtin_fmaf((float)q, twoeb, lo);
    bool ok = in && (__builtin_fabs((double)xr - (double)x) <= (double)eb);
    outlier = !ok;
    return q;
}

template <int ITEMS>
__device__ __forceinline__ void load_block(const float* __restrict__ x, uint64_t base, uint32_t nb,
                                           uint32_t lane, float (&v)[ITEMS]) {
    const float* p = x + base + (uint64_t)lane * ITEMS;
    const bool full = (lane + 1) * ITEMS <= nb;
    if (full && ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)) {
        const f32x4* p4 = reinterpret_cast<const f32x4*>(p);
#pragma unroll
        for (int k = 0; k < ITEMS / 4; k++) {
            f32x4 t = __builtin_nontemporal_load(p4 + k);
            v[4 * k + 0] = t.x;
            v[4 * k + 1] = t.y;
            v[4 * k + 2] = t.z;
            v[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t i = lane * ITEMS + j;
            v[j] = i < nb ? p[j] : 0.0f;
        }
    }
}

// Block minimum over finite values; zero (either sign) and "none" give +0.
template <int ITEMS>
__device__ __forceinline__ float block_low(const float (&v)[ITEMS], uint32_t lane, uint32_t nb) {
    float m = __builtin_inff();
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        bool ok = (lane * ITEMS + j < nb) && __builtin_isfinite(v[j]);
        m = fminf(m, ok ? v[j] : __builtin_inff());
    }
    m = wave_min_f32(m);
    return (m == __builtin_inff() || m == 0.0f) ? 0.0f : m;
}

// Quantize one field of the block: q | outlier << 31 per value (0 for
// positions beyond the block), returns lo.
template <int ITEMS>
__device__ __forceinline__ float quantize_field(const float* __restrict__ x, uint64_t base,
                                                uint32_t nb, uint32_t lane, float inv, float twoeb,
                                                float eb, uint32_t (&q)[ITEMS]) {
    float v[ITEMS];
    load_block<ITEMS>(x, base, nb, lane, v);
    float lo = block_low<ITEMS>(v, lane, nb);
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        bool o;
        uint32_t qq = quantize(v[j], lo, inv, twoeb, eb, o);
        q[j] = (lane * ITEMS + j < nb) ? (qq | ((uint32_t)o << 31)) : 0u;
    }
    return lo;
}

// Fixed-length packing (Sec. 4.3): value i of `count` values, width w, goes
// to bits [i*w, i*w+w) of dst.  Bits are OR-ed into an LDS staging area
// (order-independent), then copied out with coalesced stores.
template <int ITEMS>
__device__ __forceinline__ void pack_store(const uint32_t (&val)[ITEMS], uint32_t count, uint32_t w,
                                           uint32_t* __restrict__ dst, uint32_t* stage,
                                           uint32_t lane) {
    const uint32_t nwords = words_for(count, w);
    if (nwords == 0) return;
    for (uint32_t k = lane; k < nwords; k += 64) stage[k] = 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        uint32_t i = lane * ITEMS + j;
        uint32_t v = val[j];
        if (i < count && v != 0u) {
            uint32_t bit = i * w;
            uint32_t wd = bit >> 5, sh = bit & 31u;
            atomicOr(&stage[wd], v << sh);
            if (sh + w > 32u) atomicOr(&stage[wd + 1], v >> (32u - sh));
        }
    }
    __syncthreads();
    for (uint32_t k = lane; k < nwords; k += 64) dst[k] = stage[k];
    __syncthreads();
}

// One stable LSD pass over 5 key bits starting at bit `sh` of the key
// (key = kv >> 16).  Each lane counts its own items per digit (LDS atomics on
// its private counter column give the within-lane rank), a raking scan in
// (digit, lane) order gives every (digit, lane) its first slot, and items are
// scattered to their slots and read back blocked.
template <int ITEMS>
__device__ __forceinline__ void radix_pass(uint32_t (&kv)[ITEMS], uint32_t sh, uint32_t nb,
                                           uint32_t lane, uint32_t* cnt, uint32_t* kvbuf) {
    uint4* c4 = reinterpret_cast<uint4*>(cnt);
#pragma unroll
    for (int k = 0; k < 9; k++) c4[lane * 9 + k] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    uint32_t rank[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        uint32_t d = (kv[j] >> (16 + sh)) & (kDigits - 1);
        rank[j] = (lane * ITEMS + j < nb) ? atomicAdd(&cnt[counter_addr(d, lane)], 1u) : 0u;
    }
    __syncthreads();
    {
        // lane r scans flat entries [32r, 32r+32) stored at 36r..36r+31
        uint4* row = reinterpret_cast<uint4*>(cnt + 36 * lane);
        uint32_t c[32];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            uint4 t = row[k];
            c[4 * k + 0] = t.x;
            c[4 * k + 1] = t.y;
            c[4 * k + 2] = t.z;
            c[4 * k + 3] = t.w;
        }
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < 32; k++) {
            uint32_t t = c[k];
            c[k] = run;
            run += t;
        }
        uint32_t before = wave_incl_scan_u32(run) - run;
#pragma unroll
        for (int k = 0; k < 8; k++)
            row[k] = make_uint4(c[4 * k] + before, c[4 * k + 1] + before, c[4 * k + 2] + before,
                                c[4 * k + 3] + before);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        if (lane * ITEMS + j < nb) {
            uint32_t d = (kv[j] >> (16 + sh)) & (kDigits - 1);
            uint32_t dest = cnt[counter_addr(d, lane)] + rank[j];
            kvbuf[pad_addr<ITEMS>(dest)] = kv[j];
        }
    }
    __syncthreads();
    const uint4* mine = reinterpret_cast<const uint4*>(kvbuf + lane * (ITEMS + 4));
#pragma unroll
    for (int k = 0; k < ITEMS / 4; k++) {
        uint4 t = mine[k];
        kv[4 * k + 0] = t.x;
        kv[4 * k + 1] = t.y;
        kv[4 * k + 2] = t.z;
        kv[4 * k + 3] = t.w;
    }
    __syncthreads();
}

template <int ITEMS>
__global__ __launch_bounds__(64) void encode_blocks(EncodeArgs a) {
    constexpr uint32_t B = 64 * ITEMS;
    constexpr uint32_t kKvWords = 64 * (ITEMS + 4);
    constexpr uint32_t kWorkA = kCounterWords > 2 * B + 2 ? kCounterWords : 2 * B + 2;
    constexpr uint32_t kWorkWords = kWorkA > kKvWords ? kWorkA : kKvWords;
    __shared__ __align__(16) uint32_t kvbuf[kKvWords];
    __shared__ __align__(16) uint32_t work[kWorkWords];

    const uint32_t lane = threadIdx.x;
    const uint32_t b = blockIdx.x;
    const uint64_t base = (uint64_t)b * B;
    const uint32_t nb = (uint32_t)((a.n - base) < B ? (a.n - base) : B);
    const uint32_t F = a.F, K = a.K, KF = a.KF;
    uint32_t* __restrict__ rec = a.temp + (uint64_t)b * a.slot_words;
    const uint32_t cap = 1 + F * nb;  // raw record length

    // ---- Stage 1 (Sec. 4.1): key axes -- block minimum, grid index, segment shift
    uint32_t qk[3][ITEMS];
    float lok[3];
    uint32_t sk[3];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        sk[ax] = 0;
        lok[ax] = 0.0f;
        if ((uint32_t)ax < KF) {
            lok[ax] = quantize_field<ITEMS>(a.x[ax], base, nb, lane, a.inv[ax], a.twoeb[ax],
                                            a.eb[ax], qk[ax]);
            uint32_t m = 0;
#pragma unroll
            for (int j = 0; j < ITEMS; j++) m = max(m, qk[ax][j] & 0xFFFFFFu);
            uint32_t W = bit_width(wave_max_u32(m));
            sk[ax] = W > K ? W - K : 0;
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; j++) qk[ax][j] = 0;
        }
    }

    // Linearised segment ID (axis 0 most significant), packed with the index.
    uint32_t kv[ITEMS];
    uint32_t keyor = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        uint32_t key = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ax++)
            if ((uint32_t)ax < KF) key = (key << K) | ((qk[ax][j] & 0xFFFFFFu) >> sk[ax]);
        uint32_t i = lane * ITEMS + j;
        kv[j] = (key << 16) | i;
        if (i < nb) keyor |= key;
    }
    keyor = wave_or_u32(keyor);

    // ---- Stage 2 (Sec. 4.2): stable in-block sort by segment ID
    const uint32_t keybits = K * KF;
    for (uint32_t sh = 0; sh < keybits; sh += kDigitBits) {
        if (((keyor >> sh) & (kDigits - 1)) == 0) continue;  // identity pass
        radix_pass<ITEMS>(kv, sh, nb, lane, work, kvbuf);
    }
    uint32_t key_s[ITEMS], idx_s[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        key_s[j] = kv[j] >> 16;
        idx_s[j] = kv[j] & 0xFFFFu;
    }

    // ---- Stage 3 (Sec. 4.3): run-length coding of the sorted IDs
    uint32_t* uniq = work;
    uint32_t* start = work + B;
    uint32_t prev = (uint32_t)__shfl_up((int)key_s[ITEMS - 1], 1);
    uint32_t nflag = 0;
    bool flag[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        uint32_t p = lane * ITEMS + j;
        uint32_t before = j == 0 ? prev : key_s[j - 1];
        flag[j] = (p < nb) && (p == 0 || key_s[j] != before);
        nflag += flag[j];
    }
    uint32_t incl = wave_incl_scan_u32(nflag);
    const uint32_t U = (uint32_t)__shfl((int)incl, 63);
    {
        uint32_t k = incl - nflag;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            if (flag[j]) {
                uniq[k] = key_s[j];
                start[k] = lane * ITEMS + j;
                k++;
            }
        }
    }
    __syncthreads();
    if (lane == 0) start[U] = nb;
    __syncthreads();
    // delta coding of the distinct IDs (stored as delta - 1) and counts - 1
    uint32_t gap[ITEMS], cnt[ITEMS];
    uint32_t gmax = 0, cmax = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        uint32_t i = lane * ITEMS + j;
        gap[j] = 0;
        cnt[j] = 0;
        if (i < U) {
            uint32_t u = uniq[i];
            uint32_t up = i ? uniq[i - 1] : 0xFFFFFFFFu;
            gap[j] = u - up - 1u;
            cnt[j] = start[i + 1] - start[i] - 1u;
        }
        gmax = max(gmax, gap[j]);
        cmax = max(cmax, cnt[j]);
    }
    const uint32_t w_gap = bit_width(wave_max_u32(gmax));
    const uint32_t w_cnt = bit_width(wave_max_u32(cmax));
    __syncthreads();

    uint32_t pos = 2;
    bool over = false;
    {
        uint32_t gw = words_for(U, w_gap), cw = words_for(U, w_cnt);
        if (pos + gw + cw > cap) {
            over = true;
        } else {
            if (lane == 0) {
                rec[0] = U << 2;
                rec[1] = w_gap | (w_cnt << 5) | (sk[0] << 10) | (sk[1] << 15) | (sk[2] << 20);
            }
            pack_store<ITEMS>(gap, U, w_gap, rec + pos, kvbuf, lane);
            pack_store<ITEMS>(cnt, U, w_cnt, rec + pos + gw, kvbuf, lane);
        }
        pos += gw + cw;
    }

    // ---- per field: fixed-length payload in sorted order + outlier list
    for (uint32_t f = 0; f < F && !over; f++) {
        uint32_t q[ITEMS];
        float lo;
        uint32_t mask;
        if (f < KF) {
            // f is 0, 1 or 2 here; pick the registers without dynamic indexing
#pragma unroll
            for (int j = 0; j < ITEMS; j++) q[j] = f == 0 ? qk[0][j] : (f == 1 ? qk[1][j] : qk[2][j]);
            lo = f == 0 ? lok[0] : (f == 1 ? lok[1] : lok[2]);
            uint32_t s = f == 0 ? sk[0] : (f == 1 ? sk[1] : sk[2]);
            mask = (1u << s) - 1u;
        } else {
            lo = quantize_field<ITEMS>(a.x[f], base, nb, lane, a.inv[f], a.twoeb[f], a.eb[f], q);
            mask = 0xFFFFFFu;
        }
        uint32_t vmax = 0, nout = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            vmax = max(vmax, q[j] & mask);
            nout += q[j] >> 31;
        }
        const uint32_t w = bit_width(wave_max_u32(vmax));
        const uint32_t nout_all = wave_sum_u32(nout);
        const uint32_t pw = words_for(nb, w);
        const uint32_t sec = 2 + pw + 2 * nout_all;
        if (pos + sec > cap) {
            over = true;
            break;
        }
        if (lane == 0) {
            rec[pos] = f2u(lo);
            rec[pos + 1] = w | (nout_all << 5);
        }
        // permute to sorted order through LDS
        uint4* mine = reinterpret_cast<uint4*>(work + lane * (ITEMS + 4));
#pragma unroll
        for (int k = 0; k < ITEMS / 4; k++)
            mine[k] = make_uint4(q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]);
        __syncthreads();
        uint32_t qs[ITEMS], vs[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            qs[j] = (lane * ITEMS + j < nb) ? work[pad_addr<ITEMS>(idx_s[j])] : 0u;
            vs[j] = qs[j] & mask;
        }
        __syncthreads();
        pack_store<ITEMS>(vs, nb, w, rec + pos + 2, kvbuf, lane);
        if (nout_all) {
            uint32_t c = 0;
#pragma unroll
            for (int j = 0; j < ITEMS; j++) c += qs[j] >> 31;
            uint32_t k = wave_incl_scan_u32(c) - c;
            uint32_t* ol = rec + pos + 2 + pw;
            const float* xf = a.x[f] + base;
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                if (qs[j] >> 31) {
                    ol[2 * k] = lane * ITEMS + j;
                    ol[2 * k + 1] = f2u(xf[idx_s[j]]);
                    k++;
                }
            }
        }
        pos += sec;
    }

    const bool raw = over || pos >= cap;
    if (raw) {
        // Raw form: the block's floats verbatim, field-major, input order.
        // The barrier orders these stores after the coded ones they replace.
        __syncthreads();
        if (lane == 0) rec[0] = 1u;
        for (uint32_t f = 0; f < F; f++) {
            const float* xf = a.x[f] + base;
            uint32_t* dst = rec + 1 + f * nb;
            for (uint32_t i = lane; i < nb; i += 64) dst[i] = f2u(xf[i]);
        }
    }
    if (lane == 0) a.lens[b] = raw ? cap : pos;
    if (a.perm) {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t p = lane * ITEMS + j;
            if (p < nb) a.perm[base + p] = (uint32_t)(base + (raw ? p : idx_s[j]));
        }
    }
}

}  // namespace

hipError_t launch_encode(const EncodeArgs& a, hipStream_t s) {
    if (a.nblocks == 0) return hipSuccess;
    dim3 grid(a.nblocks), block(64);
    switch (a.B) {
        case 256: hipLaunchKernelGGL(encode_blocks<4>, grid, block, 0, s, a); break;
        case 512: hipLaunchKernelGGL(encode_blocks<8>, grid, block, 0, s, a); break;
        case 1024: hipLaunchKernelGGL(encode_blocks<16>, grid, block, 0, s, a); break;
        case 2048: hipLaunchKernelGGL(encode_blocks<32>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gpz
