// Block decoder (Sec. 3.2: decompression reverses the compression steps,
// without un-sorting): one wave64 per block locates its record through the
// superblock table, undoes the delta and run-length coding of the segment
// IDs, unpacks the fixed-length payloads, rebuilds every value with
// fma(q, 2eb, lo), patches outliers and stores the block in sorted order.
//
// Each coded array is first copied into LDS with coalesced loads; values are
// then extracted from LDS.  Outputs are written "striped": lane l produces
// positions 256k + 4l + {0..3}, so one 16-byte store per lane covers 1 KB of
// contiguous output per instruction.  One wave per workgroup: LDS traffic
// between its lanes is ordered by wave_lds_sync().  Every read of the record
// is checked against its length first; a malformed record sets the error
// flag and the block is skipped.
#include "generic_block.h"

namespace gpz {
namespace {

template <int ITEMS>
__device__ __forceinline__ uint32_t pad_addr(uint32_t p) {
    return p + 4 * (p / ITEMS);
}

__device__ __forceinline__ bool eb_ok(float eb) {
    return __builtin_isfinite(eb) && eb >= 0x1p-120f && eb <= 0x1p120f;
}

// Copy `count` words (at most 64*L) from global memory into LDS with
// coalesced loads, all issued before the first LDS store, so the copy costs
// one memory round trip.  The number of 64-word steps selects a fully
// unrolled copy (a wave-uniform choice); inside the last step the lanes past
// the end load the array's last word again (so every load stays in bounds)
// and store it past the end, where the buffer still has room.  Offsets are
// 32-bit byte offsets from the array start, so each load takes the array's
// scalar base address and one offset register.
template <int N>
__device__ __forceinline__ void stage_steps(uint32_t* __restrict__ dst,
                                            const uint32_t* __restrict__ src, uint32_t count,
                                            uint32_t ln) {
    const uint8_t* b = reinterpret_cast<const uint8_t*>(src);
    uint32_t t[N];
#pragma unroll
    for (int u = 0; u < N; u++)
        t[u] = *reinterpret_cast<const uint32_t*>(b + 4u * min(ln + 64u * u, count - 1));
#pragma unroll
    for (int u = 0; u < N; u++) dst[ln + 64u * u] = t[u];
}

template <int N>
__device__ __forceinline__ void stage_pick(uint32_t steps, uint32_t* __restrict__ dst,
                                           const uint32_t* __restrict__ src, uint32_t count,
                                           uint32_t ln) {
    if constexpr (N > 0) {
        if (steps == N) stage_steps<N>(dst, src, count, ln);
        else stage_pick<N - 1>(steps, dst, src, count, ln);
    }
}

template <int L>
__device__ __forceinline__ void stage_words(uint32_t* __restrict__ dst,
                                            const uint32_t* __restrict__ src, uint32_t count,
                                            uint32_t lane) {
    if (count == 0) return;
    stage_pick<L>((count + 63) / 64, dst, src, count, lane);
}

// Value i of a fixed-length array of width w held in LDS (bits [i*w, i*w+w)).
__device__ __forceinline__ uint32_t extract(const uint32_t* __restrict__ words, uint32_t i,
                                            uint32_t w, uint32_t mask) {
    uint32_t bit = i * w;
    uint32_t wd = bit >> 5;
    uint32_t lo = words[wd], hi = words[wd + 1];
    return __builtin_amdgcn_alignbit(hi, lo, bit & 31u) & mask;
}

__device__ __forceinline__ uint32_t low_mask(uint32_t w) { return w >= 32u ? ~0u : ((1u << w) - 1u); }

// Sum over the wave of one 64-bit value per lane (every lane gets it).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Whether the stream's header or eb table does not describe the stream the
// caller asked for (lane k < 8 checks header word k, every lane a share of
// the eb table).  Per-lane result.
__device__ __forceinline__ bool header_bad(const DecodeArgs& a, uint32_t lane) {
    bool bad = false;
    const uint32_t* ebt = a.in + kHeaderWords + 2 * nsuper_of(a.nblocks);
    for (uint32_t f = lane; f < a.F; f += 64)
        if (!eb_ok(u2f(ebt[f]))) bad = true;
    if (lane < kHeaderWords) {
        const uint32_t expect[kHeaderWords] = {kMagic, kVersion, (uint32_t)(a.n & 0xFFFFFFFFu),
                                               (uint32_t)(a.n >> 32), a.F, a.B,
                                               a.K | (a.KF << 8), a.nblocks};
        uint32_t want = expect[0];
#pragma unroll
        for (uint32_t k = 1; k < kHeaderWords; k++) want = lane == k ? expect[k] : want;
        // word 1 may carry the wide-record flag (a float32 stream otherwise)
        const uint32_t got = lane == 1 ? (a.in[lane] & ~(2u << 16)) : a.in[lane];
        if (got != want) bad = true;
    }
    return bad;
}

template <int ITEMS>
struct DecodeSmem {
    static constexpr uint32_t B = 64 * ITEMS;
    // widest coded arrays: payload 24 bits/value; gaps 15 + counts 12 bits
    static constexpr uint32_t kPay = (B * 24) / 32 + 2;
    static constexpr uint32_t kRle = (B * 15) / 32 + (B * 12) / 32 + 4;
    static constexpr uint32_t kWords = ((kPay > kRle ? kPay : kRle) + 3) & ~3u;  // 16-byte multiple
    static constexpr uint32_t kPadB = 64 * (ITEMS + 4);
    // The packed words, the key expansion and the outlier staging are never
    // live at the same time: one region serves all three (barriers between
    // the phases), which keeps the workgroup's LDS small enough for high
    // occupancy.
    static constexpr uint32_t kA = kWords > kPadB ? kWords : kPadB;
    static constexpr uint32_t kBuf = kA > B ? kA : B;
    // 64-word steps of the widest array, which stage_words fills whole
    static constexpr int kSteps = (int)((kWords + 63) / 64);
    static_assert(64 * kSteps <= kBuf, "staged steps stay inside buf");
    uint32_t buf[kBuf];
};

// The decoder's LDS: its own buffer, or the generic record decoder's when a
// record holds a field coded with 64-bit steps.
template <int ITEMS>
union DecodeShared {
    DecodeSmem<ITEMS> fast;
    GenDecodeSmem<64 * ITEMS> wide;
};

template <int ITEMS>
__device__ __forceinline__ void decode_block(const DecodeArgs& a, uint32_t b,
                                             DecodeShared<ITEMS>& shared) {
    DecodeSmem<ITEMS>& sm = shared.fast;
    constexpr uint32_t B = 64 * ITEMS;
    constexpr uint32_t G = ITEMS / 4;  // 16-byte groups per lane
    uint32_t* words = sm.buf;
    uint32_t* keys = sm.buf;
    uint32_t* ystage = sm.buf;

    const uint32_t lane = threadIdx.x;
    const uint64_t base = (uint64_t)b * B;
    const uint32_t nb = (uint32_t)((a.n - base) < B ? (a.n - base) : B);
    const uint32_t F = a.F, K = a.K, KF = a.KF;
    const uint64_t nsup = nsuper_of(a.nblocks);
    const uint32_t* sup = a.in + kHeaderWords;
    const uint32_t* ebt = sup + 2 * nsup;
    const uint32_t* lens = ebt + F;
    const uint32_t* recs = a.in + a.prefix;
    const uint64_t rec_total = a.in_words - a.prefix;

    // ---- locate the record: superblock offset + lengths before it.  The
    // superblock entry is checked against the record area before anything is
    // added to it, and the lengths are summed in 64 bits, so no sum can wrap
    // and every accepted [off, off + len) lies inside the record area.
    const uint32_t sb = b / kSuper;
    const uint32_t first = sb * kSuper;
    const uint64_t sup_off = (uint64_t)sup[2 * sb] | ((uint64_t)sup[2 * sb + 1] << 32);
    const uint64_t mine = (first + lane < b) ? (uint64_t)lens[first + lane] : 0ull;
    const uint64_t sum = sup_off + wave_sum_u64(mine);
    // every lane holds the same sum: taken from lane 0 it is a scalar, and so
    // are the record pointer and every header word read through it
    const uint64_t off = ((uint64_t)readlane((uint32_t)(sum >> 32), 0) << 32) |
                         (uint64_t)readlane((uint32_t)sum, 0);
    const uint32_t len = lens[b];
    bool bad = sup_off > rec_total || off > rec_total || (uint64_t)len > rec_total - off;
    if (b == 0 && (sup[0] | sup[1]) != 0u) bad = true;
    if (a.exact && b + 1 == a.nblocks && off + len != rec_total) bad = true;
    if (header_bad(a, lane)) bad = true;
    if (b == first && sb > 0) {
        // consistency of this superblock's offset with the previous one
        const uint64_t pl = lens[first - kSuper + lane];
        const uint64_t prev = ((uint64_t)sup[2 * sb - 2] | ((uint64_t)sup[2 * sb - 1] << 32));
        if (prev > rec_total || prev + wave_sum_u64(pl) != off) bad = true;
    }
    if (__any(bad)) {
        if (lane == 0) *a.err = 1u;
        return;
    }
    const uint32_t* rec = recs + off;
    const uint32_t h0 = len ? rec[0] : 0u;
    const uint32_t mode = h0 & 3u;

    if (len != 0 && mode == 0 && (h0 >> 31)) {
        // a field coded with 64-bit steps (Sec. 5.3): the generic record
        // decoder, run by this wave, when the header announces such records
        // (corrupt otherwise)
        if (!((a.in[1] >> 17) & 1u)) {
            if (lane == 0) *a.err = 1u;
            return;
        }
        gen_decode_record<64 * ITEMS, 64, false>(a, b, rec, len, shared.wide);
        return;
    }
    if (len == 0 || mode > 1) {
        if (lane == 0) *a.err = 1u;
        return;
    }
    if (mode == 1) {
        if (h0 != 1u || len != 1 + F * nb) {
            if (lane == 0) *a.err = 1u;
            return;
        }
        for (uint32_t f = 0; f < F; f++) {
            float* yf = a.y[f] + base;
            const uint32_t* src = rec + 1 + f * nb;
            for (uint32_t i = lane; i < nb; i += 64) yf[i] = u2f(src[i]);
        }
        return;
    }

    // ---- coded record header
    const uint32_t U = h0 >> 2;
    const uint32_t h1 = len > 1 ? rec[1] : 0xFFFFFFFFu;
    const uint32_t w_gap = h1 & 31u, w_cnt = (h1 >> 5) & 31u;
    const uint32_t s0 = (h1 >> 10) & 31u, s1 = (h1 >> 15) & 31u, s2 = (h1 >> 20) & 31u;
    bad = len < 2 || (h1 >> 25) != 0u || U < 1 || U > nb || w_gap > 15 || w_cnt > 12;
    bad |= (KF < 2 && s1 != 0) || (KF < 3 && s2 != 0);
    bad |= (s0 + K > 24) || (KF > 1 && s1 + K > 24) || (KF > 2 && s2 + K > 24);
    const uint32_t gw = words_for(U, w_gap), cw = words_for(U, w_cnt);
    bad |= (uint64_t)2 + gw + cw > len;
    if (bad) {
        if (lane == 0) *a.err = 1u;
        return;
    }

    // ---- undo delta + run-length coding (Sec. 4.3)
    stage_words<DecodeSmem<ITEMS>::kSteps>(words, rec + 2, gw + cw, lane);
    wave_lds_sync();
    uint32_t g1[ITEMS], c1[ITEMS];
    uint32_t gs = 0, cs = 0;
    {
        const uint32_t gm = low_mask(w_gap), cm = low_mask(w_cnt);
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t i = lane * ITEMS + j;
            g1[j] = i < U ? extract(words, i, w_gap, gm) + 1u : 0u;
            c1[j] = i < U ? extract(words + gw, i, w_cnt, cm) + 1u : 0u;
            gs += g1[j];
            cs += c1[j];
        }
    }
    const uint32_t gincl = wave_incl_scan_u32(gs), cincl = wave_incl_scan_u32(cs);
    const uint32_t gtot = (uint32_t)__shfl((int)gincl, 63), ctot = (uint32_t)__shfl((int)cincl, 63);
    // largest ID = sum(gap+1) - 1 must fit K*KF bits; run lengths sum to nb
    if (ctot != nb || gtot == 0 || gtot - 1u >= (1u << (K * KF))) {
        if (lane == 0) *a.err = 1u;
        return;
    }
    // mark run starts with their ID; IDs increase with position, so a prefix
    // maximum over positions gives every position its ID
    wave_lds_sync();  // the packed gaps and counts are read; `keys` reuses them
    for (uint32_t p = lane; p < B; p += 64) keys[pad_addr<ITEMS>(p)] = 0u;
    wave_lds_sync();
    {
        uint32_t u = gincl - gs, st = cincl - cs;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t i = lane * ITEMS + j;
            if (i < U) {
                u += g1[j];
                keys[pad_addr<ITEMS>(st)] = u - 1u;
                st += c1[j];
            }
        }
    }
    wave_lds_sync();
    {
        uint32_t key[ITEMS];
        uint32_t run = 0;
        const uint4* kb = reinterpret_cast<const uint4*>(keys + lane * (ITEMS + 4));
#pragma unroll
        for (int g = 0; g < G; g++) {
            uint4 t = kb[g];
            run = max(run, t.x);
            key[4 * g + 0] = run;
            run = max(run, t.y);
            key[4 * g + 1] = run;
            run = max(run, t.z);
            key[4 * g + 2] = run;
            run = max(run, t.w);
            key[4 * g + 3] = run;
        }
        uint32_t carry = wave_incl_max_u32(run);
        carry = (uint32_t)__shfl_up((int)carry, 1);
        if (lane == 0) carry = 0;
        wave_lds_sync();
        uint4* kw = reinterpret_cast<uint4*>(keys + lane * (ITEMS + 4));
#pragma unroll
        for (int g = 0; g < G; g++)
            kw[g] = make_uint4(max(key[4 * g], carry), max(key[4 * g + 1], carry),
                               max(key[4 * g + 2], carry), max(key[4 * g + 3], carry));
    }
    wave_lds_sync();
    // striped positions of this lane: p = 256 g + 4 lane + e
    uint32_t skey[ITEMS];
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int e = 0; e < 4; e++) skey[4 * g + e] = keys[pad_addr<ITEMS>(256 * g + 4 * lane + e)];

    // ---- fields
    uint64_t pos = 2 + gw + cw;
    const bool full = nb == B;
    for (uint32_t f = 0; f < F; f++) {
        if (pos + 2 > len) {
            bad = true;
            break;
        }
        const float lo = u2f(rec[pos]);
        const uint32_t wn = rec[pos + 1];
        const uint32_t w = wn & 31u, nout = wn >> 5;
        uint32_t s = 0, shift = 0;
        if (f < KF) {
            s = f == 0 ? s0 : (f == 1 ? s1 : s2);
            shift = K * (KF - 1 - f);
        }
        const uint32_t wlim = f < KF ? s : 24u;
        const uint32_t pw = words_for(nb, w);
        if (w > wlim || nout > nb || pos + 2 + pw + 2 * (uint64_t)nout > len) {
            bad = true;
            break;
        }
        const float twoeb = 2.0f * u2f(ebt[f]);
        wave_lds_sync();  // previous users of `words` are done
        stage_words<DecodeSmem<ITEMS>::kSteps>(words, rec + pos + 2, pw, lane);
        wave_lds_sync();
        const uint32_t mask = low_mask(w);
        uint32_t y[ITEMS];
        if (f < KF) {
            // a key field's code: the position's segment (its K bits of the
            // ID) above the s stored offset bits
#pragma unroll
            for (int g = 0; g < G; g++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint32_t p = 256 * g + 4 * lane + e;
                    const uint32_t v = extract(words, p, w, mask);
                    const uint32_t q = (__builtin_amdgcn_ubfe(skey[4 * g + e], shift, K) << s) | v;
                    y[4 * g + e] = f2u(__builtin_fmaf((float)q, twoeb, lo));
                }
        } else {
#pragma unroll
            for (int g = 0; g < G; g++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint32_t p = 256 * g + 4 * lane + e;
                    const uint32_t v = extract(words, p, w, mask);
                    y[4 * g + e] = f2u(__builtin_fmaf((float)v, twoeb, lo));
                }
        }
        if (nout) {
            // patch outliers through LDS (the staging reuses `words`)
            const uint32_t* ol = rec + pos + 2 + pw;
            wave_lds_sync();
#pragma unroll
            for (int g = 0; g < G; g++)
                reinterpret_cast<uint4*>(ystage)[64 * g + lane] =
                    make_uint4(y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]);
            wave_lds_sync();
            bool obad = false;
            for (uint32_t k = lane; k < nout; k += 64) {
                uint32_t op = ol[2 * k];
                uint32_t prevp = k ? ol[2 * k - 2] : 0u;
                if (op >= nb || (k && prevp >= op)) obad = true;
                else ystage[op] = ol[2 * k + 1];
            }
            if (__any(obad)) {
                bad = true;
                break;
            }
            wave_lds_sync();
#pragma unroll
            for (int g = 0; g < G; g++) {
                uint4 t = reinterpret_cast<const uint4*>(ystage)[64 * g + lane];
                y[4 * g] = t.x;
                y[4 * g + 1] = t.y;
                y[4 * g + 2] = t.z;
                y[4 * g + 3] = t.w;
            }
        }
        float* yf = a.y[f] + base;
        if (full && ((reinterpret_cast<uintptr_t>(a.y[f]) & 15u) == 0)) {
#pragma unroll
            for (int g = 0; g < G; g++) {
                u32x4 t = {y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]};
                __builtin_nontemporal_store(t, reinterpret_cast<u32x4*>(yf + 256 * g + 4 * lane));
            }
        } else {
#pragma unroll
            for (int g = 0; g < G; g++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint32_t p = 256 * g + 4 * lane + e;
                    if (p < nb) yf[p] = u2f(y[4 * g + e]);
                }
        }
        pos += 2 + pw + 2 * (uint64_t)nout;
    }
    if (bad || pos != len) {
        if (lane == 0) *a.err = 1u;
    }
}

template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void decode_blocks(DecodeArgs a) {
    __shared__ __align__(16) DecodeShared<ITEMS> sm;
    decode_block<ITEMS>(a, blockIdx.x, sm);
}

// Persistent decoder over the blocks of many streams: each wave takes `tile`
// consecutive blocks from a device work queue until the queue is empty.
template <int ITEMS>
__global__ __launch_bounds__(64) void decode_batch(const DecodeArgs* __restrict__ jobs,
                                                   const BatchLaunch* __restrict__ L) {
    __shared__ __align__(16) DecodeShared<ITEMS> sm;
    const uint32_t total = L->total_blocks, njobs = L->njobs, tile = L->tile;
    const uint32_t* prefix = L->block_prefix;
    for (;;) {
        uint32_t item = 0;
        if (threadIdx.x == 0) item = atomicAdd(L->counter + 1, tile);
        item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
        if (item >= total) break;
        const uint32_t end = min(item + tile, total);
        for (uint32_t g = item; g < end; g++) {
            const uint32_t j = find_job(prefix, njobs, g);
            decode_block<ITEMS>(jobs[j], g - prefix[j], sm);
            __syncthreads();
        }
    }
}

// Direct form of decode_batch: one workgroup per block of the batch's
// capacity (no loop around the block, so a smaller register budget).
template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(ITEMS == 32 ? 3 : 8))) void decode_batch_direct(const DecodeArgs* __restrict__ jobs,
                                                          const BatchLaunch* __restrict__ L) {
    __shared__ __align__(16) DecodeShared<ITEMS> sm;
    const uint32_t g = blockIdx.x;
    if (g >= L->total_blocks) return;
    const uint32_t* prefix = L->block_prefix;
    const uint32_t j = find_job(prefix, L->njobs, g);
    decode_block<ITEMS>(jobs[j], g - prefix[j], sm);
}

// A stream of a snapshot with no particles holds only its header, its
// superblock table (empty) and its eb table: one wave checks them, so the
// caller needs no host copy of the stream.
__global__ __launch_bounds__(64) void check_empty_stream(DecodeArgs a) {
    const uint32_t lane = threadIdx.x;
    bool bad = header_bad(a, lane);
    if (a.exact && a.in_words != a.prefix) bad = true;
    if (__any(bad) && lane == 0) *a.err = 1u;
}

}  // namespace

hipError_t launch_decode_batch(const DecodeArgs* jobs, const BatchLaunch* L,
                               const BatchShape& S, hipStream_t s) {
    dim3 block(64);
    if (S.grid) {
        dim3 grid(S.grid);
        switch (S.B) {
            case 256: hipLaunchKernelGGL(decode_batch<4>, grid, block, 0, s, jobs, L); break;
            case 512: hipLaunchKernelGGL(decode_batch<8>, grid, block, 0, s, jobs, L); break;
            case 1024: hipLaunchKernelGGL(decode_batch<16>, grid, block, 0, s, jobs, L); break;
            case 2048: hipLaunchKernelGGL(decode_batch<32>, grid, block, 0, s, jobs, L); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        dim3 grid(S.direct_grid);
        switch (S.B) {
            case 256: hipLaunchKernelGGL(decode_batch_direct<4>, grid, block, 0, s, jobs, L); break;
            case 512: hipLaunchKernelGGL(decode_batch_direct<8>, grid, block, 0, s, jobs, L); break;
            case 1024: hipLaunchKernelGGL(decode_batch_direct<16>, grid, block, 0, s, jobs, L); break;
            case 2048: hipLaunchKernelGGL(decode_batch_direct<32>, grid, block, 0, s, jobs, L); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs& a, hipStream_t s) {
    if (a.nblocks == 0) {
        hipLaunchKernelGGL(check_empty_stream, dim3(1), dim3(64), 0, s, a);
        return hipGetLastError();
    }
    dim3 grid(a.nblocks), block(64);
    switch (a.B) {
        case 256: hipLaunchKernelGGL(decode_blocks<4>, grid, block, 0, s, a); break;
        case 512: hipLaunchKernelGGL(decode_blocks<8>, grid, block, 0, s, a); break;
        case 1024: hipLaunchKernelGGL(decode_blocks<16>, grid, block, 0, s, a); break;
        case 2048: hipLaunchKernelGGL(decode_blocks<32>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gpz
