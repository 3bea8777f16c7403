// Block encoder: GPZ stages 1-3 (Sec. 4.1 quantization, Sec. 4.2 in-block
// sort, Sec. 4.3 run-length / delta / fixed-length coding) for one block of
// B particles per wave64, writing the block's record into its workspace slot
// and its length (first step of the Sec. 4.4 compaction; the scan and copy
// kernels finish it).  An alternative single-pass compaction is also built:
// the block publishes its length, finds its offset in the stream by a
// decoupled look-back over the lengths of the blocks before it, and copies
// its record there itself.
//
// Lane layout: lane l owns the ITEMS = B/64 consecutive particles
// [l*ITEMS, (l+1)*ITEMS) of its block ("blocked"), so per-lane sequential
// order followed by lane order is input order; that is what makes the LDS
// radix sort stable.  One wave per workgroup: LDS traffic between lanes is
// ordered by wave_lds_sync(), which waits for nothing (a wave's LDS
// operations execute in issue order); __syncthreads() remains only where
// global-memory stores of the block must be ordered.  Full blocks take a path
// without per-item bounds checks; only the last block of a snapshot can be
// partial.
#include "gpz_internal.h"

namespace gpz {
namespace {

constexpr uint32_t kDigitBits = 5;
constexpr uint32_t kDigits = 1u << kDigitBits;
// Digit counters, digit-major: (d, lane) at d*68 + lane (4 pad words per
// digit row, so that the raking scan's 16-byte reads spread over the banks).
// The address is one multiply-add of the digit; the clearing loop writes
// 2304 words (nine 16-byte stores per lane), past the 2176 used.
constexpr uint32_t kRow = 68;
constexpr uint32_t kCounterWords = 64 * 9 * 4;
static_assert(kDigits * kRow <= kCounterWords, "counter rows fit the cleared region");

__device__ __forceinline__ uint32_t counter_addr(uint32_t d, uint32_t lane) {
    return d * kRow + lane;
}

// Padded blocked layout: position p of a block lives at p + 4*(p / ITEMS), so
// lane l's ITEMS consecutive positions start at l*(ITEMS+4) (16-byte aligned,
// spread over the banks).
template <int ITEMS>
__device__ __forceinline__ uint32_t pad_addr(uint32_t p) {
    return p + 4 * (p / ITEMS);
}

// Sort items carry (segment ID << 16) | byte offset of the particle's word
// in the padded blocked layout, so that the per-field permutation reads take
// their LDS address straight from the item.  Once the runs are coded the
// segment IDs are cleared from the items, which leaves the offset alone.
__device__ __forceinline__ uint32_t staged_at(const uint32_t* work, uint32_t offset) {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(work) + offset);
}

// The particle index of an item: padded word p + 4*(p/ITEMS) back to p.
template <int ITEMS>
__device__ __forceinline__ uint32_t index_of(uint32_t item) {
    const uint32_t w = (item & 0xFFFFu) >> 2;
    return w - 4u * (w / (ITEMS + 4));
}

// Quantizer: t = (x - lo) * inv (two IEEE float ops), q = rint(t) when t lies
// in [0, 2^24-1] (else 0); the value stays on the grid only when the float32
// error of xr = fma(q, 2eb, lo) is below eb (which bounds the exact error
// strictly), otherwise it is an outlier stored verbatim.
__device__ __forceinline__ uint32_t quantize(float x, float lo, float inv, float twoeb, float eb,
                                             bool& outlier, bool& in) {
    float t = (x - lo) * inv;
    in = (t >= 0.0f) && (t <= kQMax);
    uint32_t q = in ? (uint32_t)__builtin_rintf(t) : 0u;
    float xr = __builtin_fmaf((float)q, twoeb, lo);
    bool ok = in && (__builtin_fabsf(xr - x) < eb);
    outlier = !ok;
    return q;
}

template <int ITEMS, bool FULL>
__device__ __forceinline__ void load_block(const float* __restrict__ x, uint64_t base, uint32_t nb,
                                           uint32_t lane, float (&v)[ITEMS]) {
    const float* p = x + base + (uint64_t)lane * ITEMS;
    if (FULL && ((reinterpret_cast<uintptr_t>(x) & 15u) == 0)) {
        const f32x4* p4 = reinterpret_cast<const f32x4*>(p);
#pragma unroll
        for (int k = 0; k < ITEMS / 4; k++) {
            f32x4 t = p4[k];  // cached loads: measured faster than non-temporal ones
            v[4 * k + 0] = t.x;
            v[4 * k + 1] = t.y;
            v[4 * k + 2] = t.z;
            v[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t i = lane * ITEMS + j;
            v[j] = (FULL || i < nb) ? p[j] : 0.0f;
        }
    }
}

// A field of the block after quantization: its minimum lo, the largest code
// over the block's particles, whether no value is an outlier, and whether a
// finite value lies beyond 2^24 - 1 grid steps (the field then needs 64-bit
// steps, Sec. 5.3, which the generic encoder takes).
struct FieldCodes {
    float lo;
    uint32_t qmax;
    bool clean;
    bool wide;
};

// Quantize one field of the block (Sec. 4.1).  Codes are returned as q per
// value for a field without outliers (`clean`), as 2*q + outlier otherwise
// (0 beyond the block).
//
// Fast path, exact for a field without outliers.  Every finite value lies at
// or above the block minimum lo, so t = (x - lo) * inv is never below -0, and
// because no float32 lies strictly between 2^24-1 and 2^24, t <= 2^24-1 holds
// exactly when rint(t) <= 2^24-1.  So a value is on the grid exactly when the
// float32 error of fma(rint(t), 2eb, lo) is below eb and rint(t) does not
// exceed 2^24-1 (a t out of range is NaN, infinite or at least 2^24, and
// fails one of the two).  With q = rint(t) for every value of the field,
// fma(q, 2eb, lo) is the reconstruction the quantizer defines (q = -0 and
// q = +0 give the same result, as lo is never -0).  When any value fails,
// the whole field is quantized again with the quantizer's own steps.
template <int ITEMS, bool FULL>
__device__ __forceinline__ FieldCodes quantize_field(const float (&v)[ITEMS], uint32_t nb,
                                                     uint32_t lane, float inv, float twoeb,
                                                     float eb, uint32_t (&q)[ITEMS]) {
    // Block minimum over the finite values.  +inf is the minimum's identity,
    // so only NaN and -inf have to be skipped: a minimum that propagates NaN
    // over the raw values ends up NaN or -inf in some lane exactly when the
    // block holds one of them, and only then are values filtered one by one.
    // The test is a class test (signalling NaN, quiet NaN, -inf): the
    // compiler lowered the equivalent `m > -inf` under a wave vote to an
    // unordered compare, which a NaN passes.
    float m = __builtin_inff();
#pragma unroll
    for (int j = 0; j < ITEMS; j++)
        m = __builtin_elementwise_minimum(
            m, (FULL || lane * ITEMS + j < nb) ? v[j] : __builtin_inff());
    if (__any(__builtin_amdgcn_classf(m, 7))) {
        m = __builtin_inff();
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            bool ok = (FULL || lane * ITEMS + j < nb) && __builtin_isfinite(v[j]);
            m = fminf(m, ok ? v[j] : __builtin_inff());
        }
    }
    m = wave_min_f32(m);
    const float lo = (m == __builtin_inff() || m == 0.0f) ? 0.0f : m;
    // Every error is below eb exactly when the largest one is.  The maximum
    // propagates NaN (a non-finite value's error), which then fails the test
    // like the value's own comparison would; it takes two errors per
    // instruction where a per-value flag took a compare and a select.
    float emax = 0.0f;
    float rmax = 0.0f;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const bool valid = FULL || lane * ITEMS + j < nb;
        const float r = __builtin_rintf((v[j] - lo) * inv);
        const float xr = __builtin_fmaf(r, twoeb, lo);
        emax = __builtin_elementwise_maximum(emax, valid ? __builtin_fabsf(xr - v[j]) : 0.0f);
        rmax = fmaxf(rmax, valid ? r : 0.0f);
        q[j] = valid ? (uint32_t)r : 0u;
    }
    uint32_t qmax = wave_max_u32(rmax <= kQMax ? (uint32_t)rmax : 0xFFFFFFFFu);
    if (__all(emax < eb) && qmax <= 0xFFFFFFu) return {lo, qmax, true, false};
    // some value is an outlier: the quantizer's steps, value by value
    uint32_t mx = 0;
    bool far = false;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const bool valid = FULL || lane * ITEMS + j < nb;
        bool o, in;
        const uint32_t qq = quantize(v[j], lo, inv, twoeb, eb, o, in);
        q[j] = valid ? (qq << 1) | (uint32_t)o : 0u;
        mx = max(mx, valid ? qq : 0u);
        far = far || (valid && !in && __builtin_isfinite(v[j]));
    }
    qmax = wave_max_u32(mx);
    return {lo, qmax, false, __any(far) != 0};
}

// Fixed-length packing (Sec. 4.3): value i of `count` values of width w
// (1 <= w <= 24) goes to bits [i*w, i*w+w) of dst.  Lane l packs its ITEMS
// consecutive values (blocked in v).  Bit positions inside the lane's
// segment, j*w, are the same for every lane, so the lane accumulates into one
// register and flushes on wave-uniform branches; each completed segment word
// is shifted to the lane's start bit with one 64-bit shift and stored into
// LDS staging.  The lane owning bit 0 of a word stores it; a lane whose
// segment starts inside a word ORs its part in after a barrier.  The staged
// words are then copied to dst with coalesced stores.
template <int ITEMS>
__device__ __forceinline__ void pack_generic(const uint32_t (&v)[ITEMS], uint32_t nwords,
                                             uint32_t count, uint32_t w, uint32_t* stage,
                                             uint32_t lane) {
    const bool active = lane * ITEMS < count;
    const uint32_t S = lane * ITEMS * w;            // first bit of the lane's segment
    const uint32_t w0 = S >> 5, shl = S & 31u;
    const uint32_t lastw = (S + ITEMS * w - 1) >> 5;  // last word the segment touches
    uint32_t acc = 0u, prev = 0u, first = 0u;
    uint32_t k = 0, pos = 0;  // segment word index and bit position in it (uniform)
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        acc |= v[j] << pos;
        pos += w;
        if (pos >= 32u) {
            const uint32_t gi = w0 + k;
            const uint32_t word = (uint32_t)((((uint64_t)acc << 32) | prev) >> (32u - shl));
            if (active && gi < nwords && (k > 0 || shl == 0)) stage[gi] = word;
            if (k == 0) first = acc;
            prev = acc;
            pos -= 32u;
            acc = pos ? v[j] >> (w - pos) : 0u;
            k++;
        }
    }
    if (pos > 0u) {  // last, partly filled segment word
        const uint32_t gi = w0 + k;
        const uint32_t word = (uint32_t)((((uint64_t)acc << 32) | prev) >> (32u - shl));
        if (active && gi < nwords && (k > 0 || shl == 0)) stage[gi] = word;
        if (k == 0) first = acc;
        prev = acc;
        k++;
    }
    if (shl != 0u) {  // spill-over of the segment's top bits into one more word
        const uint32_t gi = w0 + k;
        if (active && gi <= lastw && gi < nwords) stage[gi] = prev >> (32u - shl);
    }
    wave_lds_sync();
    if (active && shl != 0u && w0 < nwords) atomicOr(&stage[w0], first << shl);
}

// The same packing for 16 values per lane at a width W known at compile
// time: every shift is a constant and no branch depends on the bit position.
// Lane l's values take bits [16*W*l, 16*W*(l+1)) of the array.  For even W
// that is W/2 whole words.  For odd W the lanes of a pair 2m, 2m+1 share one
// word (the even lane's last, the odd lane's first): the even lane completes
// it with the odd lane's low 16 bits, moved over by a DPP lane shift within
// the row, and stores it.  Every lane packs (values past the array's count
// are zero), and words past the array's end land in the staging buffer
// without being copied out.
// `dst` is the lane's first word in the staging buffer, stage + lane*W/2
// (rounded down), computed by the caller from the run-time width so that the
// compiler has no per-width address to keep live across the field loop.
template <int W>
__device__ __forceinline__ void pack16(const uint32_t (&v)[16], uint32_t* dst, uint32_t lane) {
    constexpr int NS = (16 * W + 31) / 32;  // words of the segment, from its first bit
    uint32_t s[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) s[k] = 0u;
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int bit = j * W, k = bit >> 5, sh = bit & 31;
        s[k] |= v[j] << sh;
        if (sh + W > 32) s[k + 1] |= v[j] >> (32 - sh);
    }
    if constexpr (W % 2 == 0) {
#pragma unroll
        for (int k = 0; k < W / 2; k++) dst[k] = s[k];
    } else {
        constexpr int H = (W - 1) / 2;  // whole words of an even lane before the shared one
        const bool odd = (lane & 1u) != 0u;
        const uint32_t nxt = dpp<kRowShl1>(s[0] << 16);
#pragma unroll
        for (int t = 0; t <= H; t++) {
            const uint32_t ev = t < H ? s[t] : (s[H] | nxt);
            const uint32_t od = t ? __builtin_amdgcn_alignbit(s[t], s[t - 1], 16) : 0u;
            if (t > 0 || !odd) dst[t] = odd ? od : ev;
        }
    }
}

#define GPZ_PACK16_CASE(W) \
    case W: pack16<W>(v, first, lane); break;

// Fixed-length packing of one array (Sec. 4.3) into the LDS staging buffer:
// value i of `count` values of width w goes to bits [i*w, i*w+w) of it.
template <int ITEMS>
__device__ __forceinline__ void pack_stage(const uint32_t (&v)[ITEMS], uint32_t count, uint32_t w,
                                           uint32_t* stage, uint32_t lane) {
    const uint32_t nwords = words_for(count, w);
    if (nwords == 0) return;
    if constexpr (ITEMS == 16) {
        uint32_t* first = stage + ((lane * w) >> 1);
        switch (w) {
            GPZ_PACK16_CASE(1) GPZ_PACK16_CASE(2) GPZ_PACK16_CASE(3) GPZ_PACK16_CASE(4)
            GPZ_PACK16_CASE(5) GPZ_PACK16_CASE(6) GPZ_PACK16_CASE(7) GPZ_PACK16_CASE(8)
            GPZ_PACK16_CASE(9) GPZ_PACK16_CASE(10) GPZ_PACK16_CASE(11) GPZ_PACK16_CASE(12)
            GPZ_PACK16_CASE(13) GPZ_PACK16_CASE(14) GPZ_PACK16_CASE(15) GPZ_PACK16_CASE(16)
            GPZ_PACK16_CASE(17) GPZ_PACK16_CASE(18) GPZ_PACK16_CASE(19) GPZ_PACK16_CASE(20)
            GPZ_PACK16_CASE(21) GPZ_PACK16_CASE(22) GPZ_PACK16_CASE(23) GPZ_PACK16_CASE(24)
            default: pack_generic<ITEMS>(v, nwords, count, w, stage, lane); break;
        }
    } else {
        pack_generic<ITEMS>(v, nwords, count, w, stage, lane);
    }
}

// The nwords staged words to dst with coalesced stores, four words per lane
// at a time: the four staging reads are all issued before the stores, so
// they cost one LDS round trip, not four.  Whole 256-word steps store
// unconditionally, at 32-bit byte offsets from the array's scalar base; only
// the last, partial step is predicated.  Reads past nwords stay inside the
// staging buffer (its size is checked against the largest array, B values
// of 24 bits) and are never stored.
template <int ITEMS>
__device__ __forceinline__ void copy_out(uint32_t nwords, uint32_t* __restrict__ dst,
                                         const uint32_t* stage, uint32_t lane) {
    uint8_t* const base = reinterpret_cast<uint8_t*>(dst);
    const uint32_t whole = nwords & ~255u;
    for (uint32_t i0 = 0; i0 < whole; i0 += 256) {
        uint32_t t[4];
#pragma unroll
        for (int u = 0; u < 4; u++) t[u] = stage[i0 + 64 * u + lane];
#pragma unroll
        for (int u = 0; u < 4; u++)
            *reinterpret_cast<uint32_t*>(base + 4u * (i0 + 64u * u + lane)) = t[u];
    }
    if (whole < nwords) {
        uint32_t t[4];
#pragma unroll
        for (int u = 0; u < 4; u++) t[u] = stage[whole + 64 * u + lane];
        // keeps the compiler from sinking a read into its store's branch
        asm volatile("" : : "v"(t[0]), "v"(t[1]), "v"(t[2]), "v"(t[3]));
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (whole + 64 * u + lane < nwords)
                *reinterpret_cast<uint32_t*>(base + 4u * (whole + 64u * u + lane)) = t[u];
    }
}

// Fixed-length packing of one array into dst (Sec. 4.3), staged in LDS and
// copied out with coalesced stores.
template <int ITEMS>
__device__ __forceinline__ void pack_array(const uint32_t (&v)[ITEMS], uint32_t count, uint32_t w,
                                           uint32_t* __restrict__ dst, uint32_t* stage,
                                           uint32_t lane) {
    const uint32_t nwords = words_for(count, w);
    if (nwords == 0) return;
    pack_stage<ITEMS>(v, count, w, stage, lane);
    wave_lds_sync();
    copy_out<ITEMS>(nwords, dst, stage, lane);
    wave_lds_sync();
}

// One stable LSD pass over 5 key bits starting at bit `sh` of the key
// (key = kv >> 16).  Each lane counts its own items per digit (LDS atomics on
// its private counter column give the within-lane rank), a raking scan in
// (digit, lane) order gives every (digit, lane) its first slot, and items are
// scattered to their slots and read back blocked.
template <int ITEMS, bool FULL, bool LEAN = false>
__device__ __forceinline__ void radix_pass(uint32_t (&kv)[ITEMS], uint32_t sh, uint32_t nb,
                                           uint32_t lane, uint32_t* cnt, uint32_t* kvbuf) {
    uint4* c4 = reinterpret_cast<uint4*>(cnt);
#pragma unroll
    for (int k = 0; k < 9; k++) c4[lane * 9 + k] = make_uint4(0, 0, 0, 0);
    wave_lds_sync();
    uint32_t rank[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t d = __builtin_amdgcn_ubfe(kv[j], 16 + sh, kDigitBits);
        if (FULL || lane * ITEMS + j < nb) rank[j] = atomicAdd(&cnt[counter_addr(d, lane)], 1u);
        else rank[j] = 0u;
    }
    wave_lds_sync();
    if constexpr (LEAN) {
        // as below, in two halves of 16 counters (the counters are read
        // twice), and the digits extracted again after the scan: fewer
        // registers held across it
        uint4* row = reinterpret_cast<uint4*>(cnt + (lane >> 1) * kRow + (lane & 1) * 32);
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint4 t = row[k];
            run += t.x + t.y + t.z + t.w;
        }
        uint32_t before = wave_incl_scan_u32(run) - run;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint32_t c[16];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint4 t = row[4 * h + k];
                c[4 * k + 0] = t.x;
                c[4 * k + 1] = t.y;
                c[4 * k + 2] = t.z;
                c[4 * k + 3] = t.w;
            }
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const uint32_t t = c[k];
                c[k] = before;
                before += t;
            }
#pragma unroll
            for (int k = 0; k < 4; k++)
                row[4 * h + k] = make_uint4(c[4 * k], c[4 * k + 1], c[4 * k + 2], c[4 * k + 3]);
            wave_lds_sync();
        }
#pragma unroll
        for (int j = 0; j < ITEMS; j++) asm volatile("" : "+v"(kv[j]));
    } else {
        // lane r scans flat entries [32r, 32r+32) of (digit, lane) order:
        // digit r/2, lanes 32*(r%2) .. 32*(r%2)+31, contiguous in its row
        uint4* row = reinterpret_cast<uint4*>(cnt + (lane >> 1) * kRow + (lane & 1) * 32);
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
    wave_lds_sync();
    // All counter reads are issued before the first scatter store: a store
    // between them would make every read wait for the one before it.
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t d = __builtin_amdgcn_ubfe(kv[j], 16 + sh, kDigitBits);
        rank[j] += cnt[counter_addr(d, lane)];
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++)
        if (FULL || lane * ITEMS + j < nb) kvbuf[pad_addr<ITEMS>(rank[j])] = kv[j];
    wave_lds_sync();
    const uint4* mine = reinterpret_cast<const uint4*>(kvbuf + lane * (ITEMS + 4));
#pragma unroll
    for (int k = 0; k < ITEMS / 4; k++) {
        uint4 t = mine[k];
        kv[4 * k + 0] = t.x;
        kv[4 * k + 1] = t.y;
        kv[4 * k + 2] = t.z;
        kv[4 * k + 3] = t.w;
    }
    wave_lds_sync();
}

// A field's codes (q, or 2*q + outlier for a field with outliers) into lane
// l's LDS row.  A key field also needs the largest of its in-segment offsets
// (the low `width` bits of q); a field with outliers needs their number.
template <int ITEMS, bool KEY>
__device__ __forceinline__ void stage_codes(const uint32_t (&q)[ITEMS], uint32_t width, bool clean,
                                            uint4* mine, uint32_t& vmax, uint32_t& no) {
    if (KEY) {
#pragma unroll
        for (int j = 0; j < ITEMS; j++)
            vmax = max(vmax, __builtin_amdgcn_ubfe(q[j], clean ? 0u : 1u, width));
    }
    if (!clean) {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) no += q[j] & 1u;
    }
#pragma unroll
    for (int k = 0; k < ITEMS / 4; k++)
        mine[k] = make_uint4(q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]);
}

// Runs of the sorted segment IDs (Sec. 4.3): uniq[k] is the k-th distinct ID
// and start[k] the sorted position where its run begins, k < U, with
// start[U] = nb.  Lane l takes runs l*ITEMS .. l*ITEMS+ITEMS-1 (0 beyond U).
// Each lane reads its ITEMS words with 16-byte loads, unconditionally (the
// buffers hold B words, entries from U on are ignored), so no read waits for
// another.  Runs past U are cleared with a per-lane bit mask: a compare per
// run would give the compiler U-dependent lane masks to keep (and spill)
// across the whole field loop, so U is also made opaque here.
template <int ITEMS>
__device__ __forceinline__ void load_runs(const uint32_t* src, uint32_t lane,
                                          uint32_t (&r)[ITEMS]) {
    const uint4* p = reinterpret_cast<const uint4*>(src + lane * ITEMS);
#pragma unroll
    for (int k = 0; k < ITEMS / 4; k++) {
        uint4 t = p[k];
        r[4 * k + 0] = t.x;
        r[4 * k + 1] = t.y;
        r[4 * k + 2] = t.z;
        r[4 * k + 3] = t.w;
    }
}

// Bit j set when run lane*ITEMS + j exists (j < ITEMS <= 32).
template <int ITEMS>
__device__ __forceinline__ uint32_t run_mask(uint32_t U, uint32_t lane) {
    asm volatile("" : "+s"(U));
    const int c = min(max((int)U - (int)(lane * ITEMS), 0), ITEMS);
    return c >= 32 ? ~0u : (1u << c) - 1u;
}

// ID gaps minus one; the first ID counts from -1, so its gap is the ID.
template <int ITEMS>
__device__ __forceinline__ void run_gaps(const uint32_t* uniq, uint32_t U, uint32_t lane,
                                         uint32_t (&v)[ITEMS]) {
    uint32_t r[ITEMS];
    load_runs<ITEMS>(uniq, lane, r);
    const uint32_t m = run_mask<ITEMS>(U, lane);
    uint32_t before = (uint32_t)__shfl_up((int)r[ITEMS - 1], 1);
    if (lane == 0) before = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < ITEMS; j++)
        v[j] = (r[j] - (j ? r[j - 1] : before) - 1u) & (uint32_t)__builtin_amdgcn_sbfe(m, j, 1);
}

// Run lengths minus one: start[i+1] - start[i] - 1 (start[U] = nb).
template <int ITEMS>
__device__ __forceinline__ void run_counts(const uint32_t* start, uint32_t U, uint32_t lane,
                                           uint32_t (&v)[ITEMS]) {
    uint32_t r[ITEMS];
    load_runs<ITEMS>(start, lane, r);
    const uint32_t after = start[lane * ITEMS + ITEMS];
    const uint32_t m = run_mask<ITEMS>(U, lane);
#pragma unroll
    for (int j = 0; j < ITEMS; j++)
        v[j] = ((j + 1 < ITEMS ? r[j + 1] : after) - r[j] - 1u) &
               (uint32_t)__builtin_amdgcn_sbfe(m, j, 1);
}

// ------------------------------------------------------------ compaction
// Look-back word of a block: (value << 2) | flag, flag 1 = the block's own
// record length is known, 2 = the inclusive prefix (words of all records up
// to and including this block) is known, 0 = nothing yet.
constexpr uint64_t kFlagLen = 1u, kFlagIncl = 2u;

__device__ __forceinline__ uint64_t load_state(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_state(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Exclusive prefix (in words) of the record lengths of blocks 0..b-1.  Every
// block with a smaller index was started before this one (tickets), so the
// waits below always end.  Lane i inspects block top - i; the
// window moves back 64 blocks at a time until it meets an inclusive prefix.
__device__ __forceinline__ uint64_t exclusive_offset(uint64_t* state, uint32_t b, uint32_t len,
                                                     uint32_t lane) {
    if (lane == 0) store_state(state + b, ((uint64_t)len << 2) | (b == 0 ? kFlagIncl : kFlagLen));
    if (b == 0) return 0;
    uint64_t excl = 0;
    int64_t top = (int64_t)b - 1;
    for (;;) {
        const int64_t p = top - (int64_t)lane;
        const uint64_t st = p >= 0 ? load_state(state + p) : kFlagIncl;
        const uint64_t flag = st & 3u;
        const uint64_t incl = __ballot(flag == kFlagIncl);
        const uint64_t pending = __ballot(flag == 0);
        // lanes up to and including the nearest inclusive prefix
        const uint64_t upto = incl ? ((incl & (~incl + 1)) << 1) - 1 : ~0ull;
        if (pending & upto) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum_u64(((upto >> lane) & 1u) ? (st >> 2) : 0u);
        if (incl) break;
        top -= 64;
    }
    if (lane == 0) store_state(state + b, ((excl + len) << 2) | kFlagIncl);
    return excl;
}

// Stream header and error-bound table (format v1).
__device__ __forceinline__ void write_header(const EncodeArgs& a, uint32_t lane) {
    uint32_t* out = a.out;
    if (lane == 0) {
        out[0] = kMagic;
        out[1] = kVersion;
        out[2] = (uint32_t)(a.n & 0xFFFFFFFFu);
        out[3] = (uint32_t)(a.n >> 32);
        out[4] = a.F;
        out[5] = a.B;
        out[6] = a.K | (a.KF << 8);
        out[7] = a.nblocks;
    }
    uint32_t* ebt = out + kHeaderWords + 2 * nsuper_of(a.nblocks);
    for (uint32_t f = lane; f < a.F; f += 64) ebt[f] = f2u(a.eb[f]);
}

__device__ __forceinline__ void publish_size(const EncodeArgs& a, uint64_t total, uint32_t lane) {
    if (lane == 0) {
        *a.total_bytes = total;
        if (a.ext_bytes) *a.ext_bytes = total;
    }
    if (total <= a.capacity) write_header(a, lane);
}

// Block b's record (len words at rec) goes to its final offset; the block
// also writes its length-table entry, the superblock entry when it opens a
// superblock, and, as the last block, the stream size and header.  Nothing
// is written past the output capacity.
__device__ __forceinline__ void place_record(const EncodeArgs& a, uint32_t b, const uint32_t* rec,
                                             uint32_t len, uint32_t lane) {
    __syncthreads();  // the record's stores by all lanes before they are read back
    const uint64_t excl = exclusive_offset(a.state, b, len, lane);
    const uint64_t capw = a.capacity / 4;
    const uint64_t sup_at = kHeaderWords;
    const uint64_t lt_at = kHeaderWords + 2 * nsuper_of(a.nblocks) + a.F;
    uint32_t* out = a.out;
    if (lane == 0) {
        if (lt_at + b < capw) out[lt_at + b] = len;
        if (b % kSuper == 0) {
            const uint64_t at = sup_at + 2 * (b / kSuper);
            if (at + 1 < capw) {
                out[at] = (uint32_t)(excl & 0xFFFFFFFFu);
                out[at + 1] = (uint32_t)(excl >> 32);
            }
        }
    }
    const uint64_t off = a.prefix + excl;
    if (off + len <= capw) {
        uint32_t* dst = out + off;
        for (uint32_t k = lane; k < len; k += 256) {
            uint32_t v[4];
#pragma unroll
            for (int i = 0; i < 4; i++) v[i] = k + 64 * i < len ? rec[k + 64 * i] : 0u;
#pragma unroll
            for (int i = 0; i < 4; i++)
                if (k + 64 * i < len) dst[k + 64 * i] = v[i];
        }
    }
    if (b == a.nblocks - 1) publish_size(a, 4 * (off + len), lane);
}

// Leaves block b to the generic encoder (its record, length, superblock sum
// and permutation are all written there).
__device__ __forceinline__ void defer_block(const EncodeArgs& a, uint32_t b, uint32_t lane) {
    if (lane == 0) a.defer[atomicAdd(a.defer_count, 1u)] = b;
}

// The block's LDS: one region whose phases reuse it.
//  - sort: radix counters (kCounterWords, 68-word digit rows) and, aliased
//    with them, the scatter target in the padded blocked layout (64*(ITEMS+4)
//    words): each pass reads every counter it needs before its first
//    scatter store, and a wave's LDS operations execute in issue order;
//  - run tables: uniq[0, B), start[0, B] at B, per-lane scratch words for
//    the branch-free run stores at 2B + 64 and 2B + 128;
//  - field loop: the field's codes in the padded blocked layout at 0, and
//    the packer's staging from kStageAt (read in steps of 256 words; the
//    widest array, B values of 24 bits, stays inside).
template <int ITEMS>
struct EncodeSmem {
    static constexpr uint32_t B = 64 * ITEMS;
    static constexpr uint32_t kStageAt = 64 * (ITEMS + 4);
    static constexpr uint32_t kStageWords = (48 * ITEMS + 255) / 256 * 256;
    static constexpr uint32_t kA = kCounterWords > 2 * B + 192 ? kCounterWords : 2 * B + 192;
    static constexpr uint32_t kWords =
        kA > kStageAt + kStageWords ? kA : kStageAt + kStageWords;
    static_assert(64 * (ITEMS + 4) <= kWords, "scatter target inside the region");
    __align__(16) uint32_t buf[kWords];
};

// EARLY: how many fields after the key fields are loaded and quantized with
// them, before the sort (at most three); the others are loaded and quantized
// in the field loop.  With none, fewer values are held across the sort.
template <int ITEMS, bool FULL, bool SINGLE, int EARLY = 3>
__device__ __forceinline__ void encode_block(const EncodeArgs& a, uint32_t b, uint32_t nb,
                                             uint32_t* work) {
    uint32_t* const stage = work + EncodeSmem<ITEMS>::kStageAt;
    constexpr uint32_t B = 64 * ITEMS;
    const uint32_t lane = threadIdx.x;
    const uint64_t base = (uint64_t)b * B;
    const uint32_t F = a.F, K = a.K, KF = a.KF;
    uint32_t* __restrict__ rec = a.temp + (uint64_t)b * a.slot_words;
    const uint32_t cap = 1 + F * nb;  // raw record length

    // ---- Stage 1 (Sec. 4.1): key axes -- block minimum, grid index, segment shift
    // The loads of the key fields and of up to three other fields are all
    // issued here, before any store of the block: vector memory operations
    // complete in issue order, so a load issued behind the record's stores
    // would wait for them.
    float xk[3][ITEMS], xo[3][ITEMS];
#pragma unroll
    for (int ax = 0; ax < 3; ax++)
        if ((uint32_t)ax < KF) load_block<ITEMS, FULL>(a.x[ax], base, nb, lane, xk[ax]);
#pragma unroll
    for (int e = 0; e < EARLY; e++)
        if (KF + e < F) load_block<ITEMS, FULL>(a.x[KF + e], base, nb, lane, xo[e]);
    // codes are 2*q + outlier (Sec. 4.1)
    uint32_t qk[3][ITEMS];
    FieldCodes ck[3];
    uint32_t sk[3];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        sk[ax] = 0;
        ck[ax] = {0.0f, 0u, true};
        if ((uint32_t)ax < KF) {
            ck[ax] = quantize_field<ITEMS, FULL>(xk[ax], nb, lane, a.inv[ax], a.twoeb[ax],
                                                 a.eb[ax], qk[ax]);
            const uint32_t W = bit_width(ck[ax].qmax);
            sk[ax] = W > K ? W - K : 0;
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; j++) qk[ax][j] = 0;
        }
    }
    // the other early fields
    uint32_t qo[3][ITEMS];
    FieldCodes co[3];
#pragma unroll
    for (int e = 0; e < 3; e++) {
        co[e] = {0.0f, 0u, true};
        if (e < EARLY && KF + e < F) {
            const uint32_t f = KF + e;
            co[e] = quantize_field<ITEMS, FULL>(xo[e], nb, lane, a.inv[f], a.twoeb[f], a.eb[f],
                                                qo[e]);
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; j++) qo[e][j] = 0;
        }
    }

    // A field whose grid needs more than 24 bits: the generic encoder codes
    // the block (three-step compaction); the single pass, which cannot wait
    // for it, stores the block raw.
    bool wide = ck[0].wide || ck[1].wide || ck[2].wide || co[0].wide || co[1].wide || co[2].wide;
    if (!SINGLE && wide) {
        defer_block(a, b, lane);
        return;
    }

    // Linearised segment ID (axis 0 most significant), packed with the index.
    uint32_t kv[ITEMS];
    uint32_t keyor = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        uint32_t key = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ax++)
            if ((uint32_t)ax < KF)
                key = (key << K) | (qk[ax][j] >> (sk[ax] + (ck[ax].clean ? 0u : 1u)));
        uint32_t i = lane * ITEMS + j;
        kv[j] = (key << 16) | (4u * pad_addr<ITEMS>(i));
        if (FULL || i < nb) keyor |= key;
    }
    keyor = wave_or_u32(keyor);

    // ---- Stage 2 (Sec. 4.2): stable in-block sort by segment ID
    const uint32_t keybits = K * KF;
    for (uint32_t sh = 0; sh < keybits; sh += kDigitBits) {
        if (((keyor >> sh) & (kDigits - 1)) == 0) continue;  // identity pass
        radix_pass<ITEMS, FULL, EARLY == 0>(kv, sh, nb, lane, work, work);
    }

    // ---- Stage 3 (Sec. 4.3): run-length coding of the sorted IDs
    uint32_t* uniq = work;
    uint32_t* start = work + B;
    uint32_t U;
    {
        uint32_t prev = (uint32_t)__shfl_up((int)(kv[ITEMS - 1] >> 16), 1);
        uint32_t nflag = 0;
        bool flag[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t p = lane * ITEMS + j;
            uint32_t key = kv[j] >> 16;
            uint32_t before = j == 0 ? prev : (kv[j - 1] >> 16);
            flag[j] = (FULL || p < nb) && (p == 0 || key != before);
            nflag += flag[j];
        }
        uint32_t incl = wave_incl_scan_u32(nflag);
        U = readlane(incl, 63);
        // Every item stores, without branches: a run start at its rank k,
        // any other item to a scratch word of its lane past the tables.
        uint32_t k = incl - nflag;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uniq[flag[j] ? k : 2 * B + 64 + lane] = kv[j] >> 16;
            start[flag[j] ? k : B + 128 + lane] = lane * ITEMS + j;
            k += flag[j] ? 1u : 0u;
        }
        if (lane == 0) start[U] = nb;
    }
    wave_lds_sync();
    // from here on the items are only LDS offsets (the permutation)
#pragma unroll
    for (int j = 0; j < ITEMS; j++) kv[j] &= 0xFFFFu;
    // delta coding of the distinct IDs (stored as delta - 1) and counts - 1,
    // kept in registers until they are packed
    uint32_t gv[ITEMS], cv[ITEMS];
    run_gaps<ITEMS>(uniq, U, lane, gv);
    run_counts<ITEMS>(start, U, lane, cv);
    uint32_t gmax = 0, cmax = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        gmax = max(gmax, gv[j]);
        cmax = max(cmax, cv[j]);
    }
    const uint32_t w_gap = bit_width(wave_max_u32(gmax));
    const uint32_t w_cnt = bit_width(wave_max_u32(cmax));
    if (lane == 0) {
        rec[0] = U << 2;
        rec[1] = w_gap | (w_cnt << 5) | (sk[0] << 10) | (sk[1] << 15) | (sk[2] << 20);
    }

    // ---- arrays in record order: gaps, counts, then one section per field
    uint32_t pos = 2;
    bool over = wide;  // (single pass only: such a block is stored raw)
    const uint32_t gw = words_for(U, w_gap), cw = words_for(U, w_cnt);
    // Each array's packed words leave the staging buffer while the next
    // field's permutation reads are in flight (one LDS round trip for both):
    // `pend` words staged for `pend_dst` are still to be copied out.
    uint32_t pend = 0;
    uint32_t* pend_dst = rec;
    if (pos + gw + cw > cap) {
        over = true;
    } else {
        wave_lds_sync();  // uniq/start reads done before `work` is reused
        pack_array<ITEMS>(gv, U, w_gap, rec + pos, stage, lane);
        pack_stage<ITEMS>(cv, U, w_cnt, stage, lane);
        pend = cw;
        pend_dst = rec + pos + gw;
        pos += gw + cw;
    }
    // One field's section once its codes are staged in LDS (input order, at
    // `work` in the padded blocked layout): lo and field word, the codes
    // permuted to sorted order (a key field's in-segment offsets: its low
    // `width` bits), packed; its outliers.  Returns false when the block is
    // stored raw (or, for a wide field, left to the generic encoder).
    auto section = [&](uint32_t f, const FieldCodes& c, bool key, uint32_t width, uint32_t vmax,
                       uint32_t no) -> bool {
        if (wide) {
            over = true;
            return false;
        }
        const uint32_t w = bit_width(key ? wave_max_u32(vmax) : c.qmax);
        const uint32_t nout = c.clean ? 0u : wave_sum_u32(no);
        if (pos + 2 + words_for(nb, w) + 2 * nout > cap) {
            over = true;
            return false;
        }
        if (lane == 0) {
            rec[pos] = f2u(c.lo);
            rec[pos + 1] = w | (nout << 5);
        }
        pos += 2;
        // permute to sorted order through LDS
        wave_lds_sync();
        // the packed value: q of a clean non-key field as it is, else the
        // code's grid index (without the outlier bit) cut to `width` bits
        uint32_t vals[ITEMS];
        if (!key && c.clean) {
#pragma unroll
            for (int j = 0; j < ITEMS; j++)
                vals[j] = (FULL || lane * ITEMS + j < nb) ? staged_at(work, kv[j]) : 0u;
        } else {
            const uint32_t s0 = c.clean ? 0u : 1u;
#pragma unroll
            for (int j = 0; j < ITEMS; j++)
                vals[j] = (FULL || lane * ITEMS + j < nb)
                              ? __builtin_amdgcn_ubfe(staged_at(work, kv[j]), s0, width)
                              : 0u;
        }
        if (pend) {
            wave_lds_sync();
            copy_out<ITEMS>(pend, pend_dst, stage, lane);
        }
        wave_lds_sync();  // the staged words are read before they are replaced
        pack_stage<ITEMS>(vals, nb, w, stage, lane);
        pend = words_for(nb, w);
        pend_dst = rec + pos;
        pos += pend;
        if (nout) {
            // outlier flags of the sorted positions, read again from the staging
            uint32_t flags = 0;
#pragma unroll
            for (int j = 0; j < ITEMS; j++)
                if ((FULL || lane * ITEMS + j < nb) &&
                    (staged_at(work, kv[j]) & 1u))
                    flags |= 1u << j;
            const uint32_t cnt = __builtin_popcount(flags);
            uint32_t k = wave_incl_scan_u32(cnt) - cnt;
            uint32_t* ol = rec + pos;
            const float* xf = a.x[f] + base;
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                if ((flags >> j) & 1u) {
                    ol[2 * k] = lane * ITEMS + j;
                    ol[2 * k + 1] = f2u(xf[index_of<ITEMS>(kv[j])]);
                    k++;
                }
            }
            pos += 2 * nout;
        }
        wave_lds_sync();  // staging reads done before the next field overwrites it
        return true;
    };
    uint4* const mine = reinterpret_cast<uint4*>(work + lane * (ITEMS + 4));
    if constexpr (EARLY == 0) {
        // The key fields' codes are in registers; each other field is
        // fetched while its predecessor is staged and packed.
        for (uint32_t f = 0; f < KF && !over; f++) {
            // the permutation's LDS offsets are recomputed per field instead
            // of being held in registers across the loop
#pragma unroll
            for (int j = 0; j < ITEMS; j++) asm volatile("" : "+v"(kv[j]));
            FieldCodes c{0.0f, 0u, true, false};
            uint32_t width = 0, vmax = 0, no = 0;
            // one wave-uniform branch per source, each reading its own
            // registers (the empty asm keeps the compiler from merging the
            // branches into a select per value)
            switch (f) {
#define GPZ_STAGE(N)                                                        \
    case N:                                                                 \
        c = ck[N];                                                          \
        width = sk[N];                                                      \
        stage_codes<ITEMS, true>(qk[N], width, c.clean, mine, vmax, no);    \
        asm volatile("");                                                   \
        break;
                GPZ_STAGE(0) GPZ_STAGE(1) GPZ_STAGE(2)
#undef GPZ_STAGE
            }
            if (!section(f, c, true, width, vmax, no)) break;
        }
        float xn[ITEMS];
        if (KF < F && !over) load_block<ITEMS, FULL>(a.x[KF], base, nb, lane, xn);
        for (uint32_t f = KF; f < F && !over; f++) {
#pragma unroll
            for (int j = 0; j < ITEMS; j++) asm volatile("" : "+v"(kv[j]));
            uint32_t q[ITEMS];
            const FieldCodes c =
                quantize_field<ITEMS, FULL>(xn, nb, lane, a.inv[f], a.twoeb[f], a.eb[f], q);
            if (f + 1 < F) load_block<ITEMS, FULL>(a.x[f + 1], base, nb, lane, xn);
            wide = wide || c.wide;
            uint32_t vmax = 0, no = 0;
            stage_codes<ITEMS, false>(q, 24u, c.clean, mine, vmax, no);
            if (!section(f, c, false, 24u, vmax, no)) break;
        }
    } else {
        for (uint32_t f = 0; f < F && !over; f++) {
            FieldCodes c{0.0f, 0u, true, false};
            uint32_t width = 24, vmax = 0, no = 0;
            bool key = false;
            // The field's codes go to LDS in input order (for the
            // permutation).  Key fields and the early fields are already in
            // registers: one wave-uniform branch per source, each reading
            // its own registers (the empty asm keeps the compiler from
            // merging the branches into a select per value).  Later fields
            // are loaded and quantized here.  The packed value is the code's
            // in-segment offset for a key field (its low sk bits), the whole
            // code otherwise.
            const uint32_t src = f < KF ? f : 3 + (f - KF);
            switch (src) {
#define GPZ_STAGE(N, QA, C, KEY, WIDTH)                                  \
    case N:                                                              \
        c = C;                                                           \
        key = KEY;                                                       \
        width = WIDTH;                                                   \
        stage_codes<ITEMS, KEY>(QA, width, c.clean, mine, vmax, no);     \
        asm volatile("");                                                \
        break;
                GPZ_STAGE(0, qk[0], ck[0], true, sk[0])
                GPZ_STAGE(1, qk[1], ck[1], true, sk[1])
                GPZ_STAGE(2, qk[2], ck[2], true, sk[2])
                GPZ_STAGE(3, qo[0], co[0], false, 24u)
                GPZ_STAGE(4, qo[1], co[1], false, 24u)
                GPZ_STAGE(5, qo[2], co[2], false, 24u)
#undef GPZ_STAGE
                default: {
                    uint32_t q[ITEMS];
                    float x[ITEMS];
                    load_block<ITEMS, FULL>(a.x[f], base, nb, lane, x);
                    c = quantize_field<ITEMS, FULL>(x, nb, lane, a.inv[f], a.twoeb[f], a.eb[f], q);
                    wide = wide || c.wide;
                    stage_codes<ITEMS, false>(q, width, c.clean, mine, vmax, no);
                    break;
                }
            }
            if (!section(f, c, key, width, vmax, no)) break;
        }
    }
    if (!over && pend) {
        wave_lds_sync();
        copy_out<ITEMS>(pend, pend_dst, stage, lane);
        wave_lds_sync();
    }

    if (!SINGLE && wide) {
        defer_block(a, b, lane);
        return;
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
    if (SINGLE) {
        place_record(a, b, rec, raw ? cap : pos, lane);
    } else if (lane == 0) {
        const uint32_t len = raw ? cap : pos;
        a.lens[b] = len;
        atomicAdd(&a.supsum[b / kSuper], len);  // order-independent sum
    }
    if (a.perm) {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t p = lane * ITEMS + j;
            if (FULL || p < nb)
                a.perm[base + p] = (uint32_t)(base + (raw ? p : index_of<ITEMS>(kv[j])));
        }
    }
}


// Three-step compaction: one workgroup per block, block index = workgroup
// index.  Full blocks take the path without bounds checks, the partial last
// block (if any) the checked one.
template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void encode_blocks(EncodeArgs a) {
    constexpr uint32_t B = 64 * ITEMS;
    __shared__ EncodeSmem<ITEMS> sm;
    const uint32_t b = blockIdx.x;
    const uint64_t left = a.n - (uint64_t)b * B;
    if (left >= B) encode_block<ITEMS, true, false>(a, b, B, sm.buf);
    else encode_block<ITEMS, false, false>(a, b, (uint32_t)left, sm.buf);
}

// The same with no early fields beside the key fields (EARLY = 0) and the
// sort's lean scan: at most 168 VGPRs, three waves per SIMD instead of two.
// At B = 1024 this is faster on every workload measured (cosmology 64M x 6
// -4 %, md 32M x 6 -4 %, LiDAR 100M x 3 -13 %): the late fields' loads are
// hidden by the third wave.
template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void encode_blocks_lean(EncodeArgs a) {
    constexpr uint32_t B = 64 * ITEMS;
    __shared__ EncodeSmem<ITEMS> sm;
    const uint32_t b = blockIdx.x;
    const uint64_t left = a.n - (uint64_t)b * B;
    if (left >= B) encode_block<ITEMS, true, false, 0>(a, b, B, sm.buf);
    else encode_block<ITEMS, false, false, 0>(a, b, (uint32_t)left, sm.buf);
}

// Single-pass compaction: blocks are numbered by a ticket taken when the
// workgroup starts, so a block only ever waits on blocks already running.
template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void encode_blocks_single(EncodeArgs a) {
    constexpr uint32_t B = 64 * ITEMS;
    __shared__ EncodeSmem<ITEMS> sm;
    uint32_t t = 0;
    if (threadIdx.x == 0) t = atomicAdd(a.ticket, 1u);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
    const uint64_t left = a.n - (uint64_t)b * B;
    if (left >= B) encode_block<ITEMS, true, true>(a, b, B, sm.buf);
    else encode_block<ITEMS, false, true>(a, b, (uint32_t)left, sm.buf);
}

// Single pass, a snapshot with no particles: header only.
__global__ __launch_bounds__(64) void empty_stream(EncodeArgs a) {
    publish_size(a, 4 * a.prefix, threadIdx.x);
}

template <int ITEMS>
void launch_encode_items(const EncodeArgs& a, bool single_pass, hipStream_t s) {
    if (single_pass) {
        if (a.nblocks) hipLaunchKernelGGL(encode_blocks_single<ITEMS>, dim3(a.nblocks), dim3(64), 0, s, a);
        else hipLaunchKernelGGL(empty_stream, dim3(1), dim3(64), 0, s, a);
        return;
    }
    // one launch: full blocks take the path without bounds checks, a partial
    // last block the checked one, alongside them (not in a second launch
    // that would wait for the first)
    if (a.nblocks == 0) return;
    if constexpr (ITEMS == 16)
        hipLaunchKernelGGL(encode_blocks_lean<ITEMS>, dim3(a.nblocks), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(encode_blocks<ITEMS>, dim3(a.nblocks), dim3(64), 0, s, a);
}

// Persistent encoder over the full blocks of many snapshots: each wave takes
// `tile` consecutive blocks from a device work queue until it is empty.
template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void encode_batch(const EncodeArgs* __restrict__ jobs,
                                                   const BatchLaunch* __restrict__ L) {
    constexpr uint32_t B = 64 * ITEMS;
    __shared__ EncodeSmem<ITEMS> sm;
    const uint32_t total = L->total_full, njobs = L->njobs, tile = L->tile;
    const uint32_t* prefix = L->full_prefix;
    for (;;) {
        uint32_t item = 0;
        if (threadIdx.x == 0) item = atomicAdd(L->counter, tile);
        item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
        if (item >= total) break;
        const uint32_t end = min(item + tile, total);
        for (uint32_t g = item; g < end; g++) {
            const uint32_t j = find_job(prefix, njobs, g);
            encode_block<ITEMS, true, false>(jobs[j], g - prefix[j], B, sm.buf);
            __syncthreads();
        }
    }
}

// Direct form of encode_batch: one workgroup per block of the batch's
// capacity; workgroups past the bound jobs' blocks exit at once.  No loop
// around the block, so the compiler keeps the register budget of the plain
// kernel.  Up to B = 1024 the partial last blocks of the snapshots take their
// checked path in the same launch (as in the plain form); at B = 2048 that
// path would add spills to every block, so they go to encode_batch_tails.
template <int ITEMS>
constexpr bool kDirectTails = ITEMS <= 16;

template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(ITEMS == 16 ? 3 : 2))) void encode_batch_direct(
    const EncodeArgs* __restrict__ jobs, const BatchLaunch* __restrict__ L) {
    constexpr uint32_t B = 64 * ITEMS;
    constexpr int EARLY = ITEMS == 16 ? 0 : 3;
    __shared__ EncodeSmem<ITEMS> sm;
    const uint32_t g = blockIdx.x;
    if (g >= (kDirectTails<ITEMS> ? L->total_blocks : L->total_full)) return;
    const uint32_t* prefix = kDirectTails<ITEMS> ? L->block_prefix : L->full_prefix;
    const uint32_t j = find_job(prefix, L->njobs, g);
    const EncodeArgs& a = jobs[j];
    const uint32_t b = g - prefix[j];
    if constexpr (kDirectTails<ITEMS>) {
        const uint64_t left = a.n - (uint64_t)b * B;
        if (left < B) {
            encode_block<ITEMS, false, false, EARLY>(a, b, (uint32_t)left, sm.buf);
            return;
        }
    }
    encode_block<ITEMS, true, false, EARLY>(a, b, B, sm.buf);
}

// The partial last block of each snapshot that has one.
template <int ITEMS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(ITEMS == 16 ? 3 : 2))) void encode_batch_tails(const EncodeArgs* __restrict__ jobs,
                                                         const BatchLaunch* __restrict__ L) {
    constexpr uint32_t B = 64 * ITEMS;
    __shared__ EncodeSmem<ITEMS> sm;
    const uint32_t ntail = L->ntail;
    for (uint32_t t = blockIdx.x; t < ntail; t += gridDim.x) {
        const EncodeArgs& a = jobs[__builtin_amdgcn_readfirstlane((int)L->tail_jobs[t])];
        const uint32_t b = a.nblocks - 1;
        const uint32_t nb = (uint32_t)(a.n - (uint64_t)b * B);
        encode_block<ITEMS, false, false, ITEMS == 16 ? 0 : 3>(a, b, nb, sm.buf);
        __syncthreads();
    }
}

template <int ITEMS>
void launch_encode_batch_items(const EncodeArgs* jobs, const BatchLaunch* L, const BatchShape& S,
                               hipStream_t s) {
    if (S.grid) {
        hipLaunchKernelGGL(encode_batch<ITEMS>, dim3(S.grid), dim3(64), 0, s, jobs, L);
        hipLaunchKernelGGL(encode_batch_tails<ITEMS>, dim3(S.tail_grid), dim3(64), 0, s, jobs, L);
    } else {
        hipLaunchKernelGGL(encode_batch_direct<ITEMS>, dim3(S.direct_grid), dim3(64), 0, s, jobs, L);
        if (!kDirectTails<ITEMS>)
            hipLaunchKernelGGL(encode_batch_tails<ITEMS>, dim3(S.tail_grid), dim3(64), 0, s, jobs, L);
    }
}

}  // namespace

hipError_t launch_encode_batch(const EncodeArgs* jobs, const BatchLaunch* L, const BatchShape& S,
                               hipStream_t s) {
    switch (S.B) {
        case 256: launch_encode_batch_items<4>(jobs, L, S, s); break;
        case 512: launch_encode_batch_items<8>(jobs, L, S, s); break;
        case 1024: launch_encode_batch_items<16>(jobs, L, S, s); break;
        case 2048: launch_encode_batch_items<32>(jobs, L, S, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode(const EncodeArgs& a, bool single_pass, hipStream_t s) {
    switch (a.B) {
        case 256: launch_encode_items<4>(a, single_pass, s); break;
        case 512: launch_encode_items<8>(a, single_pass, s); break;
        case 1024: launch_encode_items<16>(a, single_pass, s); break;
        case 2048: launch_encode_items<32>(a, single_pass, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gpz
