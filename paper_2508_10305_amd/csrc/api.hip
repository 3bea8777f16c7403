// C ABI of libgpz (declared in include/gpz.h): argument checks, workspace
// layout, kernel sequencing and status reporting.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "gpz.h"
#include "gpz_internal.h"

using namespace gpz;

// Scratch of gpz_field_range_noalloc: the 2F order-preserving minimum and
// maximum keys of up to kMaxFields fields (512 bytes).  Each GPU holds its
// own copy for the life of the process.  In host code `scratch` only names
// the symbol: kernels are given its device address, looked up once per
// device (noalloc_scratch).
static __device__ __align__(256) int scratch[2 * kMaxFields];

namespace {

// Optional kernel timing: HIP events recorded around each kernel on the
// launch stream, collected later by gpz_timing_collect.
enum { kEncode = 0, kPrepare = 1, kDecode = 2, kScan = 3, kCopy = 4, kGeneric = 5, kKinds = 6 };
struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};
thread_local uint32_t g_timing = 0;  // bit k: time kernels of kind k
thread_local std::vector<TimedLaunch> g_log;

struct Timer {
    hipStream_t s;
    bool on;
    TimedLaunch cur{};
    explicit Timer(hipStream_t st) : s(st), on(g_timing != 0) {}
    void begin(int kind) {
        if (!on || !((g_timing >> kind) & 1u)) return;
        cur.kind = kind;
        if (hipEventCreate(&cur.a) != hipSuccess) return;
        if (hipEventCreate(&cur.b) != hipSuccess) {
            (void)hipEventDestroy(cur.a);
            return;
        }
        (void)hipEventRecord(cur.a, s);
    }
    void end() {
        if (!on || !cur.a) return;
        (void)hipEventRecord(cur.b, s);
        g_log.push_back(cur);
        cur = TimedLaunch{};
    }
};

bool eb_valid(float eb) { return isfinite(eb) && eb >= 0x1p-120f && eb <= 0x1p120f; }

bool params_ok(uint32_t F, const gpz_params& p) {
    if (F < 1 || F > kMaxFields) return false;
    uint32_t B = p.block_size;
    if (B < 64 || B > 4096 || (B & (B - 1)) != 0) return false;
    if (p.key_fields < 1 || p.key_fields > 3 || p.key_fields > F) return false;
    if (p.seg_bits > 5 || (p.flags & ~GPZ_FLAG_SINGLE_PASS) != 0) return false;
    return true;
}

// Block sizes of the wave-per-block kernels; the generic ones take any.
bool kernel_block_size(uint32_t B) { return B == 256 || B == 512 || B == 1024 || B == 2048; }

gpz_params resolve(const gpz_params* p, uint32_t F) {
    gpz_params q;
    gpz_default_params(&q, F);
    if (p) q = *p;
    return q;
}

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

struct CompressWs {
    uint32_t* temp;     // record slots
    uint64_t* state;    // look-back word per block
    uint32_t* ticket;   // block ticket counter (right after the look-back words)
    uint64_t* total;    // stream size
    uint32_t* defer_count;  // blocks left to the generic encoder
    uint32_t* wide_flag;    // a record codes a field with 64-bit steps
    uint32_t* done;         // workgroups of the deferred-block walk that have finished
    uint64_t clear_words;  // 32-bit words from `state` to clear before a launch
    // three-step compaction
    uint32_t* lens;
    uint32_t* supsum;
    uint64_t* supoff;
    uint32_t* defer;    // the deferred block list
    uint32_t slot_words;
    uint64_t bytes;
};

// Address `off` bytes into the workspace at `base` (nullptr when only the
// sizes are wanted: integer arithmetic, no pointer offset from null).
template <typename T>
T* ws_at(char* base, uint64_t off) {
    return base ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(base) + off) : nullptr;
}

// vw: words per value (1 float32, 2 float64)
CompressWs layout(uint64_t n, uint32_t F, uint32_t B, uint32_t vw, char* base) {
    CompressWs w{};
    const uint64_t nb = nblocks_of(n, B), ns = nsuper_of(nb);
    w.slot_words = (uint32_t)((1 + (uint64_t)F * B * vw + 3) & ~uint64_t(3));
    uint64_t o = 0;
    w.temp = ws_at<uint32_t>(base, o);
    o = align256(o + nb * w.slot_words * 4ull);
    // look-back words, ticket, total, deferred-block count, wide flag and the
    // superblock sums are contiguous: one fill clears what either compaction
    // needs zeroed (the three-step one starts it at the ticket, after the
    // look-back words only the single pass uses)
    w.state = ws_at<uint64_t>(base, o);
    w.ticket = ws_at<uint32_t>(base, o + nb * 8);
    w.total = ws_at<uint64_t>(base, o + nb * 8 + 8);
    w.defer_count = ws_at<uint32_t>(base, o + nb * 8 + 16);
    w.wide_flag = ws_at<uint32_t>(base, o + nb * 8 + 20);
    w.done = ws_at<uint32_t>(base, o + nb * 8 + 24);
    w.supsum = ws_at<uint32_t>(base, o + nb * 8 + 28);
    w.clear_words = 2 * nb + 7 + ns;
    o = align256(o + nb * 8 + 28 + ns * 4);
    w.supoff = ws_at<uint64_t>(base, o);
    o = align256(o + ns * 8);
    w.lens = ws_at<uint32_t>(base, o);
    o = align256(o + nb * 4);
    w.defer = ws_at<uint32_t>(base, o);
    o = align256(o + nb * 4);
    w.bytes = o;
    return w;
}

int to_status(hipError_t e) { return e == hipSuccess ? GPZ_OK : GPZ_EDEVICE; }
bool alloc_fault();

// Shared body of the compress entry points (float32 or float64 fields).
// The wave-per-block encoder takes float32 snapshots at block sizes
// 256..2048 and leaves blocks that need 64-bit grid steps to the generic
// encoder; float64 fields and other block sizes go to the generic encoder
// whole.
int compress_impl(const void* const* h_fields, bool f64, uint64_t n, uint32_t F, const float* h_eb,
                  const gpz_params* pp, void* d_out, uint64_t cap, uint64_t* h_out_bytes,
                  uint64_t* d_out_bytes, uint32_t* d_perm, void* d_ws, uint64_t ws_bytes,
                  hipStream_t s, bool sync) {
    if (F < 1 || F > kMaxFields || !h_eb) return GPZ_EINVAL;
    gpz_params p = resolve(pp, F);
    if (!params_ok(F, p)) return GPZ_EINVAL;
    const bool single = (p.flags & GPZ_FLAG_SINGLE_PASS) != 0;
    const bool generic = f64 || !kernel_block_size(p.block_size);
    // the single pass exists for the wave-per-block encoder only
    if (single && generic) return GPZ_EUNSUPPORTED;
    if (n > 0 && !h_fields) return GPZ_EINVAL;
    if (!d_out) return GPZ_EINVAL;
    // one workgroup per block: the dispatch size (64 or 256 lanes per block)
    // must fit 32 bits
    if (nblocks_of(n, p.block_size) > ((uint64_t)1 << (generic ? 24 : 26))) return GPZ_EINVAL;
    for (uint32_t f = 0; f < F; f++) {
        if (!eb_valid(h_eb[f])) return GPZ_EINVAL;
        if (n > 0 && !h_fields[f]) return GPZ_EINVAL;
    }
    const uint32_t B = p.block_size;
    const uint32_t vw = f64 ? 2u : 1u;
    const uint64_t nb = nblocks_of(n, B);
    CompressWs probe = layout(n, F, B, vw, nullptr);
    char* ws = static_cast<char*>(d_ws);
    bool owned = false;
    if (!ws) {
        if (!sync) return GPZ_EINVAL;
        if (alloc_fault() || hipMalloc(&ws, probe.bytes) != hipSuccess) return GPZ_ENOMEM;
        owned = true;
    } else if (ws_bytes < probe.bytes) {
        return GPZ_EINVAL;
    }
    CompressWs w = layout(n, F, B, vw, ws);

    EncodeArgs ea{};
    for (uint32_t f = 0; f < F; f++) {
        ea.x[f] = n ? static_cast<const float*>(h_fields[f]) : nullptr;
        ea.eb[f] = h_eb[f];
        ea.twoeb[f] = 2.0f * h_eb[f];
        ea.inv[f] = 1.0f / ea.twoeb[f];
    }
    ea.n = n;
    ea.F = F;
    ea.K = p.seg_bits;
    ea.KF = p.key_fields;
    ea.B = B;
    ea.nblocks = (uint32_t)nb;
    ea.slot_words = w.slot_words;
    ea.temp = w.temp;
    ea.state = w.state;
    ea.ticket = w.ticket;
    ea.perm = d_perm;
    ea.out = static_cast<uint32_t*>(d_out);
    ea.capacity = cap;
    ea.prefix = prefix_words(n, F, B);
    ea.total_bytes = w.total;
    ea.ext_bytes = d_out_bytes;
    ea.lens = w.lens;
    ea.supsum = w.supsum;
    ea.f64 = f64 ? 1u : 0u;
    ea.defer = w.defer;
    ea.defer_count = w.defer_count;
    ea.wide_flag = w.wide_flag;

    Timer tm(s);
    tm.begin(kPrepare);
    // the single pass also needs its look-back words zeroed; the three steps
    // only the counters and superblock sums that follow them
    int rc = to_status(
        single ? launch_fill_u32(reinterpret_cast<uint32_t*>(w.state), 0u, w.clear_words, s)
               : launch_fill_u32(w.ticket, 0u, w.clear_words - 2 * nb, s));
    tm.end();
    tm.begin(kEncode);
    if (rc == GPZ_OK) rc = to_status(generic ? launch_encode_generic(ea, false, s)
                                             : launch_encode(ea, single, s));
    tm.end();
    if (!single) {
        ScanArgs sa{};
        CopyArgs ca{};
        for (uint32_t f = 0; f < F; f++) memcpy(&sa.eb_bits[f], &h_eb[f], 4);
        sa.supsum = w.supsum;
        sa.supoff = w.supoff;
        sa.total_bytes = w.total;
        sa.ext_bytes = d_out_bytes;
        sa.nsuper = (uint32_t)nsuper_of(nb);
        sa.prefix = ea.prefix;
        sa.out = ea.out;
        sa.capacity = cap;
        sa.n = n;
        sa.F = F;
        sa.B = B;
        sa.K = p.seg_bits;
        sa.KF = p.key_fields;
        sa.nblocks = (uint32_t)nb;
        sa.f64 = ea.f64;
        sa.wide_flag = w.wide_flag;
        ca.temp = w.temp;
        ca.lens = w.lens;
        ca.supoff = w.supoff;
        ca.total_bytes = w.total;
        ca.out = ea.out;
        ca.capacity = cap;
        ca.slot_words = w.slot_words;
        ca.nblocks = (uint32_t)nb;
        ca.F = F;
        // after the wave-per-block encoder, the walk over the blocks it left
        // for 64-bit steps and the scan share one launch
        tm.begin(kScan);
        if (rc == GPZ_OK)
            rc = to_status(generic ? launch_scan(sa, s)
                                   : launch_encode_deferred_then_scan(ea, sa, w.done, s));
        tm.end();
        tm.begin(kCopy);
        if (rc == GPZ_OK) rc = to_status(launch_copy(ca, s));
        tm.end();
    }
    if (sync) {
        uint64_t total = 0;
        if (rc == GPZ_OK) rc = to_status(hipMemcpyAsync(&total, w.total, 8, hipMemcpyDeviceToHost, s));
        if (rc == GPZ_OK) rc = to_status(hipStreamSynchronize(s));
        if (h_out_bytes) *h_out_bytes = total;
        if (rc == GPZ_OK && total > cap) rc = GPZ_ENOSPC;
    }
    if (owned) {
        // kernels already queued may still use the workspace, also after an error
        (void)hipStreamSynchronize(s);
        (void)hipFree(ws);
    }
    return rc;
}

// Workspace of the reporting calls (error statistics, bound check, stream
// statistics, field range): 32 bytes per field and a few flags.
uint64_t stats_ws_bytes(uint32_t F) { return align256(32ull * F + 64); }

// The library's own allocations; GPZ_FAULT=alloc makes them fail (tests of
// the allocation-free paths).
bool alloc_fault() {
    const char* e = getenv("GPZ_FAULT");
    return e && strcmp(e, "alloc") == 0;
}

// The caller's workspace (at least `need` bytes), or with d_ws NULL one the
// library allocates for the call (*owned, freed by the caller of take_ws).
int take_ws(void* d_ws, uint64_t ws_bytes, uint64_t need, char** out, bool* owned) {
    *owned = false;
    if (d_ws) {
        if (ws_bytes < need) return GPZ_EINVAL;
        *out = static_cast<char*>(d_ws);
        return GPZ_OK;
    }
    if (alloc_fault() || hipMalloc(reinterpret_cast<void**>(out), need) != hipSuccess)
        return GPZ_ENOMEM;
    *owned = true;
    return GPZ_OK;
}

// Minimum / maximum keys (order-preserving integers of the float bits) set to
// the identities of atomicMin / atomicMax, by a kernel (graph-capturable).
int range_keys_reset(int* keys, uint32_t F, hipStream_t s) {
    int rc = to_status(launch_fill_u32(reinterpret_cast<uint32_t*>(keys), 0x7FFFFFFFu, F, s));
    if (rc == GPZ_OK)
        rc = to_status(launch_fill_u32(reinterpret_cast<uint32_t*>(keys) + F, 0x80000000u, F, s));
    return rc;
}

// Field range from its keys: 0, 0 when no finite value was seen, a zero
// extreme as +0.0.
void range_from_keys(int mn, int mx, float* lo, float* hi) {
    *lo = 0.0f;
    *hi = 0.0f;
    if (mn <= mx) {  // some finite value was seen
        const int a = mn ^ ((mn >> 31) & 0x7FFFFFFF), b = mx ^ ((mx >> 31) & 0x7FFFFFFF);
        memcpy(lo, &a, 4);
        memcpy(hi, &b, 4);
        if (*lo == 0.0f) *lo = 0.0f;
        if (*hi == 0.0f) *hi = 0.0f;
    }
}

// Field range of F device arrays through 8F bytes of device scratch `keys`;
// writes h_minmax[2F] and synchronizes the stream.
int field_range_into(const float* const* h_fields, uint64_t n, uint32_t F, int* keys,
                     float* h_minmax, hipStream_t s) {
    int rc = range_keys_reset(keys, F, s);
    if (rc == GPZ_OK && n > 0) rc = to_status(launch_field_range(h_fields, n, F, keys, s));
    int h[2 * kMaxFields];
    if (rc == GPZ_OK)
        rc = to_status(hipMemcpyAsync(h, keys, 8ull * F, hipMemcpyDeviceToHost, s));
    if (rc == GPZ_OK) rc = to_status(hipStreamSynchronize(s));
    else (void)hipStreamSynchronize(s);  // queued kernels may still use the keys
    if (rc) return rc;
    for (uint32_t f = 0; f < F; f++) range_from_keys(h[f], h[F + f], &h_minmax[2 * f], &h_minmax[2 * f + 1]);
    return GPZ_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device; the symbol lookup runs
// on the first call per device, with that device current.
int noalloc_scratch(int** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GPZ_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return GPZ_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GPZ_EDEVICE;
        g_scratch_ptr[dev] = static_cast<int*>(p);
    }
    *out = g_scratch_ptr[dev];
    return GPZ_OK;
}

}  // namespace

extern "C" {

void gpz_default_params(gpz_params* p, uint32_t nfields) {
    if (!p) return;
    p->block_size = 1024;
    p->seg_bits = 3;
    p->key_fields = nfields < 3 ? (nfields ? nfields : 1) : 3;
    p->flags = 0;
}

static uint64_t max_bytes(uint64_t n, uint32_t nfields, const gpz_params* pp, uint32_t vw) {
    gpz_params p = resolve(pp, nfields);
    if (!params_ok(nfields, p)) return 0;
    uint64_t nb = nblocks_of(n, p.block_size);
    return 4 * (prefix_words(n, nfields, p.block_size) + nb + (uint64_t)nfields * n * vw);
}

uint64_t gpz_max_compressed_bytes(uint64_t n, uint32_t nfields, const gpz_params* pp) {
    return max_bytes(n, nfields, pp, 1);
}

uint64_t gpz_max_compressed_bytes_f64(uint64_t n, uint32_t nfields, const gpz_params* pp) {
    return max_bytes(n, nfields, pp, 2);
}

uint64_t gpz_compress_workspace_bytes(uint64_t n, uint32_t nfields, const gpz_params* pp) {
    gpz_params p = resolve(pp, nfields);
    if (!params_ok(nfields, p)) return 0;
    return layout(n, nfields, p.block_size, 1, nullptr).bytes;
}

uint64_t gpz_compress_workspace_bytes_f64(uint64_t n, uint32_t nfields, const gpz_params* pp) {
    gpz_params p = resolve(pp, nfields);
    if (!params_ok(nfields, p)) return 0;
    return layout(n, nfields, p.block_size, 2, nullptr).bytes;
}

uint64_t gpz_decompress_workspace_bytes(void) { return 256; }

int gpz_compress(const float* const* h_fields, uint64_t n, uint32_t nfields, const float* h_eb,
                 const gpz_params* p, void* d_out, uint64_t out_capacity, uint64_t* h_out_bytes,
                 uint32_t* d_perm, void* d_ws, uint64_t ws_bytes, void* stream) {
    return compress_impl(reinterpret_cast<const void* const*>(h_fields), false, n, nfields, h_eb, p,
                         d_out, out_capacity, h_out_bytes, nullptr, d_perm, d_ws, ws_bytes,
                         static_cast<hipStream_t>(stream), true);
}

int gpz_compress_f64(const double* const* h_fields, uint64_t n, uint32_t nfields,
                     const float* h_eb, const gpz_params* p, void* d_out, uint64_t out_capacity,
                     uint64_t* h_out_bytes, uint32_t* d_perm, void* d_ws, uint64_t ws_bytes,
                     void* stream) {
    return compress_impl(reinterpret_cast<const void* const*>(h_fields), true, n, nfields, h_eb, p,
                         d_out, out_capacity, h_out_bytes, nullptr, d_perm, d_ws, ws_bytes,
                         static_cast<hipStream_t>(stream), true);
}

int gpz_compress_async(const float* const* h_fields, uint64_t n, uint32_t nfields,
                       const float* h_eb, const gpz_params* p, void* d_out, uint64_t out_capacity,
                       uint64_t* d_out_bytes, uint32_t* d_perm, void* d_ws, uint64_t ws_bytes,
                       void* stream) {
    if (!d_out_bytes || !d_ws) return GPZ_EINVAL;
    uint64_t need = gpz_max_compressed_bytes(n, nfields, p);
    if (need == 0 || out_capacity < need) return GPZ_EINVAL;
    return compress_impl(reinterpret_cast<const void* const*>(h_fields), false, n, nfields, h_eb, p,
                         d_out, out_capacity, nullptr, d_out_bytes, d_perm, d_ws, ws_bytes,
                         static_cast<hipStream_t>(stream), false);
}

// Shared body of the decompress entry points.  The wave-per-block decoder
// takes float32 streams at block sizes 256..2048 (it decodes a record with a
// wide field itself, with the generic record decoder); float64 streams and
// other block sizes go to the generic decoder.
static int decompress_impl(const void* d_in, uint64_t in_bytes, void* const* h_out, bool f64,
                           uint64_t n, uint32_t F, const gpz_params& p, uint32_t* d_err,
                           hipStream_t s, bool exact) {
    const uint32_t B = p.block_size;
    const uint64_t nb = nblocks_of(n, B);
    const uint64_t pre = prefix_words(n, F, B);
    const bool generic = f64 || !kernel_block_size(B);
    if (nb > ((uint64_t)1 << (generic ? 24 : 26))) return GPZ_EINVAL;
    if (in_bytes < 4 * pre || (exact && in_bytes % 4 != 0)) return GPZ_ECORRUPT;
    // (no blocks: the decode launch checks the header and eb table on the
    // device, so this path never waits for the stream either)
    DecodeArgs da{};
    da.in = static_cast<const uint32_t*>(d_in);
    da.in_words = in_bytes / 4;
    for (uint32_t f = 0; f < F; f++) da.y[f] = n ? static_cast<float*>(h_out[f]) : nullptr;
    da.n = n;
    da.F = F;
    da.K = p.seg_bits;
    da.KF = p.key_fields;
    da.B = B;
    da.nblocks = (uint32_t)nb;
    da.prefix = pre;
    da.err = d_err;
    da.exact = exact ? 1u : 0u;
    da.f64 = f64 ? 1u : 0u;
    int rc = to_status(launch_fill_u32(d_err, 0u, 1, s));
    Timer tm(s);
    if (generic && nb > 0) {
        tm.begin(kGeneric);
        if (rc == GPZ_OK) rc = to_status(launch_decode_generic(da, s));
        tm.end();
        return rc;
    }
    tm.begin(kDecode);
    if (rc == GPZ_OK) rc = to_status(launch_decode(da, s));
    tm.end();
    return rc;
}

// Host copy of a stream's header: its parameters and flags (synchronizes).
static int read_header(const void* d_in, uint64_t in_bytes, hipStream_t s, gpz_info* info) {
    if (in_bytes < 4 * kHeaderWords) return GPZ_ECORRUPT;
    uint32_t hdr[kHeaderWords];
    if (hipMemcpyAsync(hdr, d_in, sizeof(hdr), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GPZ_EDEVICE;
    return gpz_inspect(hdr, sizeof(hdr), info);
}

// Synchronous decompression of either value type.
static int decompress_sync(const void* d_in, uint64_t in_bytes, void* const* h_fields_out,
                           bool f64, uint64_t n, uint32_t nfields, void* d_ws, uint64_t ws_bytes,
                           hipStream_t s) {
    if (!d_in || nfields < 1 || nfields > kMaxFields) return GPZ_EINVAL;
    if (n > 0 && !h_fields_out) return GPZ_EINVAL;
    for (uint32_t f = 0; n > 0 && f < nfields; f++)
        if (!h_fields_out[f]) return GPZ_EINVAL;
    gpz_info info;
    int rc = read_header(d_in, in_bytes, s, &info);
    if (rc) return rc;
    if (info.n != n || info.nfields != nfields) return GPZ_EINVAL;
    // the caller's value type must be the stream's
    if (((info.flags & GPZ_STREAM_F64) != 0) != f64) return GPZ_EINVAL;
    gpz_params p{info.block_size, info.seg_bits, info.key_fields, 0};
    uint32_t* err = static_cast<uint32_t*>(d_ws);
    bool owned = false;
    if (!err) {
        if (alloc_fault() || hipMalloc(&err, 256) != hipSuccess) return GPZ_ENOMEM;
        owned = true;
    } else if (ws_bytes < gpz_decompress_workspace_bytes()) {
        return GPZ_EINVAL;
    }
    rc = decompress_impl(d_in, in_bytes, h_fields_out, f64, n, nfields, p, err, s, true);
    uint32_t e = 0;
    if (rc == GPZ_OK) rc = to_status(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, s));
    if (rc == GPZ_OK) rc = to_status(hipStreamSynchronize(s));
    if (owned) {
        if (rc != GPZ_OK) (void)hipStreamSynchronize(s);  // queued kernels may use the flag
        (void)hipFree(err);
    }
    if (rc == GPZ_OK && e) rc = GPZ_ECORRUPT;
    return rc;
}

int gpz_decompress(const void* d_in, uint64_t in_bytes, float* const* h_fields_out, uint64_t n,
                   uint32_t nfields, void* d_ws, uint64_t ws_bytes, void* stream) {
    return decompress_sync(d_in, in_bytes, reinterpret_cast<void* const*>(h_fields_out), false, n,
                           nfields, d_ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int gpz_decompress_f64(const void* d_in, uint64_t in_bytes, double* const* h_fields_out,
                       uint64_t n, uint32_t nfields, void* d_ws, uint64_t ws_bytes,
                       void* stream) {
    return decompress_sync(d_in, in_bytes, reinterpret_cast<void* const*>(h_fields_out), true, n,
                           nfields, d_ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int gpz_decompress_async(const void* d_in, uint64_t in_bytes, float* const* h_fields_out,
                         uint64_t n, uint32_t nfields, const gpz_params* pp, uint32_t* d_error,
                         void* stream) {
    if (!d_in || !d_error || nfields < 1 || nfields > kMaxFields) return GPZ_EINVAL;
    if (n > 0 && !h_fields_out) return GPZ_EINVAL;
    for (uint32_t f = 0; n > 0 && f < nfields; f++)
        if (!h_fields_out[f]) return GPZ_EINVAL;
    gpz_params p = resolve(pp, nfields);
    if (!params_ok(nfields, p)) return GPZ_EINVAL;
    return decompress_impl(d_in, in_bytes, reinterpret_cast<void* const*>(h_fields_out), false, n,
                           nfields, p, d_error, static_cast<hipStream_t>(stream), false);
}

uint64_t gpz_stats_workspace_bytes(uint32_t nfields) {
    if (nfields < 1 || nfields > kMaxFields) return 0;
    return stats_ws_bytes(nfields);
}

int gpz_error_stats(const float* const* h_orig, const float* const* h_recon,
                    const uint32_t* d_perm, uint64_t n, uint32_t nfields, const float* h_eb,
                    gpz_field_error* h_out, double* h_psnr, void* d_ws, uint64_t ws_bytes,
                    void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nfields < 1 || nfields > kMaxFields || !h_eb || !h_out) return GPZ_EINVAL;
    if (n > 0 && (!h_orig || !h_recon)) return GPZ_EINVAL;
    for (uint32_t f = 0; n > 0 && f < nfields; f++)
        if (!h_orig[f] || !h_recon[f]) return GPZ_EINVAL;
    const uint32_t F = nfields;
    char* ws = nullptr;
    bool owned = false;
    int rc = take_ws(d_ws, ws_bytes, stats_ws_bytes(F), &ws, &owned);
    if (rc) return rc;
    // per field: violation count, maximum-error bits, sum of squares (8 bytes
    // each), then the range keys of the originals (2 x 4 bytes)
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(ws);
    int* keys = reinterpret_cast<int*>(acc + 3 * F);
    double* sumsq = reinterpret_cast<double*>(acc + 2 * F);
    rc = to_status(launch_fill_u32(reinterpret_cast<uint32_t*>(acc), 0u, 6ull * F, s));
    if (rc == GPZ_OK) rc = range_keys_reset(keys, F, s);
    if (rc == GPZ_OK && n > 0)
        rc = to_status(launch_bound_check(h_orig, h_recon, d_perm, n, F, h_eb, acc, acc + F,
                                          sumsq, s));
    if (rc == GPZ_OK && n > 0) rc = to_status(launch_field_range(h_orig, n, F, keys, s));
    std::vector<unsigned long long> h(4 * F);
    if (rc == GPZ_OK)
        rc = to_status(hipMemcpyAsync(h.data(), acc, 32ull * F, hipMemcpyDeviceToHost, s));
    if (rc == GPZ_OK) rc = to_status(hipStreamSynchronize(s));
    else (void)hipStreamSynchronize(s);  // queued kernels may still use the buffer
    if (owned) (void)hipFree(ws);
    if (rc) return rc;
    // Normalized RMSE of every field over its original finite range, and the
    // aggregate PSNR of the rate-distortion analysis (Sec. 3.1):
    // -20 log10 sqrt(mean over fields of NRMSE^2).
    const int* hk = reinterpret_cast<const int*>(h.data() + 3 * F);
    double mean = 0.0;
    for (uint32_t f = 0; f < F; f++) {
        gpz_field_error& e = h_out[f];
        e.violations = h[f];
        memcpy(&e.max_abs_err, &h[F + f], 8);
        memcpy(&e.sum_sq_err, &h[2 * F + f], 8);
        range_from_keys(hk[f], hk[F + f], &e.min, &e.max);
        const double range = (double)e.max - (double)e.min;
        const double rmse = n ? sqrt(e.sum_sq_err / (double)n) : 0.0;
        e.nrmse = range > 0.0 ? rmse / range : (rmse == 0.0 ? 0.0 : INFINITY);
        mean += e.nrmse * e.nrmse;
    }
    if (h_psnr) *h_psnr = -20.0 * log10(sqrt(mean / (double)F));
    return GPZ_OK;
}

int gpz_bound_check(const float* const* h_orig, const float* const* h_recon,
                    const uint32_t* d_perm, uint64_t n, uint32_t nfields, const float* h_eb,
                    uint64_t* h_violations, double* h_max_abs_err, void* d_ws, uint64_t ws_bytes,
                    void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nfields < 1 || nfields > kMaxFields || !h_eb || !h_violations || !h_max_abs_err)
        return GPZ_EINVAL;
    if (n > 0 && (!h_orig || !h_recon)) return GPZ_EINVAL;
    for (uint32_t f = 0; n > 0 && f < nfields; f++)
        if (!h_orig[f] || !h_recon[f]) return GPZ_EINVAL;
    const uint32_t F = nfields;
    char* ws = nullptr;
    bool owned = false;
    int rc = take_ws(d_ws, ws_bytes, stats_ws_bytes(F), &ws, &owned);
    if (rc) return rc;
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(ws);
    rc = to_status(launch_fill_u32(reinterpret_cast<uint32_t*>(acc), 0u, 4ull * F, s));
    if (rc == GPZ_OK && n > 0)
        rc = to_status(launch_bound_check(h_orig, h_recon, d_perm, n, F, h_eb, acc, acc + F,
                                          nullptr, s));
    std::vector<unsigned long long> h(2 * F);
    if (rc == GPZ_OK)
        rc = to_status(hipMemcpyAsync(h.data(), acc, 16ull * F, hipMemcpyDeviceToHost, s));
    if (rc == GPZ_OK) rc = to_status(hipStreamSynchronize(s));
    else (void)hipStreamSynchronize(s);
    if (owned) (void)hipFree(ws);
    if (rc) return rc;
    for (uint32_t f = 0; f < F; f++) {
        h_violations[f] = h[f];
        memcpy(&h_max_abs_err[f], &h[F + f], 8);
    }
    return GPZ_OK;
}

int gpz_stream_stats(const void* d_in, uint64_t in_bytes, uint64_t n, uint32_t nfields,
                     uint64_t* h_outliers, uint64_t* h_raw_blocks, void* d_ws, uint64_t ws_bytes,
                     void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!d_in || nfields < 1 || nfields > kMaxFields || !h_outliers || !h_raw_blocks)
        return GPZ_EINVAL;
    if (d_ws && ws_bytes < stats_ws_bytes(nfields)) return GPZ_EINVAL;
    if (in_bytes < 4 * kHeaderWords) return GPZ_ECORRUPT;
    uint32_t hdr[kHeaderWords];
    if (hipMemcpyAsync(hdr, d_in, sizeof(hdr), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GPZ_EDEVICE;
    gpz_info info;
    int rc = gpz_inspect(hdr, sizeof(hdr), &info);
    if (rc) return rc;
    if (info.n != n || info.nfields != nfields) return GPZ_EINVAL;
    const uint64_t prefix = prefix_words(n, nfields, info.block_size);
    if (4 * prefix > in_bytes) return GPZ_ECORRUPT;
    char* ws = nullptr;
    bool owned = false;
    rc = take_ws(d_ws, ws_bytes, stats_ws_bytes(nfields), &ws, &owned);
    if (rc) return rc;
    // outliers per field, raw blocks, error flag
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(ws);
    uint32_t* err = reinterpret_cast<uint32_t*>(acc + nfields + 1);
    rc = to_status(launch_fill_u32(reinterpret_cast<uint32_t*>(acc), 0u, 2ull * (nfields + 2), s));
    if (rc == GPZ_OK)
        rc = to_status(launch_stream_stats(static_cast<const uint32_t*>(d_in), in_bytes / 4, n,
                                           nfields, info.block_size, acc, acc + nfields, err, s));
    std::vector<unsigned long long> h(nfields + 2);
    if (rc == GPZ_OK)
        rc = to_status(hipMemcpyAsync(h.data(), acc, 8ull * (nfields + 2), hipMemcpyDeviceToHost, s));
    if (rc == GPZ_OK) rc = to_status(hipStreamSynchronize(s));
    else (void)hipStreamSynchronize(s);  // queued kernels may still use the buffer
    if (owned) (void)hipFree(ws);
    if (rc) return rc;
    if (h[nfields + 1] & 0xFFFFFFFFull) return GPZ_ECORRUPT;
    for (uint32_t f = 0; f < nfields; f++) h_outliers[f] = h[f];
    *h_raw_blocks = h[nfields];
    return GPZ_OK;
}

int gpz_field_range(const float* const* h_fields, uint64_t n, uint32_t nfields, float* h_minmax,
                    void* d_ws, uint64_t ws_bytes, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nfields < 1 || nfields > kMaxFields || !h_minmax) return GPZ_EINVAL;
    if (n > 0 && !h_fields) return GPZ_EINVAL;
    for (uint32_t f = 0; n > 0 && f < nfields; f++)
        if (!h_fields[f]) return GPZ_EINVAL;
    char* ws = nullptr;
    bool owned = false;
    int rc = take_ws(d_ws, ws_bytes, stats_ws_bytes(nfields), &ws, &owned);
    if (rc) return rc;
    rc = field_range_into(h_fields, n, nfields, reinterpret_cast<int*>(ws), h_minmax, s);
    if (owned) (void)hipFree(ws);
    return rc;
}

int gpz_field_range_async(const float* const* h_fields, uint64_t n, uint32_t nfields,
                          float* d_minmax, void* d_ws, uint64_t ws_bytes, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nfields < 1 || nfields > kMaxFields || !d_minmax || !d_ws) return GPZ_EINVAL;
    if (ws_bytes < stats_ws_bytes(nfields)) return GPZ_EINVAL;
    if (n > 0 && !h_fields) return GPZ_EINVAL;
    for (uint32_t f = 0; n > 0 && f < nfields; f++)
        if (!h_fields[f]) return GPZ_EINVAL;
    int* keys = static_cast<int*>(d_ws);
    int rc = range_keys_reset(keys, nfields, s);
    if (rc == GPZ_OK && n > 0) rc = to_status(launch_field_range(h_fields, n, nfields, keys, s));
    if (rc == GPZ_OK) rc = to_status(launch_range_to_floats(keys, nfields, d_minmax, s));
    return rc;
}

int gpz_field_range_noalloc(const float* const* h_fields, uint64_t n, uint32_t nfields,
                            float* h_minmax, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nfields < 1 || nfields > kMaxFields || !h_minmax) return GPZ_EINVAL;
    if (n > 0 && !h_fields) return GPZ_EINVAL;
    for (uint32_t f = 0; n > 0 && f < nfields; f++)
        if (!h_fields[f]) return GPZ_EINVAL;
    int* keys = nullptr;
    int rc = noalloc_scratch(&keys);
    if (rc) return rc;
    // the keys are reset by fill kernels inside field_range_into before use
    return field_range_into(h_fields, n, nfields, keys, h_minmax, s);
}

float gpz_rel_to_abs(float rel, float lo, float hi) {
    float eb = (float)((double)rel * ((double)hi - (double)lo));
    if (!(eb >= 0x1p-120f)) eb = rel;
    if (eb > 0x1p120f) eb = 0x1p120f;
    return eb;
}

int gpz_inspect(const void* h_prefix, uint64_t bytes, gpz_info* out) {
    if (!h_prefix || !out) return GPZ_EINVAL;
    if (bytes < 4 * kHeaderWords) return GPZ_ECORRUPT;
    uint32_t w[kHeaderWords];
    memcpy(w, h_prefix, sizeof(w));
    const uint32_t flags = w[1] >> 16;
    if (w[0] != kMagic || (w[1] & 0xFFFFu) != kVersion ||
        (flags & ~(uint32_t)(GPZ_STREAM_F64 | GPZ_STREAM_WIDE)) != 0)
        return GPZ_ECORRUPT;
    gpz_params p{w[5], w[6] & 0xFFu, (w[6] >> 8) & 0xFFu, 0};
    if ((w[6] >> 16) != 0 || !params_ok(w[4], p)) return GPZ_ECORRUPT;
    uint64_t n = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
    uint64_t nb = nblocks_of(n, p.block_size);
    if (nb > 0xFFFFFFFFull || w[7] != (uint32_t)nb) return GPZ_ECORRUPT;
    out->n = n;
    out->nfields = w[4];
    out->block_size = p.block_size;
    out->seg_bits = p.seg_bits;
    out->key_fields = p.key_fields;
    out->nblocks = nb;
    out->flags = flags;
    return GPZ_OK;
}

int gpz_set_timing(int enable) {
    g_timing = enable != 0 ? (1u << kKinds) - 1u : 0u;
    return GPZ_OK;
}

int gpz_set_timing_kinds(uint32_t mask) {
    if (mask >> kKinds) return GPZ_EINVAL;
    g_timing = mask;
    return GPZ_OK;
}

int gpz_timing_collect(double* total_ms, uint32_t* counts, int nkinds) {
    if (!total_ms || !counts || nkinds < 1) return GPZ_EINVAL;
    for (int k = 0; k < nkinds; k++) {
        total_ms[k] = 0.0;
        counts[k] = 0;
    }
    int rc = GPZ_OK;
    for (auto& t : g_log) {
        float ms = 0.0f;
        if (hipEventSynchronize(t.b) != hipSuccess ||
            hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess)
            rc = GPZ_EDEVICE;
        if (t.kind < nkinds) {
            total_ms[t.kind] += ms;
            counts[t.kind]++;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_log.clear();
    return rc;
}

const char* gpz_strerror(int status) {
    switch (status) {
        case GPZ_OK: return "ok";
        case GPZ_EINVAL: return "invalid argument";
        case GPZ_ENOSPC: return "output buffer too small";
        case GPZ_ECORRUPT: return "corrupt or inconsistent stream";
        case GPZ_EDEVICE: return "HIP runtime error";
        case GPZ_ENOMEM: return "workspace allocation failed";
        case GPZ_EUNSUPPORTED: return "request without a gfx950 kernel (single pass with float64 or a block size outside 256..2048)";
        default: return "unknown status";
    }
}

}  // extern "C"
