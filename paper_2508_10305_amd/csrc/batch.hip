// Batched form: many snapshots of uneven sizes compressed (or decompressed)
// by persistent kernels that pull blocks from a device work queue, the whole
// sequence optionally captured once into a HIP graph and replayed.  Job
// tables and launch descriptors live in device memory, so a batch can be
// rebound to new jobs (within its capacities) without allocating and without
// recapturing its graphs.  Every job's stream is the same, byte for byte, as
// the one gpz_compress writes for that snapshot alone.
#include <math.h>
#include <string.h>


#include "gpz.h"
#include "gpz_internal.h"

using namespace gpz;

struct gpz_batch {
    gpz_params p{};
    gpz_batch_config cfg{};
    BatchShape shape{};
    uint32_t max_jobs = 0;
    uint64_t max_blocks = 0, max_super = 0, ws_capacity = 0;
    uint32_t njobs = 0;
    bool can_compress = false, can_decompress = false;
    // one device allocation holding every table below
    void* tables = nullptr;
    EncodeArgs* d_enc = nullptr;
    ScanArgs* d_scan = nullptr;
    CopyArgs* d_copy = nullptr;
    DecodeArgs* d_dec = nullptr;
    BatchLaunch* d_launch = nullptr;
    uint32_t* d_full_prefix = nullptr;
    uint32_t* d_block_prefix = nullptr;
    uint32_t* d_tail = nullptr;
    uint32_t* d_counters = nullptr;  // [0] encode queue, [1] decode queue
    uint32_t* d_lens = nullptr;
    uint32_t* d_supsum = nullptr;
    uint64_t* d_supoff = nullptr;
    uint64_t* d_total = nullptr;
    uint64_t* d_sizes = nullptr;   // stream size per job
    uint32_t* d_errors = nullptr;  // decode error flag per job
    // blocks left to the generic encoder (their grid needs 64-bit steps):
    // one list per job inside d_defer, its length and the job's wide-record
    // flag (d_dcount and d_wide are contiguous, cleared by one fill)
    uint32_t* d_defer = nullptr;
    uint32_t* d_dcount = nullptr;
    uint32_t* d_wide = nullptr;
    // Pinned host image of the job tables and launch descriptor (the first
    // upload_bytes of `tables`), uploaded with one asynchronous copy per bind;
    // `uploaded` marks the last copy, after which the image may be rewritten.
    char* h_tables = nullptr;
    uint64_t upload_bytes = 0;
    hipEvent_t uploaded = nullptr;
    hipStream_t capture = nullptr;
    hipGraphExec_t g_comp = nullptr, g_dec = nullptr;
};

namespace {

bool eb_ok_host(float eb) { return isfinite(eb) && eb >= 0x1p-120f && eb <= 0x1p120f; }

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

uint32_t slot_words_of(uint32_t F, uint32_t B) {
    return (uint32_t)((1 + (uint64_t)F * B + 3) & ~uint64_t(3));
}

gpz_params resolve(const gpz_params* pp, uint32_t F) {
    gpz_params p;
    gpz_default_params(&p, F);
    if (pp) p = *pp;
    return p;
}

int validate_params(const gpz_params& p) {
    if (p.block_size != 256 && p.block_size != 512 && p.block_size != 1024 &&
        p.block_size != 2048)
        return (p.block_size >= 64 && p.block_size <= 4096 &&
                (p.block_size & (p.block_size - 1)) == 0)
                   ? GPZ_EUNSUPPORTED
                   : GPZ_EINVAL;
    if (p.seg_bits > 5 || p.flags != 0 || p.key_fields < 1 || p.key_fields > 3)
        return GPZ_EINVAL;
    return GPZ_OK;
}

int validate_jobs(const gpz_job* jobs, uint32_t njobs, const gpz_params& p) {
    if (!jobs && njobs) return GPZ_EINVAL;
    for (uint32_t j = 0; j < njobs; j++) {
        const gpz_job& J = jobs[j];
        if (J.nfields < 1 || J.nfields > kMaxFields || p.key_fields > J.nfields) return GPZ_EINVAL;
        if (!J.eb || !J.out) return GPZ_EINVAL;
        if (nblocks_of(J.n, p.block_size) > ((uint64_t)1 << 26)) return GPZ_EINVAL;
        for (uint32_t f = 0; f < J.nfields; f++) {
            if (!eb_ok_host(J.eb[f])) return GPZ_EINVAL;
            if (J.n > 0 && J.fields && !J.fields[f]) return GPZ_EINVAL;
            if (J.n > 0 && J.dec_fields && !J.dec_fields[f]) return GPZ_EINVAL;
        }
        const uint64_t nb = nblocks_of(J.n, p.block_size);
        const uint64_t maxb =
            4 * (prefix_words(J.n, J.nfields, p.block_size) + nb + (uint64_t)J.nfields * J.n);
        // a compressing batch never runs out of space; a stream to decompress
        // only has to hold its header
        if (J.fields && J.out_capacity < maxb) return GPZ_EINVAL;
        if (J.out_capacity < 4 * prefix_words(J.n, J.nfields, p.block_size)) return GPZ_EINVAL;
    }
    return GPZ_OK;
}

// Record slots the batch workspace must hold for a job: none when the job
// brings its own or only decompresses.
uint64_t job_workspace(const gpz_job& J, uint32_t B) {
    if (!J.fields || J.ws) return 0;
    return align256(nblocks_of(J.n, B) * (uint64_t)slot_words_of(J.nfields, B) * 4);
}

uint64_t jobs_workspace(const gpz_job* jobs, uint32_t njobs, uint32_t B) {
    uint64_t total = 0;
    for (uint32_t j = 0; j < njobs; j++) total += job_workspace(jobs[j], B);
    return total;
}

int to_status(hipError_t e) { return e == hipSuccess ? GPZ_OK : GPZ_EDEVICE; }

int enqueue_compress(gpz_batch* b, hipStream_t s) {
    int rc = to_status(launch_fill_u32(b->d_counters, 0u, 1, s));
    if (rc == GPZ_OK) rc = to_status(launch_fill_u32(b->d_supsum, 0u, b->max_super + 1, s));
    if (rc == GPZ_OK) rc = to_status(launch_fill_u32(b->d_dcount, 0u, 2ull * b->max_jobs, s));
    if (rc == GPZ_OK) rc = to_status(launch_encode_batch(b->d_enc, b->d_launch, b->shape, s));
    if (rc == GPZ_OK)
        rc = to_status(launch_encode_generic_batch(b->d_enc, b->d_launch, b->p.block_size,
                                                   (uint32_t)b->max_blocks, s));
    if (rc == GPZ_OK) rc = to_status(launch_scan_batch(b->d_scan, b->d_launch, b->shape, s));
    if (rc == GPZ_OK) rc = to_status(launch_copy_batch(b->d_copy, b->d_launch, b->shape, s));
    return rc;
}

int enqueue_decompress(gpz_batch* b, hipStream_t s) {
    int rc = to_status(launch_fill_u32(b->d_counters + 1, 0u, 1, s));
    if (rc == GPZ_OK) rc = to_status(launch_fill_u32(b->d_errors, 0u, b->max_jobs, s));
    if (rc == GPZ_OK) rc = to_status(launch_decode_batch(b->d_dec, b->d_launch, b->shape, s));
    return rc;
}

int capture(gpz_batch* b, int (*enqueue)(gpz_batch*, hipStream_t), hipGraphExec_t* exec) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed) != hipSuccess)
        return GPZ_EDEVICE;
    int rc = enqueue(b, b->capture);
    hipError_t e = hipStreamEndCapture(b->capture, &g);
    if (rc == GPZ_OK && e != hipSuccess) rc = GPZ_EDEVICE;
    if (rc == GPZ_OK && hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess)
        rc = GPZ_EDEVICE;
    if (g) (void)hipGraphDestroy(g);
    return rc;
}

template <typename T>
T* host_image(gpz_batch* b, T* device_ptr) {
    return reinterpret_cast<T*>(b->h_tables +
                                (reinterpret_cast<char*>(device_ptr) - static_cast<char*>(b->tables)));
}

// Host image of the tables of a job list, then one asynchronous upload on
// stream s (ordered before whatever s runs next).
int bind(gpz_batch* b, const gpz_job* jobs, uint32_t njobs, void* d_ws, uint64_t ws_bytes,
         hipStream_t s) {
    const gpz_params& p = b->p;
    const uint32_t B = p.block_size;
    int rc = validate_jobs(jobs, njobs, p);
    if (rc) return rc;
    if (njobs > b->max_jobs) return GPZ_EINVAL;
    uint64_t nblocks_all = 0, nsuper_all = 0;
    for (uint32_t j = 0; j < njobs; j++) {
        const uint64_t nb = nblocks_of(jobs[j].n, B);
        nblocks_all += nb;
        nsuper_all += nsuper_of(nb);
    }
    if (nblocks_all > b->max_blocks || nsuper_all > b->max_super) return GPZ_EINVAL;
    const uint64_t ws_need = jobs_workspace(jobs, njobs, B);
    if (ws_need > ws_bytes || (ws_need && !d_ws)) return GPZ_EINVAL;

    // the previous upload must have read the image before it is rewritten
    if (hipEventSynchronize(b->uploaded) != hipSuccess) return GPZ_EDEVICE;
    EncodeArgs* enc = host_image(b, b->d_enc);
    ScanArgs* scan = host_image(b, b->d_scan);
    CopyArgs* copy = host_image(b, b->d_copy);
    DecodeArgs* dec = host_image(b, b->d_dec);
    uint32_t* full_prefix = host_image(b, b->d_full_prefix);
    uint32_t* block_prefix = host_image(b, b->d_block_prefix);
    uint32_t* tails = host_image(b, b->d_tail);
    uint32_t ntail = 0;
    full_prefix[0] = block_prefix[0] = 0;
    bool can_c = true, can_d = true;
    char* ws = static_cast<char*>(d_ws);
    uint64_t ws_at = 0, blk_at = 0, sup_at = 0;
    for (uint32_t j = 0; j < njobs; j++) {
        const gpz_job& J = jobs[j];
        const uint32_t F = J.nfields;
        const uint64_t nb = nblocks_of(J.n, B);
        const uint32_t sw = slot_words_of(F, B);
        full_prefix[j + 1] = full_prefix[j] + (uint32_t)(J.n / B);
        block_prefix[j + 1] = block_prefix[j] + (uint32_t)nb;
        if (J.n % B) tails[ntail++] = j;
        if (J.n > 0 && !J.fields) can_c = false;
        if (J.n > 0 && !J.dec_fields) can_d = false;
        uint32_t* temp = !J.fields ? nullptr
                         : J.ws   ? static_cast<uint32_t*>(J.ws)
                                  : reinterpret_cast<uint32_t*>(ws + ws_at);
        ws_at += job_workspace(J, B);
        EncodeArgs& e = enc[j];
        ScanArgs& sa = scan[j];
        CopyArgs& ca = copy[j];
        DecodeArgs& da = dec[j];
        memset(&e, 0, sizeof(e));
        memset(&sa, 0, sizeof(sa));
        memset(&ca, 0, sizeof(ca));
        memset(&da, 0, sizeof(da));
        for (uint32_t f = 0; f < F; f++) {
            e.x[f] = J.fields && J.n ? J.fields[f] : nullptr;
            e.eb[f] = J.eb[f];
            e.twoeb[f] = 2.0f * J.eb[f];
            e.inv[f] = 1.0f / e.twoeb[f];
            memcpy(&sa.eb_bits[f], &J.eb[f], 4);
            da.y[f] = J.dec_fields && J.n ? J.dec_fields[f] : nullptr;
        }
        e.n = J.n;
        e.F = F;
        e.K = p.seg_bits;
        e.KF = p.key_fields;
        e.B = B;
        e.nblocks = (uint32_t)nb;
        e.slot_words = sw;
        e.temp = temp;
        e.lens = b->d_lens + blk_at;
        e.supsum = b->d_supsum + sup_at;
        e.perm = nullptr;
        e.defer = b->d_defer + blk_at;
        e.defer_count = b->d_dcount + j;
        e.wide_flag = b->d_wide + j;
        sa.wide_flag = e.wide_flag;
        sa.supsum = e.supsum;
        sa.supoff = b->d_supoff + sup_at;
        sa.total_bytes = b->d_total + j;
        sa.ext_bytes = b->d_sizes + j;
        sa.nsuper = (uint32_t)nsuper_of(nb);
        sa.prefix = prefix_words(J.n, F, B);
        sa.out = static_cast<uint32_t*>(J.out);
        sa.capacity = J.out_capacity;
        sa.n = J.n;
        sa.F = F;
        sa.B = B;
        sa.K = p.seg_bits;
        sa.KF = p.key_fields;
        sa.nblocks = (uint32_t)nb;
        ca.temp = temp;
        ca.lens = e.lens;
        ca.supoff = sa.supoff;
        ca.total_bytes = sa.total_bytes;
        ca.out = sa.out;
        ca.capacity = J.out_capacity;
        ca.slot_words = sw;
        ca.nblocks = (uint32_t)nb;
        ca.F = F;
        da.in = static_cast<const uint32_t*>(J.out);
        da.in_words = J.out_capacity / 4;
        da.n = J.n;
        da.F = F;
        da.K = p.seg_bits;
        da.KF = p.key_fields;
        da.B = B;
        da.nblocks = (uint32_t)nb;
        da.prefix = sa.prefix;
        da.err = b->d_errors + j;
        da.exact = 0;
        blk_at += nb;
        sup_at += nsuper_of(nb);
    }
    BatchLaunch& L = *host_image(b, b->d_launch);
    L = BatchLaunch{};
    L.njobs = njobs;
    L.total_full = full_prefix[njobs];
    L.total_blocks = block_prefix[njobs];
    L.ntail = ntail;
    L.tile = b->cfg.tile;
    L.full_prefix = b->d_full_prefix;
    L.block_prefix = b->d_block_prefix;
    L.tail_jobs = b->d_tail;
    L.counter = b->d_counters;

    // one copy from pinned memory, queued on s: it runs after the work
    // already on s and before the launches that follow
    hipError_t e = hipMemcpyAsync(b->tables, b->h_tables, b->upload_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, s);
    if (e != hipSuccess) return GPZ_EDEVICE;
    b->njobs = njobs;
    b->can_compress = can_c;
    b->can_decompress = can_d;
    return GPZ_OK;
}

}  // namespace

extern "C" {

void gpz_default_batch_config(gpz_batch_config* c) {
    if (!c) return;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
    c->grid = (uint32_t)cus * 8;
    c->tile = 1;
    c->use_graph = 1;
    c->max_jobs = 0;
    c->max_blocks = 0;
}

uint64_t gpz_batch_workspace_bytes(const gpz_job* jobs, uint32_t njobs, const gpz_params* pp) {
    gpz_params p = resolve(pp, jobs && njobs ? jobs[0].nfields : 3);
    if (validate_params(p) != GPZ_OK || validate_jobs(jobs, njobs, p) != GPZ_OK) return 0;
    uint64_t w = jobs_workspace(jobs, njobs, p.block_size);
    return w ? w : 256;
}

int gpz_batch_create(gpz_batch** out, const gpz_job* jobs, uint32_t njobs, const gpz_params* pp,
                     const gpz_batch_config* cfg, void* d_ws, uint64_t ws_bytes) {
    if (!out) return GPZ_EINVAL;
    *out = nullptr;
    gpz_params p = resolve(pp, jobs && njobs ? jobs[0].nfields : 3);
    int rc = validate_params(p);
    if (rc) return rc;
    rc = validate_jobs(jobs, njobs, p);
    if (rc) return rc;
    gpz_batch_config c;
    gpz_default_batch_config(&c);
    if (cfg) c = *cfg;
    if (c.tile == 0) return GPZ_EINVAL;
    const uint32_t B = p.block_size;
    uint64_t nblocks_all = 0, nsuper_all = 0;
    for (uint32_t j = 0; j < njobs; j++) {
        nblocks_all += nblocks_of(jobs[j].n, B);
        nsuper_all += nsuper_of(nblocks_of(jobs[j].n, B));
    }
    gpz_batch* b = new gpz_batch();
    b->p = p;
    b->cfg = c;
    b->max_jobs = c.max_jobs ? c.max_jobs : njobs;
    b->max_blocks = c.max_blocks ? c.max_blocks : nblocks_all;
    // every job adds at most one partially filled superblock
    b->max_super = c.max_blocks ? (c.max_blocks / kSuper + b->max_jobs) : nsuper_all;
    if (b->max_jobs < njobs || b->max_blocks < nblocks_all || b->max_super < nsuper_all ||
        b->max_blocks > ((uint64_t)1 << 30) || b->max_jobs == 0 ||
        (c.grid == 0 && b->max_blocks > ((uint64_t)1 << 26))) {
        // direct launches run one 64-lane workgroup per block of the
        // capacity: the dispatch size (64 * blocks) must fit 32 bits
        delete b;
        return GPZ_EINVAL;
    }
    b->shape.B = B;
    b->shape.grid = c.grid;
    b->shape.direct_grid = (uint32_t)(b->max_blocks ? b->max_blocks : 1);
    b->shape.scan_grid = b->max_jobs < 256 ? b->max_jobs : 256;
    b->shape.copy_grid = c.grid ? c.grid : 2048;  // persistent grids: 4-wave workgroups copying
    b->shape.tail_grid = b->max_jobs < 1024 ? b->max_jobs : 1024;  // every tail at once
    const uint32_t mj = b->max_jobs;
    const uint64_t mb = b->max_blocks, ms = b->max_super;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const uint64_t o_enc = take(sizeof(EncodeArgs) * mj);
    const uint64_t o_scan = take(sizeof(ScanArgs) * mj);
    const uint64_t o_copy = take(sizeof(CopyArgs) * mj);
    const uint64_t o_dec = take(sizeof(DecodeArgs) * mj);
    const uint64_t o_launch = take(sizeof(BatchLaunch));
    const uint64_t o_fp = take(4ull * (mj + 1));
    const uint64_t o_bp = take(4ull * (mj + 1));
    const uint64_t o_tail = take(4ull * (mj + 1));
    const uint64_t o_cnt = take(8);
    const uint64_t o_lens = take(4 * mb + 4);
    const uint64_t o_sups = take(4 * ms + 4);
    const uint64_t o_supo = take(8 * ms + 8);
    const uint64_t o_tot = take(8ull * mj);
    const uint64_t o_sizes = take(8ull * mj);
    const uint64_t o_err = take(4ull * mj);
    const uint64_t o_defer = take(4 * mb + 4);
    const uint64_t o_dcount = take(8ull * mj);  // counts, then wide flags
    if (hipMalloc(&b->tables, o) != hipSuccess) {
        delete b;
        return GPZ_ENOMEM;
    }
    char* base = static_cast<char*>(b->tables);
    b->d_enc = reinterpret_cast<EncodeArgs*>(base + o_enc);
    b->d_scan = reinterpret_cast<ScanArgs*>(base + o_scan);
    b->d_copy = reinterpret_cast<CopyArgs*>(base + o_copy);
    b->d_dec = reinterpret_cast<DecodeArgs*>(base + o_dec);
    b->d_launch = reinterpret_cast<BatchLaunch*>(base + o_launch);
    b->d_full_prefix = reinterpret_cast<uint32_t*>(base + o_fp);
    b->d_block_prefix = reinterpret_cast<uint32_t*>(base + o_bp);
    b->d_tail = reinterpret_cast<uint32_t*>(base + o_tail);
    b->d_counters = reinterpret_cast<uint32_t*>(base + o_cnt);
    b->d_lens = reinterpret_cast<uint32_t*>(base + o_lens);
    b->d_supsum = reinterpret_cast<uint32_t*>(base + o_sups);
    b->d_supoff = reinterpret_cast<uint64_t*>(base + o_supo);
    b->d_total = reinterpret_cast<uint64_t*>(base + o_tot);
    b->d_sizes = reinterpret_cast<uint64_t*>(base + o_sizes);
    b->d_errors = reinterpret_cast<uint32_t*>(base + o_err);
    b->d_defer = reinterpret_cast<uint32_t*>(base + o_defer);
    b->d_dcount = reinterpret_cast<uint32_t*>(base + o_dcount);
    b->d_wide = b->d_dcount + mj;
    b->upload_bytes = o_cnt;  // the tables and launch descriptor come first
    if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&b->h_tables), b->upload_bytes) != hipSuccess) {
        gpz_batch_destroy(b);
        return GPZ_EDEVICE;
    }
    memset(b->h_tables, 0, b->upload_bytes);
    // the first bind's upload is on the batch's own stream, waited for here
    // (the caller's streams are not ordered with it)
    rc = bind(b, jobs, njobs, d_ws, ws_bytes, b->capture);
    if (rc == GPZ_OK && hipStreamSynchronize(b->capture) != hipSuccess) rc = GPZ_EDEVICE;
    if (rc) {
        gpz_batch_destroy(b);
        return rc;
    }
    *out = b;
    return GPZ_OK;
}

int gpz_batch_rebind(gpz_batch* b, const gpz_job* jobs, uint32_t njobs, void* d_ws,
                     uint64_t ws_bytes, void* stream) {
    if (!b) return GPZ_EINVAL;
    // earlier work of this batch must be done before its tables change
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return GPZ_EDEVICE;
    return bind(b, jobs, njobs, d_ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int gpz_batch_compress(gpz_batch* b, void* stream) {
    if (!b) return GPZ_EINVAL;
    if (!b->can_compress) return GPZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!b->cfg.use_graph) return enqueue_compress(b, s);
    if (!b->g_comp) {
        int rc = capture(b, enqueue_compress, &b->g_comp);
        if (rc) return rc;
    }
    return to_status(hipGraphLaunch(b->g_comp, s));
}

int gpz_batch_decompress(gpz_batch* b, void* stream) {
    if (!b) return GPZ_EINVAL;
    if (!b->can_decompress) return GPZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!b->cfg.use_graph) return enqueue_decompress(b, s);
    if (!b->g_dec) {
        int rc = capture(b, enqueue_decompress, &b->g_dec);
        if (rc) return rc;
    }
    return to_status(hipGraphLaunch(b->g_dec, s));
}

const uint64_t* gpz_batch_sizes(const gpz_batch* b) { return b ? b->d_sizes : nullptr; }

const uint32_t* gpz_batch_errors(const gpz_batch* b) { return b ? b->d_errors : nullptr; }

int gpz_batch_destroy(gpz_batch* b) {
    if (!b) return GPZ_OK;
    (void)hipDeviceSynchronize();  // launches of this batch may still be queued
    if (b->g_comp) (void)hipGraphExecDestroy(b->g_comp);
    if (b->g_dec) (void)hipGraphExecDestroy(b->g_dec);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    if (b->h_tables) (void)hipHostFree(b->h_tables);
    if (b->tables) (void)hipFree(b->tables);
    delete b;
    return GPZ_OK;
}

}  // extern "C"
