// C-ABI of batched traces (tm_batch_*, declared in include/tetrt.h): one launch
// walks the rays of many meshes.  The job table lives in device memory; each
// job owns a contiguous range of blocks (and of binning chunks), so a block
// finds its job by a binary search over the table.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"
#include "handle.h"
#include "tetrt.h"

namespace {

using tetrt::fail;
using tetrt::hip_fail;

constexpr int64_t kMaxRays = (int64_t(1) << 32) - (int64_t(1) << 24);  // keeps blocks * threads < 2^32
constexpr int32_t kMaxJobs = 65536;
constexpr int64_t kPermAlign = 64;  // ints; each binned job's permutation starts on a 256-byte line

// The launch as captured in a graph; a new capture is needed when any differs.
struct Shape {
    int32_t n_jobs = -1, block = 0, chunk_log2 = 0, layout = -1, xcds = 1;
    int64_t blocks = -1, chunks = -1;
    bool steps = false;   // some job asks for step counts
    int32_t kernel = 1;   // 1 = one lane per ray, 3 = persistent waves on a queue
    int32_t qchunk = 0, refill = 0;   // kernel 3: rays per wave fetch, refill threshold
    int64_t qchunks = 0;  // kernel 3: chunks over all jobs
    float eps = 0.0f;     // the precision variant (kernel 1)
    bool operator==(const Shape& o) const {
        return n_jobs == o.n_jobs && block == o.block && chunk_log2 == o.chunk_log2 && layout == o.layout &&
               xcds == o.xcds && blocks == o.blocks && chunks == o.chunks && steps == o.steps &&
               kernel == o.kernel && qchunk == o.qchunk && refill == o.refill && qchunks == o.qchunks &&
               eps == o.eps;
    }
};

}  // namespace

struct tm_batch_s {
    int device = 0;
    int cus = 256;
    int32_t max_jobs = 0;
    int64_t max_rays = 0;
    tetrt::Job* d_table = nullptr;
    tetrt::Job* h_stage = nullptr;   // pinned staging copy of the table
    int32_t* d_perm = nullptr;       // binning permutations of every job
    uint32_t* d_cursor = nullptr;    // the queue kernel's counters
    hipEvent_t staged = nullptr;     // recorded after the last table copy
    bool copy_recorded = false;
    Shape shape;                     // of the current table
    std::vector<tm_job> jobs;        // the current jobs (the tuner sets them again)
    tm_trace_opts opts{};
    hipStream_t cap = nullptr;       // private stream for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Shape captured;
};

namespace {

void drop_graph(tm_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->captured = Shape{};
}

void release(tm_batch_s* b) {
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->d_table) (void)hipFree(b->d_table);
    if (b->d_perm) (void)hipFree(b->d_perm);
    if (b->d_cursor) (void)hipFree(b->d_cursor);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
}

// Validate the jobs and options and build the table on the host.
int build_table(tm_batch_s* b, int32_t n_jobs, const tm_job* jobs, const tm_trace_opts& o,
                std::vector<tetrt::Job>* table, Shape* shape) {
    if (n_jobs < 0 || n_jobs > b->max_jobs)
        return fail(TM_ERR_ARG, "tm_batch_set: n_jobs = %d out of range [0, %d]", n_jobs, b->max_jobs);
    if (n_jobs > 0 && !jobs) return fail(TM_ERR_ARG, "tm_batch_set: jobs is NULL");
    if (o.max_steps < 0) return fail(TM_ERR_ARG, "tm_batch_set: negative max_steps");
    if (o.block != 0 && o.block != 64 && o.block != 128 && o.block != 256)
        return fail(TM_ERR_ARG, "tm_batch_set: block must be 64, 128 or 256");
    if (o.kernel != 0 && o.kernel != 1 && o.kernel != 3)
        return fail(TM_ERR_ARG, "tm_batch_set: batches run one lane per ray or persistent waves on a queue "
                                "(kernel 0, 1 or 3)");
    if (o.queue_chunk < 0 || o.queue_chunk > 4096 || (o.queue_chunk & 63))
        return fail(TM_ERR_ARG, "tm_batch_set: queue_chunk must be a multiple of 64 in [64, 4096]");
    if (o.refill < 0 || o.refill > 64) return fail(TM_ERR_ARG, "tm_batch_set: refill must be in [0, 64]");
    if (!(o.eps >= 0.0f) || !(o.eps < 1.0f)) return fail(TM_ERR_ARG, "tm_batch_set: eps must be in [0, 1)");
    if (o.eps > 0.0f && o.kernel == 3)
        return fail(TM_ERR_ARG, "tm_batch_set: the precision variant (eps > 0) runs one lane per ray");
    if (o.sort < 0 || o.sort > 2) return fail(TM_ERR_ARG, "tm_batch_set: sort must be 0, 1 or 2");
    if (o.xcds < 0 || o.xcds > 64) return fail(TM_ERR_ARG, "tm_batch_set: xcds must be in [0, 64]");
    const int32_t block = o.block ? o.block : 256;
    const int32_t chunk_log2 = o.sort_chunk_log2 ? o.sort_chunk_log2 : 12;
    table->assign(size_t(n_jobs), tetrt::Job{});
    const int32_t kernel = o.kernel == 3 ? 3 : 1;
    const int32_t qchunk = o.queue_chunk ? o.queue_chunk : 64;
    int64_t blocks = 0, chunks = 0, rays = 0, perm_at = 0, qchunks = 0;
    int32_t layout = -1;
    for (int32_t k = 0; k < n_jobs; ++k) {
        const tm_job& j = jobs[k];
        tetrt::Job& J = (*table)[size_t(k)];
        if (!j.mesh) return fail(TM_ERR_ARG, "tm_batch_set: job %d: NULL mesh", k);
        if (j.mesh->device != b->device)
            return fail(TM_ERR_ARG, "tm_batch_set: job %d: mesh on device %d, batch on device %d", k,
                        j.mesh->device, b->device);
        if (layout >= 0 && j.mesh->layout != layout)
            return fail(TM_ERR_ARG, "tm_batch_set: job %d: record layout %d differs from job 0's %d", k,
                        j.mesh->layout, layout);
        layout = j.mesh->layout;
        if (j.n_rays < 0 || j.n_rays > int64_t(0x7FFFFFFF))
            return fail(TM_ERR_ARG, "tm_batch_set: job %d: n_rays = %lld out of range [0, 2^31)", k,
                        (long long)j.n_rays);
        if (j.n_rays > 0 && (!j.d_orig || !j.d_dir || !j.d_tri || !j.d_t || !j.d_bary))
            return fail(TM_ERR_ARG, "tm_batch_set: job %d: NULL required array", k);
        if ((reinterpret_cast<uintptr_t>(j.d_bary) & 7) || (reinterpret_cast<uintptr_t>(j.d_hit_tets) & 7))
            return fail(TM_ERR_ARG, "tm_batch_set: job %d: bary / hit_tets must be 8-byte aligned", k);
        rays += j.n_rays;
        if (rays > b->max_rays)
            return fail(TM_ERR_ARG, "tm_batch_set: more than max_rays = %lld rays in total",
                        (long long)b->max_rays);
        bool binned = false;
        int rc = tetrt::sort_config(j.mesh, o, j.n_rays, j.d_tmax != nullptr, &J.sc, &binned);
        if (rc != TM_OK) return rc;
        J.m = j.mesh->dev;
        tetrt::RayArgs& r = J.r;
        r.perm = nullptr;
        r.orig = j.d_orig;
        r.dir = j.d_dir;
        r.tmax = j.d_tmax;
        r.start_tet = j.d_start_tet;
        r.start_face = j.d_start_face;
        r.tri = j.d_tri;
        r.t = j.d_t;
        r.bary = j.d_bary;
        r.hit_tets = j.d_hit_tets;
        r.steps = j.d_steps;
        if (j.d_steps && j.n_rays > 0) shape->steps = true;
        r.fp64_steps = nullptr;
        r.n = j.n_rays;
        r.max_steps = o.max_steps > 0 ? o.max_steps : 65536;
        J.block0 = blocks;
        blocks += (j.n_rays + block - 1) / block;
        J.qchunk0 = qchunks;
        qchunks += (j.n_rays + qchunk - 1) / qchunk;
        J.chunk0 = chunks;
        if (binned && j.n_rays > 0) {
            r.perm = b->d_perm + perm_at;
            perm_at += (j.n_rays + kPermAlign - 1) / kPermAlign * kPermAlign;
            chunks += (j.n_rays + (int64_t(1) << chunk_log2) - 1) >> chunk_log2;
        }
    }
    shape->n_jobs = n_jobs;
    shape->block = block;
    shape->chunk_log2 = chunk_log2;
    shape->layout = layout < 0 ? 0 : layout;
    shape->blocks = blocks;
    shape->chunks = chunks;
    shape->kernel = kernel;
    shape->qchunk = qchunk;
    shape->refill = o.refill ? o.refill : (kernel == 3 ? 64 : 16);
    shape->qchunks = qchunks;
    shape->eps = o.eps;
    if (kernel == 3 && qchunks >= int64_t(0xFFFFFFFFu))
        return fail(TM_ERR_ARG, "tm_batch_set: too many queue chunks (raise queue_chunk)");
    // automatic: round-robin placement.  One contiguous range per XCD over a
    // whole batch splits jobs of unequal walks unevenly over the XCDs (measured
    // slower on many-mesh batches); the tuner tries it
    shape->xcds = o.xcds ? o.xcds : (kernel == 3 ? tetrt::xcd_count(b->cus) : 1);
    return TM_OK;
}

int set_jobs(tm_batch_s* b, int32_t n_jobs, const tm_job* jobs, const tm_trace_opts& o, hipStream_t s) {
    std::vector<tetrt::Job> table;
    Shape shape;
    int rc = build_table(b, n_jobs, jobs, o, &table, &shape);
    if (rc != TM_OK) return rc;
    hipError_t e;
    if (b->copy_recorded) {
        // the staging buffer is reused once the previous copy has read it
        e = hipEventSynchronize(b->staged);
        if (e != hipSuccess) return hip_fail(e, "tm_batch_set: wait for the previous table copy");
    }
    if (n_jobs > 0) {
        std::memcpy(b->h_stage, table.data(), table.size() * sizeof(tetrt::Job));
        e = hipMemcpyAsync(b->d_table, b->h_stage, table.size() * sizeof(tetrt::Job), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "tm_batch_set: table copy");
        e = hipEventRecord(b->staged, s);
        if (e != hipSuccess) return hip_fail(e, "tm_batch_set: event record");
        b->copy_recorded = true;
    }
    b->shape = shape;
    b->jobs.assign(jobs, jobs + n_jobs);
    b->opts = o;
    return TM_OK;
}

hipError_t enqueue(const tm_batch_s* b, hipStream_t s) {
    const Shape& sh = b->shape;
    if (sh.n_jobs <= 0 || sh.blocks <= 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (sh.chunks > 0) e = tetrt::launch_sort_batch(b->d_table, sh.n_jobs, sh.chunks, sh.chunk_log2, s);
    if (e != hipSuccess) return e;
    if (sh.kernel == 3) {
        tetrt::Queue q;
        q.cursor = b->d_cursor;
        q.n_chunks = uint32_t(sh.qchunks);
        q.chunk = uint32_t(sh.qchunk);
        q.xcds = uint32_t(std::max(1, sh.xcds));
        q.refill = sh.refill;
        return tetrt::launch_trace_batch_queue(b->d_table, sh.n_jobs, q, sh.layout, sh.steps, b->cus, s);
    }
    return tetrt::launch_trace_batch(b->d_table, sh.n_jobs, sh.blocks, sh.block, sh.layout, sh.xcds, sh.steps,
                                     sh.eps, s);
}

int check_batch(const tm_batch_s* b, const char* what) {
    if (!b) return fail(TM_ERR_ARG, "%s: NULL batch", what);
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != b->device)
        return fail(TM_ERR_ARG, "%s: batch on device %d, current device %d", what, b->device, dev);
    return TM_OK;
}

}  // namespace

extern "C" {

int tm_batch_create(int32_t max_jobs, int64_t max_rays, tm_batch* out) {
    tetrt::clear_error();
    if (!out) return fail(TM_ERR_ARG, "tm_batch_create: out is NULL");
    *out = nullptr;
    if (max_jobs < 1 || max_jobs > kMaxJobs)
        return fail(TM_ERR_ARG, "tm_batch_create: max_jobs = %d out of range [1, %d]", max_jobs, kMaxJobs);
    if (max_rays < 0 || max_rays > kMaxRays)
        return fail(TM_ERR_ARG, "tm_batch_create: max_rays = %lld out of range [0, %lld]",
                    (long long)max_rays, (long long)kMaxRays);
    tm_batch_s* b = new (std::nothrow) tm_batch_s();
    if (!b) return fail(TM_ERR_OOM, "tm_batch_create: host allocation failed");
    (void)hipGetDevice(&b->device);
    if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess ||
        b->cus <= 0) {
        (void)hipGetLastError();
        b->cus = 256;
    }
    b->max_jobs = max_jobs;
    b->max_rays = max_rays;
    const size_t table_bytes = size_t(max_jobs) * sizeof(tetrt::Job);
    const size_t perm_bytes = size_t(max_rays + int64_t(max_jobs) * kPermAlign) * sizeof(int32_t);
    hipError_t e;
    if ((e = hipMalloc(&b->d_table, table_bytes)) != hipSuccess ||
        (e = hipMalloc(&b->d_perm, perm_bytes)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&b->d_cursor), size_t(tetrt::kQueueCursorBytes))) != hipSuccess ||
        (e = hipHostMalloc(&b->h_stage, table_bytes, hipHostMallocDefault)) != hipSuccess) {
        (void)hipGetLastError();
        release(b);
        delete b;
        return fail(TM_ERR_OOM, "tm_batch_create: allocation of %zu + %zu bytes failed: %s", table_bytes,
                    perm_bytes, hipGetErrorString(e));
    }
    if ((e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
        release(b);
        delete b;
        return hip_fail(e, "tm_batch_create");
    }
    b->shape.n_jobs = 0;
    *out = b;
    return TM_OK;
}

int tm_batch_set(tm_batch b, int32_t n_jobs, const tm_job* jobs, const tm_trace_opts* opts, void* hip_stream) {
    tetrt::clear_error();
    int rc = check_batch(b, "tm_batch_set");
    if (rc != TM_OK) return rc;
    tm_trace_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    return set_jobs(b, n_jobs, jobs, o, static_cast<hipStream_t>(hip_stream));
}

int tm_batch_launch(tm_batch b, void* hip_stream) {
    tetrt::clear_error();
    int rc = check_batch(b, "tm_batch_launch");
    if (rc != TM_OK) return rc;
    hipError_t e = enqueue(b, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "tm_batch_launch: kernel launch");
    return TM_OK;
}

int tm_batch_graph_launch(tm_batch b, void* hip_stream) {
    tetrt::clear_error();
    int rc = check_batch(b, "tm_batch_graph_launch");
    if (rc != TM_OK) return rc;
    if (b->shape.n_jobs <= 0 || b->shape.blocks <= 0) return TM_OK;
    hipError_t e;
    if (!b->exec || !(b->captured == b->shape)) {
        drop_graph(b);
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "tm_batch_graph_launch: begin capture");
        hipError_t le = enqueue(b, b->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(le, "tm_batch_graph_launch: kernel launch during capture");
        }
        if (e != hipSuccess) return hip_fail(e, "tm_batch_graph_launch: end capture");
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hip_fail(e, "tm_batch_graph_launch: instantiate");
        }
        b->captured = b->shape;
    }
    e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "tm_batch_graph_launch: graph launch");
    return TM_OK;
}

int tm_batch_tune(tm_batch b, int32_t reps, void* hip_stream, tm_trace_opts* chosen, float* ms) {
    tetrt::clear_error();
    int rc = check_batch(b, "tm_batch_tune");
    if (rc != TM_OK) return rc;
    if (reps < 1 || reps > 1000) return fail(TM_ERR_ARG, "tm_batch_tune: reps must be in [1, 1000]");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const std::vector<tm_job> jobs = b->jobs;
    const tm_trace_opts base = b->opts;
    const int32_t n_jobs = int32_t(jobs.size());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "tm_batch_tune: event create");
    }
    static const int32_t kBlocks[3] = {64, 128, 256};
    static const int32_t kChunks[4] = {0, 11, 12, 13};  // 0 = no binning
    static const int32_t kQChunks[3] = {64, 256, 1024};
    static const int32_t kRefills[2] = {16, 64};
    const int32_t xcd_opts[2] = {1, tetrt::xcd_count(b->cus)};
    // candidates: the one-lane-per-ray kernel over block size x binning x placement,
    // then the queue kernel over binning x rays per fetch x refill threshold
    std::vector<tm_trace_opts> cands;
    for (int32_t blk : kBlocks)
        for (int32_t cand = 0; cand < 8; ++cand) {
            const int32_t ch = kChunks[cand % 4];
            tm_trace_opts o = base;
            o.kernel = 1;
            o.block = blk;
            o.sort = ch ? 2 : 1;
            o.sort_chunk_log2 = ch ? ch : base.sort_chunk_log2;
            o.xcds = xcd_opts[cand / 4];
            if (cand >= 4 && o.xcds == 1) continue;   // a device with one XCD
            cands.push_back(o);
        }
    for (int32_t ch : (base.eps > 0.0f ? std::vector<int32_t>{} : std::vector<int32_t>(kChunks, kChunks + 4)))
        for (int32_t qc : kQChunks)
            for (int32_t rf : kRefills) {
                tm_trace_opts o = base;
                o.kernel = 3;
                o.sort = ch ? 2 : 1;
                o.sort_chunk_log2 = ch ? ch : base.sort_chunk_log2;
                o.queue_chunk = qc;
                o.refill = rf;
                o.xcds = 0;
                cands.push_back(o);
            }
    tm_trace_opts best = base;
    float best_ms = -1.0f;
    rc = TM_OK;
    {
        for (const tm_trace_opts& o : cands) {
            if ((rc = set_jobs(b, n_jobs, jobs.data(), o, s)) != TM_OK) break;
            if ((e = enqueue(b, s)) != hipSuccess || (e = hipEventRecord(e0, s)) != hipSuccess) {
                rc = hip_fail(e, "tm_batch_tune: launch");
                break;
            }
            for (int32_t i = 0; i < reps && e == hipSuccess; ++i) e = enqueue(b, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) {
                rc = hip_fail(e, "tm_batch_tune: timed launches");
                break;
            }
            t /= float(reps);
            if (best_ms < 0.0f || t < best_ms) {
                best_ms = t;
                best = o;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TM_OK) {
        (void)set_jobs(b, n_jobs, jobs.data(), base, s);
        return rc;
    }
    rc = set_jobs(b, n_jobs, jobs.data(), best, s);
    if (rc != TM_OK) return rc;
    if (chosen) *chosen = best;
    if (ms) *ms = best_ms;
    return TM_OK;
}

int tm_batch_free(tm_batch b) {
    tetrt::clear_error();
    if (!b) return TM_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != b->device) (void)hipSetDevice(b->device);
    hipError_t e = hipDeviceSynchronize();
    release(b);
    if (prev != b->device) (void)hipSetDevice(prev);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "tm_batch_free: device synchronize");
    return TM_OK;
}

}  // extern "C"
