// C-ABI entry points declared in include/tetrt.h.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "device.h"
#include "handle.h"
#include "pack.h"
#include "tetrt.h"

namespace tetrt {

namespace {
thread_local std::string g_error;
}  // namespace

void clear_error() { g_error.clear(); }

const char* last_error() { return g_error.c_str(); }

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(TM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Binning configuration of a trace; *on = false when the rays are not binned.
int sort_config(const tm_mesh_s* m, const tm_trace_opts& o, int64_t n, bool has_tmax,
                tetrt::SortCfg* c, bool* on) {
    // automatic: bin batches of secondary-style rays (with tmax) of at least 2^18 rays
    *on = o.sort == 2 || (o.sort == 0 && has_tmax && n >= (int64_t(1) << 18));
    c->chunk_log2 = o.sort_chunk_log2 ? o.sort_chunk_log2 : 12;
    c->cells_log2 = o.sort_cells_log2;   // 0: by direction only
    c->dirq = o.sort_dirq ? o.sort_dirq : 4;
    if (c->chunk_log2 < 10 || c->chunk_log2 > 13 || c->cells_log2 < 0 || c->cells_log2 > 7 ||
        c->dirq < 1 || c->dirq > 4)
        return fail(TM_ERR_ARG, "trace_closest: sort_chunk_log2 must be in [10, 13], sort_cells_log2 "
                                "in [0, 7] and sort_dirq in [1, 4]");
    const double G = double(int64_t(1) << c->cells_log2);
    for (int a = 0; a < 3; ++a) {
        c->lo[a] = m->lo[a];
        c->inv[a] = m->ext[a] > 0 ? float(G / m->ext[a]) : 0.0f;
    }
    return TM_OK;
}

}  // namespace tetrt

namespace {

using tetrt::fail;
using tetrt::hip_fail;
using tetrt::sort_config;

// Kernels of a mesh run on the device it was uploaded to: that device must be
// current (its pointers mean nothing on another).
int check_device(const tm_mesh_s* m, const char* what) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != m->device)
        return fail(TM_ERR_ARG, "%s: mesh on device %d, current device %d", what, m->device, dev);
    return TM_OK;
}

void release(tm_mesh_s* m) {
    for (void* p : m->allocations) (void)hipFree(p);
    m->allocations.clear();
    if (m->ws_done) (void)hipEventDestroy(m->ws_done);
    m->ws_done = nullptr;
    m->ws = nullptr;
    m->ws_bytes = 0;
}

// Copy a host vector into a new device buffer owned by the handle.
template <class T>
int upload_array(tm_mesh_s* m, const std::vector<T>& v, const T** out, int64_t* bytes_acc) {
    size_t bytes = v.size() * sizeof(T);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(TM_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    m->allocations.push_back(p);
    if (bytes > 0) {
        e = hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    *out = static_cast<const T*>(p);
    *bytes_acc += int64_t(bytes);
    return TM_OK;
}

}  // namespace

namespace tetrt {

int trace_impl(tm_mesh_s* m, int64_t n_rays, const float* d_orig, const float* d_dir,
               const float* d_tmax, const int32_t* d_start_tet, const int32_t* d_start_face,
               int32_t* d_tri, float* d_t, float* d_bary, int32_t* d_hit_tets, int32_t* d_steps,
               const tm_trace_opts* opts, void* hip_stream, void* fixed_ws, int64_t fixed_ws_bytes,
               const char* name) {
    if (!m) return fail(TM_ERR_ARG, "%s: NULL mesh", name);
    if (int rc = check_device(m, name)) return rc;
    if (n_rays < 0 || n_rays > int64_t(0x7FFFFFFF))
        return fail(TM_ERR_ARG, "%s: n_rays = %lld out of range [0, 2^31)", name, (long long)n_rays);
    if (n_rays == 0) return TM_OK;
    if (!d_orig || !d_dir || !d_tri || !d_t || !d_bary)
        return fail(TM_ERR_ARG, "%s: NULL required array", name);
    if ((reinterpret_cast<uintptr_t>(d_bary) & 7) || (reinterpret_cast<uintptr_t>(d_hit_tets) & 7))
        return fail(TM_ERR_ARG, "%s: bary / hit_tets must be 8-byte aligned", name);
    tm_trace_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.max_steps < 0) return fail(TM_ERR_ARG, "%s: negative max_steps", name);
    if (o.block != 0 && o.block != 64 && o.block != 128 && o.block != 256)
        return fail(TM_ERR_ARG, "%s: block must be 64, 128 or 256", name);
    if (o.kernel < 0 || o.kernel > 3) return fail(TM_ERR_ARG, "%s: kernel must be 0, 1, 2 or 3", name);
    if (o.queue_chunk < 0 || o.queue_chunk > 4096 || (o.queue_chunk & 63))
        return fail(TM_ERR_ARG, "%s: queue_chunk must be a multiple of 64 in [64, 4096]", name);
    if (o.refill < 0 || o.refill > 64) return fail(TM_ERR_ARG, "%s: refill must be in [0, 64]", name);
    if (o.grid_cap < 0) return fail(TM_ERR_ARG, "%s: negative grid_cap", name);
    if (o.xcds < 0 || o.xcds > 64) return fail(TM_ERR_ARG, "%s: xcds must be in [0, 64]", name);
    if (o.xcd_blocks < 0 || o.xcd_blocks > 65536)
        return fail(TM_ERR_ARG, "%s: xcd_blocks must be in [0, 65536]", name);
    if (o.sort < 0 || o.sort > 2) return fail(TM_ERR_ARG, "%s: sort must be 0, 1 or 2", name);
    if (!(o.eps >= 0.0f) || !(o.eps < 1.0f)) return fail(TM_ERR_ARG, "%s: eps must be in [0, 1)", name);
    if (o.eps > 0.0f && o.kernel >= 2)
        return fail(TM_ERR_ARG, "%s: the precision variant (eps > 0) runs one lane per ray", name);
    if (o.workspace_bytes < 0 || (o.workspace_bytes > 0 && !o.workspace))
        return fail(TM_ERR_ARG, "%s: bad workspace", name);
    if (fixed_ws && o.workspace)
        return fail(TM_ERR_ARG, "%s: takes no workspace (it bins through its own)", name);
    SortCfg sc;
    bool binned = false;
    int rc = sort_config(m, o, n_rays, d_tmax != nullptr, &sc, &binned);
    if (rc != TM_OK) return rc;
    if (o.order) binned = false;   // the caller's order replaces the call's binning
    const bool queue = o.kernel == 3;
    // workspace: the binning permutation, then (kernel 3) the queue's counters and
    // its one-entry job table
    int64_t perm_bytes = binned ? sort_workspace_bytes(n_rays) : 0;
    const int64_t queue_bytes = queue ? queue_workspace_bytes() : 0;
    // the precision variant's two-pass form: a counter and a list of deferred rays
    // (without room for them it runs in one pass, with the same results)
    if (o.passes < 0 || o.passes > 2) return fail(TM_ERR_ARG, "%s: passes must be 0, 1 or 2", name);
    int64_t defer_bytes = (o.eps > 0.0f && o.passes == 2) ? 256 + sort_workspace_bytes(n_rays) : 0;
    // the one-pass precision variant's tie list (without room for it each wave
    // resolves its own ties, with the same results)
    int64_t tie_bytes = (o.eps > 0.0f && o.passes != 2 && o.kernel < 2) ? tie_workspace_bytes() : 0;
    // where it goes: the given fixed workspace, the caller's, or the handle's own;
    // with none of them large enough an explicit sort = 2 or kernel = 3 is an
    // error and the automatic choice traces the rays unbinned
    void* ws = nullptr;
    bool handle_ws = false;
    while (perm_bytes + queue_bytes + defer_bytes + tie_bytes > 0) {
        const int64_t need = perm_bytes + queue_bytes + defer_bytes + tie_bytes;
        const int64_t avail = fixed_ws ? fixed_ws_bytes : (o.workspace ? o.workspace_bytes : m->ws_bytes);
        if (avail < need && defer_bytes > 0) {
            defer_bytes = 0;
            continue;
        }
        if (avail < need && tie_bytes > 0) {
            tie_bytes = 0;
            continue;
        }
        if (fixed_ws) {
            if (perm_bytes > fixed_ws_bytes - kFixedExtraBytes || fixed_ws_bytes < need)
                return fail(TM_ERR_ARG, "%s: %lld rays to bin, at most %lld", name, (long long)n_rays,
                            (long long)((fixed_ws_bytes - kFixedExtraBytes) / 4));
            ws = fixed_ws;
        } else if (o.workspace) {
            if (o.workspace_bytes < need)
                return fail(TM_ERR_ARG, "%s: workspace of %lld bytes, %lld needed", name,
                            (long long)o.workspace_bytes, (long long)need);
            ws = o.workspace;
        } else if (m->ws_bytes >= need) {
            ws = m->ws;
            handle_ws = true;
        } else if (o.sort == 2 || queue) {
            return fail(TM_ERR_ARG, "%s: %s needs a workspace of %lld bytes (opts.workspace, or "
                        "tm_upload_opts.bin_rays >= n_rays)", name, queue ? "the queue kernel" : "binning",
                        (long long)need);
        } else {
            binned = false;
            perm_bytes = 0;
            continue;
        }
        break;
    }
    RayArgs r;
    r.perm = o.order;
    r.orig = d_orig;
    r.dir = d_dir;
    r.tmax = d_tmax;
    r.start_tet = d_start_tet;
    r.start_face = d_start_face;
    r.tri = d_tri;
    r.t = d_t;
    r.bary = d_bary;
    r.hit_tets = d_hit_tets;
    r.steps = d_steps;
    r.fp64_steps = o.fp64_steps;
    r.n = n_rays;
    r.max_steps = o.max_steps > 0 ? o.max_steps : 65536;
    LaunchCfg c;
    // automatic: 256-thread blocks for binned (or caller-ordered) rays, 128 for
    // the rest, whose walks differ more in length from lane to lane; smaller
    // blocks retire sooner and even out the XCDs' loads (camera rays: 0.834 vs
    // 0.853 ms; binned AO rays: 1.396 vs 1.340 ms)
    c.block = o.block ? o.block : ((binned || o.order) ? 256 : 128);
    c.cus = m->cus;
    c.waves_per_simd = 8;
    // persistent lanes refill at 16 finished lanes; the queue kernel's waves only once
    // all their lanes are done (refilling idle lanes earlier cost more than it saved:
    // main workload, primary 1.64 against 1.11 ms, AO 5.71 against 2.29 ms)
    c.refill = o.refill ? o.refill : (o.kernel == 3 ? 64 : 16);
    c.grid_cap = o.grid_cap;
    // automatic: binned launches (their rays are ordered along the image, then by
    // direction inside each chunk) give each XCD one contiguous range of blocks, so
    // an XCD's L2 holds the tets of its part of the scene; unbinned launches keep
    // the dispatcher's round-robin placement, which balances walks of uneven length
    c.xcds = o.xcds ? o.xcds : ((binned || o.order) ? xcd_count(m->cus) : 1);
    c.xcd_blocks = o.xcd_blocks;
    // automatic: one lane per ray (the persistent-lane kernel is slower on every
    // measured workload and runs only when asked for)
    c.kernel = o.kernel ? o.kernel : 1;
    c.eps = o.eps;
    if (queue) {
        char* base = static_cast<char*>(ws) + perm_bytes;
        c.queue.cursor = reinterpret_cast<uint32_t*>(base);
        // 64 rays per fetch (one per lane) balances the waves' loads best (main
        // workload, refill 64: primary 1.11 against 2.00 ms with 256, AO 2.29 against 2.86)
        c.queue.chunk = uint32_t(o.queue_chunk ? o.queue_chunk : 64);
        c.queue.n_chunks = uint32_t((n_rays + c.queue.chunk - 1) / c.queue.chunk);
        c.queue.xcds = uint32_t(o.xcds ? o.xcds : xcd_count(m->cus));
        c.queue.refill = c.refill;
        c.queue_job = reinterpret_cast<Job*>(base + kQueueCursorBytes);
    }
    c.defer_count = nullptr;
    c.defer_list = nullptr;
    if (defer_bytes > 0) {
        char* base = static_cast<char*>(ws) + perm_bytes + queue_bytes;
        c.defer_count = reinterpret_cast<uint32_t*>(base);
        c.defer_list = reinterpret_cast<int32_t*>(base + 256);
    }
    c.ties = TieList{};
    if (tie_bytes > 0) c.ties = tie_list_at(static_cast<char*>(ws) + perm_bytes + queue_bytes + defer_bytes);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e;
    std::unique_lock<std::mutex> lock(m->ws_mu, std::defer_lock);
    if (handle_ws) {
        // the previous trace through the handle's workspace (permutation, queue
        // counters, lists) may still be using it on another stream: this stream
        // waits for it (stream order covers the same stream)
        lock.lock();
        if (m->ws_used && m->ws_stream != stream) {
            e = hipStreamWaitEvent(stream, m->ws_done, 0);
            if (e != hipSuccess) return hip_fail(e, name);
        }
    }
    if (binned) {
        int32_t* perm = nullptr;
        e = launch_sort(sc, d_orig, d_dir, n_rays, ws, &perm, stream);
        if (e != hipSuccess) return hip_fail(e, "ray binning launch");
        r.perm = perm;
    }
    e = launch_trace(m->dev, r, c, stream);
    if (e != hipSuccess) return hip_fail(e, "trace kernel launch");
    if (handle_ws) {
        e = hipEventRecord(m->ws_done, stream);
        if (e != hipSuccess) return hip_fail(e, name);
        m->ws_stream = stream;
        m->ws_used = true;
    }
    return TM_OK;
}

}  // namespace tetrt

extern "C" {

const char* tm_last_error(void) { return tetrt::last_error(); }

int tetmesh_upload(const float* points, int64_t n_points, const int32_t* tets, const int32_t* nbrs,
                   const uint8_t* cflag, int64_t n_tets, const tm_upload_opts* opts, tm_mesh* out) {
    tetrt::clear_error();
    if (!out) return fail(TM_ERR_ARG, "tetmesh_upload: out is NULL");
    *out = nullptr;
    if (!points || !tets || !nbrs || !cflag)
        return fail(TM_ERR_ARG, "tetmesh_upload: NULL input array");
    if (n_tets < 1 || n_tets >= int64_t(0x7FFFFFFF))
        return fail(TM_ERR_ARG, "tetmesh_upload: n_tets = %lld out of range [1, 2^31-1)",
                    (long long)n_tets);
    if (n_points < 4 || n_points >= int64_t(0x80000000LL))
        return fail(TM_ERR_ARG, "tetmesh_upload: n_points = %lld out of range [4, 2^31)",
                    (long long)n_points);
    // records and points below 4 GiB each: the sizes the packer's index arithmetic
    // is written for
    {
        const int64_t rb = (opts && (opts->layout == TM_LAYOUT_TET32N || opts->layout == TM_LAYOUT_TET32)) ? 32 : 20;
        if (n_tets * rb > int64_t(0xFFFFFFFFLL) || n_points * 12 > int64_t(0xFFFFFFFFLL))
            return fail(TM_ERR_ARG, "tetmesh_upload: mesh too large (at most %lld tets and %lld points)",
                        (long long)(0xFFFFFFFFLL / rb), (long long)(0xFFFFFFFFLL / 12));
    }
    tm_upload_opts o = {TM_LAYOUT_TET20, TM_SFC_HILBERT, 1, 0, 0};
    if (opts) o = *opts;
    if (o.bin_rays < 0 || o.bin_rays > int64_t(0x7FFFFFFF))
        return fail(TM_ERR_ARG, "tetmesh_upload: bin_rays = %lld out of range [0, 2^31)",
                    (long long)o.bin_rays);
    if (o.layout != TM_LAYOUT_TET20 && o.layout != TM_LAYOUT_TET16 && o.layout != TM_LAYOUT_TET32N &&
        o.layout != TM_LAYOUT_TET32)
        return fail(TM_ERR_ARG, "tetmesh_upload: unsupported layout %d", o.layout);
    if (o.sfc < TM_SFC_HILBERT || o.sfc > TM_SFC_HILBERT_REGIONS)
        return fail(TM_ERR_ARG, "tetmesh_upload: unknown sfc %d", o.sfc);
    if (o.seed_grid < 0 || o.seed_grid > 256)
        return fail(TM_ERR_ARG, "tetmesh_upload: seed_grid %d out of range [0, 256]", o.seed_grid);

    tetrt::PackedMesh pm;
    std::string err;
    int rc;
    try {
        rc = tetrt::pack_mesh(points, n_points, tets, nbrs, cflag, n_tets, o, &pm, &err);
    } catch (const std::bad_alloc&) {
        return fail(TM_ERR_OOM, "tetmesh_upload: host allocation failed while packing");
    }
    if (rc != TM_OK) return fail(rc, "tetmesh_upload: %s", err.c_str());

    tm_mesh_s* m = new (std::nothrow) tm_mesh_s();
    if (!m) return fail(TM_ERR_OOM, "tetmesh_upload: host allocation failed");
    (void)hipGetDevice(&m->device);
    if (hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess ||
        m->cus <= 0) {
        (void)hipGetLastError();
        m->cus = 256;
    }
    m->np = pm.np;
    m->nt = pm.nt;
    m->ntri = pm.ntri;
    m->layout = pm.layout;
    m->sfc = pm.sfc;
    m->n_regions = pm.n_regions;
    int64_t hot = 0, cold = 0;
    tetrt::DevMesh& d = m->dev;
    if ((rc = upload_array(m, pm.rec, &d.rec, &hot)) ||
        (!pm.n3.empty() && (rc = upload_array(m, pm.n3, &d.n3, &cold))) ||
        (rc = upload_array(m, pm.pts, &d.pts, &hot)) ||
        (rc = upload_array(m, pm.tetv, &d.tetv, &cold)) ||
        (rc = upload_array(m, pm.cfv, &d.cfv, &cold)) ||
        (rc = upload_array(m, pm.cft, &d.cft, &cold)) ||
        (rc = upload_array(m, pm.t_new2old, &d.t_new2old, &cold)) ||
        (rc = upload_array(m, pm.t_old2new, &d.t_old2new, &cold)) ||
        (rc = upload_array(m, pm.seed, &d.seed, &cold))) {
        release(m);
        delete m;
        return rc;
    }
    if (o.bin_rays > 0) {
        // the handle's binning workspace, allocated once here (traces never allocate)
        // room for binning, the queue kernel and the precision variant's two passes
        const int64_t need = 2 * tetrt::sort_workspace_bytes(o.bin_rays) + 256 + tetrt::queue_workspace_bytes() +
                             tetrt::tie_workspace_bytes();
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, size_t(need));
        if (e == hipSuccess) {
            m->allocations.push_back(p);
            e = hipEventCreateWithFlags(&m->ws_done, hipEventDisableTiming);
        } else {
            (void)hipGetLastError();
        }
        if (e != hipSuccess) {
            release(m);
            delete m;
            return fail(e == hipErrorOutOfMemory ? TM_ERR_OOM : TM_ERR_HIP,
                        "tetmesh_upload: binning workspace of %lld bytes: %s", (long long)need,
                        hipGetErrorString(e));
        }
        m->ws = p;
        m->ws_bytes = need;
        cold += need;
    }
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = pm.lo[a];
        d.inv_cell[a] = pm.inv_cell[a];
    }
    d.G = pm.G;
    d.nt = int32_t(pm.nt);
    d.np = int32_t(pm.np);
    d.ntri = int32_t(pm.ntri);
    d.layout = pm.layout;
    m->hot_bytes = hot;
    m->cold_bytes = cold;
    m->tri_verts_user.swap(pm.tri_verts_user);
    for (int a = 0; a < 3; ++a) {
        float lo = points[a], hi = points[a];
        for (int64_t i = 1; i < n_points; ++i) {
            lo = std::fmin(lo, points[3 * i + a]);
            hi = std::fmax(hi, points[3 * i + a]);
        }
        m->lo[a] = lo;
        m->ext[a] = hi - lo;
    }
    *out = m;
    return TM_OK;
}

int trace_closest(tm_mesh m, int64_t n_rays, const float* d_orig, const float* d_dir,
                  const float* d_tmax, const int32_t* d_start_tet, const int32_t* d_start_face,
                  int32_t* d_tri, float* d_t, float* d_bary, int32_t* d_hit_tets, int32_t* d_steps,
                  const tm_trace_opts* opts, void* hip_stream) {
    tetrt::clear_error();
    return tetrt::trace_impl(m, n_rays, d_orig, d_dir, d_tmax, d_start_tet, d_start_face, d_tri, d_t,
                             d_bary, d_hit_tets, d_steps, opts, hip_stream, nullptr, 0, "trace_closest");
}

int tetmesh_bin_rays(tm_mesh m, int64_t n_rays, const float* d_orig, const float* d_dir,
                     const tm_trace_opts* opts, int32_t* d_order, void* hip_stream) {
    tetrt::clear_error();
    if (!m) return fail(TM_ERR_ARG, "tetmesh_bin_rays: NULL mesh");
    if (int rc = check_device(m, "tetmesh_bin_rays")) return rc;
    if (n_rays < 0 || n_rays > int64_t(0x7FFFFFFF))
        return fail(TM_ERR_ARG, "tetmesh_bin_rays: n_rays = %lld out of range [0, 2^31)", (long long)n_rays);
    if (n_rays == 0) return TM_OK;
    if (!d_orig || !d_dir || !d_order) return fail(TM_ERR_ARG, "tetmesh_bin_rays: NULL array");
    tm_trace_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    o.sort = 2;
    tetrt::SortCfg sc;
    bool on = false;
    int rc = sort_config(m, o, n_rays, true, &sc, &on);
    if (rc != TM_OK) return rc;
    int32_t* perm = nullptr;
    hipError_t e = tetrt::launch_sort(sc, d_orig, d_dir, n_rays, d_order, &perm,
                                      static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "tetmesh_bin_rays: kernel launch");
    return TM_OK;
}

int tetmesh_trace_workspace(tm_mesh m, int64_t n_rays, const float* d_tmax_present,
                            const tm_trace_opts* opts, int64_t* bytes) {
    tetrt::clear_error();
    if (!m || !bytes) return fail(TM_ERR_ARG, "tetmesh_trace_workspace: NULL argument");
    if (n_rays < 0 || n_rays > int64_t(0x7FFFFFFF))
        return fail(TM_ERR_ARG, "tetmesh_trace_workspace: n_rays out of range");
    tm_trace_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    tetrt::SortCfg sc;
    bool binned = false;
    int rc = sort_config(m, o, n_rays, d_tmax_present != nullptr, &sc, &binned);
    if (rc != TM_OK) return rc;
    if (o.order) binned = false;
    *bytes = (binned ? tetrt::sort_workspace_bytes(n_rays) : 0) + (o.kernel == 3 ? tetrt::queue_workspace_bytes() : 0) +
             ((o.eps > 0.0f && o.passes == 2) ? 256 + tetrt::sort_workspace_bytes(n_rays) : 0) +
             ((o.eps > 0.0f && o.passes != 2 && o.kernel < 2) ? tetrt::tie_workspace_bytes() : 0);
    return TM_OK;
}

int tetmesh_locate(tm_mesh m, int64_t n, const float* d_pts, int32_t* d_tet, void* hip_stream) {
    tetrt::clear_error();
    if (!m) return fail(TM_ERR_ARG, "tetmesh_locate: NULL mesh");
    if (int rc = check_device(m, "tetmesh_locate")) return rc;
    if (n < 0 || n > int64_t(0x7FFFFFFF))
        return fail(TM_ERR_ARG, "tetmesh_locate: n = %lld out of range [0, 2^31)", (long long)n);
    if (n == 0) return TM_OK;
    if (!d_pts || !d_tet) return fail(TM_ERR_ARG, "tetmesh_locate: NULL array");
    hipError_t e = tetrt::launch_locate(m->dev, n, d_pts, d_tet, 65536,
                                        static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "tetmesh_locate: kernel launch");
    return TM_OK;
}

int tetmesh_tri_vertices(tm_mesh m, int64_t n, const int32_t* tri, int32_t* out) {
    tetrt::clear_error();
    if (!m) return fail(TM_ERR_ARG, "tetmesh_tri_vertices: NULL mesh");
    if (n < 0) return fail(TM_ERR_ARG, "tetmesh_tri_vertices: negative n");
    if (n > 0 && (!tri || !out)) return fail(TM_ERR_ARG, "tetmesh_tri_vertices: NULL array");
    for (int64_t i = 0; i < n; ++i) {
        if (tri[i] < 0 || tri[i] >= m->ntri)
            return fail(TM_ERR_ARG, "tetmesh_tri_vertices: triangle id %d out of range", tri[i]);
        std::memcpy(out + 3 * i, &m->tri_verts_user[3 * (size_t)tri[i]], 3 * sizeof(int32_t));
    }
    return TM_OK;
}

int tetmesh_info(tm_mesh m, tm_info* out) {
    tetrt::clear_error();
    if (!m || !out) return fail(TM_ERR_ARG, "tetmesh_info: NULL argument");
    out->n_tets = m->nt;
    out->n_points = m->np;
    out->n_tris = m->ntri;
    out->hot_bytes = m->hot_bytes;
    out->cold_bytes = m->cold_bytes;
    out->layout = m->layout;
    out->sfc = m->sfc;
    out->seed_grid = m->dev.G;
    out->n_regions = int32_t(m->n_regions);
    return TM_OK;
}

int tetmesh_free(tm_mesh m) {
    tetrt::clear_error();
    if (!m) return TM_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != m->device) (void)hipSetDevice(m->device);
    hipError_t e = hipDeviceSynchronize();
    release(m);
    if (prev != m->device) (void)hipSetDevice(prev);
    delete m;
    if (e != hipSuccess) return hip_fail(e, "tetmesh_free: device synchronize");
    return TM_OK;
}

int tetrt_sfc_keys(int32_t curve, int32_t bits, int64_t n, const uint32_t* xyz, uint64_t* out) {
    tetrt::clear_error();
    if (bits < 1 || bits > 21) return fail(TM_ERR_ARG, "tetrt_sfc_keys: bits must be in [1, 21]");
    if (curve != TM_SFC_HILBERT && curve != TM_SFC_MORTON)
        return fail(TM_ERR_ARG, "tetrt_sfc_keys: unknown curve %d", curve);
    if (n < 0 || (n > 0 && (!xyz || !out))) return fail(TM_ERR_ARG, "tetrt_sfc_keys: bad arrays");
    const uint32_t lim = 1u << bits;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t* c = xyz + 3 * i;
        if (c[0] >= lim || c[1] >= lim || c[2] >= lim)
            return fail(TM_ERR_ARG, "tetrt_sfc_keys: coordinate of point %lld >= 2^bits", (long long)i);
        out[i] = curve == TM_SFC_HILBERT ? tetrt::hilbert_key(c[0], c[1], c[2], bits)
                                         : tetrt::morton_key(c[0], c[1], c[2], bits);
    }
    return TM_OK;
}

}  // extern "C"
