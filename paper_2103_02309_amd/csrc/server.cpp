// C-ABI of the serving loop (tm_server_*, declared in include/tetrt.h).
//
// Host-side scheduler: FIFO admission of requests into a ray pool (first-fit
// ranges of slots), then per step one generation launch and one batched trace
// over the pending phase of every admitted request.  Launches go round a ring
// of slots, each with its own batch object, generation table and completion
// event, so building a step never waits for an earlier one to finish.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "device.h"
#include "handle.h"
#include "tetrt.h"

namespace {

using tetrt::fail;
using tetrt::hip_fail;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum class St { Queued, Pending0, Flight0, Pending1, Flight1 };

struct Req {
    tm_request r;
    int64_t id = 0, submit_ns = 0, admit_ns = 0;
    int64_t base = -1, n = 0;
    St st = St::Queued;
    tetrt::GenEntry gen{};  // camera basis, filled at submit
};

// One in-flight launch.
struct Slot {
    tm_batch batch = nullptr;
    tetrt::GenEntry* d_gen = nullptr;
    tetrt::GenEntry* h_gen = nullptr;   // pinned
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<std::pair<int64_t, bool>> items;  // request id, final phase
};

// First-fit allocator over [0, cap) pool slots.
struct Ranges {
    std::map<int64_t, int64_t> free_;  // begin -> end
    void reset(int64_t cap) {
        free_.clear();
        if (cap > 0) free_[0] = cap;
    }
    int64_t take(int64_t n) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second - it->first >= n) {
                const int64_t b = it->first, e = it->second;
                free_.erase(it);
                if (b + n < e) free_[b + n] = e;
                return b;
            }
        }
        return -1;
    }
    void give(int64_t b, int64_t n) {
        int64_t e = b + n;
        auto next = free_.lower_bound(b);
        if (next != free_.end() && next->first == e) {
            e = next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->second == b) {
                prev->second = e;
                return;
            }
        }
        free_[b] = e;
    }
};

}  // namespace

struct tm_server_s {
    int device = 0;
    std::vector<tm_mesh> meshes;
    tm_server_opts o{};
    tetrt::RayPool pool{};
    std::vector<void*> allocations;
    Ranges ranges;
    std::vector<Slot> ring;
    int next_slot = 0;                 // the slot the next launch uses
    std::deque<int> order;             // busy slots, oldest first
    std::deque<int64_t> queue;         // queued request ids, FIFO
    std::unordered_map<int64_t, Req> reqs;
    std::deque<tm_done> finished;
    int64_t next_id = 1, admitted = 0;
};

namespace {

void release(tm_server_s* s) {
    for (Slot& sl : s->ring) {
        if (sl.batch) (void)tm_batch_free(sl.batch);
        if (sl.d_gen) (void)hipFree(sl.d_gen);
        if (sl.h_gen) (void)hipHostFree(sl.h_gen);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    s->ring.clear();
    for (void* p : s->allocations) (void)hipFree(p);
    s->allocations.clear();
}

template <class T>
int alloc(tm_server_s* s, T** p, int64_t count) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), size_t(count) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(TM_ERR_OOM, "tm_server_create: device allocation of %lld bytes failed: %s",
                    (long long)(count * int64_t(sizeof(T))), hipGetErrorString(e));
    }
    s->allocations.push_back(*p);
    return TM_OK;
}

// Move finished launches' requests on: the next phase, or done.  Returns the
// first device error seen (hipSuccess while launches are merely running).
hipError_t retire(tm_server_s* s, bool wait) {
    while (!s->order.empty()) {
        Slot& sl = s->ring[size_t(s->order.front())];
        hipError_t e = wait ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
        if (e == hipErrorNotReady) return hipSuccess;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        const int64_t t = now_ns();
        for (const auto& it : sl.items) {
            auto r = s->reqs.find(it.first);
            if (r == s->reqs.end()) continue;
            Req& q = r->second;
            if (it.second) {
                tm_done d;
                d.id = q.id;
                d.submit_ns = q.submit_ns;
                d.admit_ns = q.admit_ns;
                d.done_ns = t;
                d.rays = q.n * (q.r.kind == TM_REQ_PRIMARY ? 1 : 2);
                s->finished.push_back(d);
                s->ranges.give(q.base, q.n);
                s->admitted -= 1;
                s->reqs.erase(r);
            } else {
                q.st = St::Pending1;
            }
        }
        sl.items.clear();
        sl.busy = false;
        s->order.pop_front();
        wait = false;  // waited for the oldest; the rest only if already complete
    }
    return hipSuccess;
}

int step(tm_server_s* s, hipStream_t stream, int64_t* launched) {
    if (launched) *launched = 0;
    hipError_t e = retire(s, false);
    if (e != hipSuccess) return hip_fail(e, "tm_server_step: an earlier launch failed");
    Slot& sl = s->ring[size_t(s->next_slot)];
    if (sl.busy) return TM_OK;  // ring full
    // admission, first come first served
    while (!s->queue.empty() && s->admitted < s->o.max_requests) {
        Req& q = s->reqs[s->queue.front()];
        const int64_t b = s->ranges.take(q.n);
        if (b < 0) break;
        q.base = b;
        q.admit_ns = now_ns();
        q.st = St::Pending0;
        s->admitted += 1;
        s->queue.pop_front();
    }
    // the pending phase of every admitted request
    std::vector<tetrt::GenEntry> gen;
    std::vector<tm_job> jobs;
    sl.items.clear();
    int64_t blocks = 0, rays = 0;
    for (auto& kv : s->reqs) {
        Req& q = kv.second;
        if (q.st != St::Pending0 && q.st != St::Pending1) continue;
        const bool two = q.r.kind != TM_REQ_PRIMARY;
        const bool final_phase = q.st == St::Pending1 || !two;
        tetrt::GenEntry g = q.gen;
        g.kind = q.st == St::Pending0 ? tetrt::kGenCamera
                                      : (q.r.kind == TM_REQ_SHADOW ? tetrt::kGenShadow : tetrt::kGenAO);
        g.base = q.base;
        g.block0 = blocks;
        blocks += (q.n + tetrt::kGenBlock - 1) / tetrt::kGenBlock;
        gen.push_back(g);
        tm_job j;
        std::memset(&j, 0, sizeof j);
        j.mesh = s->meshes[size_t(q.r.mesh)];
        j.n_rays = q.n;
        j.d_orig = s->pool.orig + 3 * q.base;
        j.d_dir = s->pool.dir + 3 * q.base;
        // camera rays carry no tmax (so the automatic rule leaves them unbinned, as
        // primary rays gain nothing from binning); secondary rays do
        j.d_tmax = q.st == St::Pending0 ? nullptr : s->pool.tmax + q.base;
        j.d_start_face = s->pool.sf + q.base;
        if (final_phase) {
            j.d_tri = q.r.d_tri;
            j.d_t = q.r.d_t;
            j.d_bary = q.r.d_bary;
        } else {
            j.d_tri = s->pool.tri + q.base;
            j.d_t = s->pool.t + q.base;
            j.d_bary = s->pool.bary + 2 * q.base;
        }
        jobs.push_back(j);
        sl.items.emplace_back(q.id, final_phase);
        q.st = q.st == St::Pending0 ? St::Flight0 : St::Flight1;
        rays += q.n;
    }
    if (jobs.empty()) return TM_OK;
    // on a failed launch the step's requests go back to pending, to be launched
    // again by a later step
    auto undo = [&](int rc) {
        for (const auto& it : sl.items) {
            auto r = s->reqs.find(it.first);
            if (r != s->reqs.end()) r->second.st = r->second.st == St::Flight0 ? St::Pending0 : St::Pending1;
        }
        sl.items.clear();
        return rc;
    };
    std::memcpy(sl.h_gen, gen.data(), gen.size() * sizeof(tetrt::GenEntry));
    e = hipMemcpyAsync(sl.d_gen, sl.h_gen, gen.size() * sizeof(tetrt::GenEntry), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = tetrt::launch_gen(sl.d_gen, int32_t(gen.size()), blocks, s->pool, stream);
    if (e != hipSuccess) return undo(hip_fail(e, "tm_server_step: ray generation"));
    tm_trace_opts to;
    std::memset(&to, 0, sizeof to);
    to.block = s->o.block;
    to.sort = s->o.sort;
    to.max_steps = s->o.max_steps;
    to.eps = s->o.eps;
    int rc = tm_batch_set(sl.batch, int32_t(jobs.size()), jobs.data(), &to, stream);
    if (rc == TM_OK) rc = tm_batch_launch(sl.batch, stream);
    if (rc != TM_OK) return undo(rc);
    e = hipEventRecord(sl.done, stream);
    if (e != hipSuccess) return undo(hip_fail(e, "tm_server_step: event record"));
    sl.busy = true;
    s->order.push_back(s->next_slot);
    s->next_slot = (s->next_slot + 1) % int(s->ring.size());
    if (launched) *launched = rays;
    return TM_OK;
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Validate a request's image, camera and outputs and fill its generation entry
// (kind, base and block0 are the caller's).  what names the calling entry point.
int make_entry(const tm_request& r, const tm_mesh_s* m, const char* what, bool outputs,
               tetrt::GenEntry* out) {
    if (r.kind < TM_REQ_PRIMARY || r.kind > TM_REQ_AO) return fail(TM_ERR_ARG, "%s: unknown kind %d", what, r.kind);
    if (r.width < 8 || r.height < 8 || r.width > 8192 || r.height > 8192 || (r.width & 7) || (r.height & 7))
        return fail(TM_ERR_ARG, "%s: image size must be multiples of 8 in [8, 8192]", what);
    if (!(r.fov_h_deg > 0.0f && r.fov_h_deg <= 179.0f))
        return fail(TM_ERR_ARG, "%s: fov_h_deg must be in (0, 179]", what);
    if (!finite3(r.eye) || !finite3(r.forward) || !finite3(r.up) ||
        (r.kind == TM_REQ_SHADOW && !finite3(r.light)))
        return fail(TM_ERR_ARG, "%s: non-finite camera or light", what);
    if (r.kind == TM_REQ_AO && !(r.ao_tmax > 0.0f)) return fail(TM_ERR_ARG, "%s: ao_tmax must be > 0", what);
    if (outputs && (!r.d_tri || !r.d_t || !r.d_bary || (reinterpret_cast<uintptr_t>(r.d_bary) & 7)))
        return fail(TM_ERR_ARG, "%s: NULL or misaligned output", what);
    // camera basis in double: unit forward, right and up scaled to the image plane at distance 1
    double f[3] = {r.forward[0], r.forward[1], r.forward[2]};
    const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0)) return fail(TM_ERR_ARG, "%s: zero forward", what);
    for (double& v : f) v /= fl;
    double rt[3] = {f[1] * r.up[2] - f[2] * r.up[1], f[2] * r.up[0] - f[0] * r.up[2], f[0] * r.up[1] - f[1] * r.up[0]};
    const double rl = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    const double ul = std::sqrt(double(r.up[0]) * r.up[0] + double(r.up[1]) * r.up[1] + double(r.up[2]) * r.up[2]);
    if (!(rl > 1e-6 * ul)) return fail(TM_ERR_ARG, "%s: up is parallel to forward", what);
    for (double& v : rt) v /= rl;
    const double u[3] = {rt[1] * f[2] - rt[2] * f[1], rt[2] * f[0] - rt[0] * f[2], rt[0] * f[1] - rt[1] * f[0]};
    const double th = std::tan(double(r.fov_h_deg) * 3.14159265358979323846 / 360.0);
    const double tv = th * double(r.height) / double(r.width);
    tetrt::GenEntry g{};
    g.W = r.width;
    g.H = r.height;
    g.seed = r.seed;
    for (int a = 0; a < 3; ++a) {
        g.eye[a] = r.eye[a];
        g.fwd[a] = float(f[a]);
        g.right[a] = float(rt[a] * th);
        g.up[a] = float(u[a] * tv);
        g.light[a] = r.light[a];
    }
    g.ao_tmax = r.ao_tmax;
    g.pts = m->dev.pts;
    g.cfv = m->dev.cfv;
    *out = g;
    return TM_OK;
}

}  // namespace

extern "C" {

int tm_server_create(const tm_mesh* meshes, int32_t n_meshes, const tm_server_opts* opts, tm_server* out) {
    tetrt::clear_error();
    if (!out) return fail(TM_ERR_ARG, "tm_server_create: out is NULL");
    *out = nullptr;
    if (!meshes || n_meshes < 1 || n_meshes > 65536)
        return fail(TM_ERR_ARG, "tm_server_create: need 1..65536 meshes");
    tm_server_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.max_rays < 1 || o.max_rays > int64_t(0x7FFFFFFF))
        return fail(TM_ERR_ARG, "tm_server_create: max_rays = %lld out of range [1, 2^31)",
                    (long long)o.max_rays);
    if (o.max_requests == 0) o.max_requests = 4096;
    // one launch in flight: each step then carries every request that arrived
    // during the previous launch (lowest latency measured at up to 75% load)
    if (o.ring == 0) o.ring = 1;
    if (o.max_requests < 1 || o.max_requests > 65536)
        return fail(TM_ERR_ARG, "tm_server_create: max_requests out of range [1, 65536]");
    if (o.ring < 1 || o.ring > 8) return fail(TM_ERR_ARG, "tm_server_create: ring out of range [1, 8]");
    if (o.block != 0 && o.block != 64 && o.block != 128 && o.block != 256)
        return fail(TM_ERR_ARG, "tm_server_create: block must be 64, 128 or 256");
    if (o.sort < 0 || o.sort > 2 || o.max_steps < 0)
        return fail(TM_ERR_ARG, "tm_server_create: bad sort or max_steps");
    if (!(o.eps >= 0.0f) || !(o.eps < 1.0f)) return fail(TM_ERR_ARG, "tm_server_create: eps must be in [0, 1)");
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (int32_t k = 0; k < n_meshes; ++k) {
        if (!meshes[k]) return fail(TM_ERR_ARG, "tm_server_create: mesh %d is NULL", k);
        if (meshes[k]->device != dev)
            return fail(TM_ERR_ARG, "tm_server_create: mesh %d is on device %d, current device %d", k,
                        meshes[k]->device, dev);
        if (meshes[k]->layout != meshes[0]->layout)
            return fail(TM_ERR_ARG, "tm_server_create: mesh %d has another record layout than mesh 0", k);
    }
    tm_server_s* s = new (std::nothrow) tm_server_s();
    if (!s) return fail(TM_ERR_OOM, "tm_server_create: host allocation failed");
    s->device = dev;
    s->meshes.assign(meshes, meshes + n_meshes);
    s->o = o;
    const int64_t cap = o.max_rays;
    int rc;
    if ((rc = alloc(s, &s->pool.orig, 3 * cap)) || (rc = alloc(s, &s->pool.dir, 3 * cap)) ||
        (rc = alloc(s, &s->pool.tmax, cap)) || (rc = alloc(s, &s->pool.sf, cap)) ||
        (rc = alloc(s, &s->pool.tri, cap)) || (rc = alloc(s, &s->pool.t, cap)) ||
        (rc = alloc(s, &s->pool.bary, 2 * cap))) {
        release(s);
        delete s;
        return rc;
    }
    s->ranges.reset(cap);
    s->ring.resize(size_t(o.ring));
    for (Slot& sl : s->ring) {
        hipError_t e = hipSuccess;
        const size_t gb = size_t(o.max_requests) * sizeof(tetrt::GenEntry);
        if ((rc = tm_batch_create(o.max_requests, cap, &sl.batch)) != TM_OK) {
            release(s);
            delete s;
            return rc;
        }
        if ((e = hipMalloc(&sl.d_gen, gb)) != hipSuccess || (e = hipHostMalloc(&sl.h_gen, gb, hipHostMallocDefault)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) {
            (void)hipGetLastError();
            release(s);
            delete s;
            return fail(TM_ERR_OOM, "tm_server_create: launch ring: %s", hipGetErrorString(e));
        }
    }
    *out = s;
    return TM_OK;
}

int tm_server_submit(tm_server s, const tm_request* req, int64_t* id) {
    tetrt::clear_error();
    if (!s || !req || !id) return fail(TM_ERR_ARG, "tm_server_submit: NULL argument");
    const tm_request& r = *req;
    if (r.mesh < 0 || r.mesh >= int32_t(s->meshes.size()))
        return fail(TM_ERR_ARG, "tm_server_submit: mesh index %d out of range", r.mesh);
    Req q;
    int rc = make_entry(r, s->meshes[size_t(r.mesh)], "tm_server_submit", true, &q.gen);
    if (rc != TM_OK) return rc;
    const int64_t n = int64_t(r.width) * r.height;
    if (n > s->o.max_rays)
        return fail(TM_ERR_ARG, "tm_server_submit: %lld pixels exceed the ray pool (%lld)", (long long)n,
                    (long long)s->o.max_rays);
    q.r = r;
    q.id = s->next_id++;
    q.submit_ns = now_ns();
    q.n = n;
    s->reqs[q.id] = q;
    s->queue.push_back(q.id);
    *id = q.id;
    return TM_OK;
}

int tm_request_rays(tm_mesh m, const tm_request* req, int32_t phase, float* d_orig, float* d_dir,
                    float* d_tmax, int32_t* d_start_face, const int32_t* d_tri, const float* d_t,
                    void* hip_stream) {
    tetrt::clear_error();
    if (!m || !req) return fail(TM_ERR_ARG, "tm_request_rays: NULL argument");
    if (phase != 0 && !(phase == 1 && req->kind != TM_REQ_PRIMARY))
        return fail(TM_ERR_ARG, "tm_request_rays: phase must be 0, or 1 for shadow and AO requests");
    if (!d_orig || !d_dir || !d_tmax || !d_start_face || (phase == 1 && (!d_tri || !d_t)))
        return fail(TM_ERR_ARG, "tm_request_rays: NULL array");
    tetrt::GenEntry g;
    int rc = make_entry(*req, m, "tm_request_rays", false, &g);
    if (rc != TM_OK) return rc;
    g.kind = phase == 0 ? tetrt::kGenCamera : (req->kind == TM_REQ_SHADOW ? tetrt::kGenShadow : tetrt::kGenAO);
    g.base = 0;
    g.block0 = 0;
    tetrt::RayPool p{};
    p.orig = d_orig;
    p.dir = d_dir;
    p.tmax = d_tmax;
    p.sf = d_start_face;
    p.tri = const_cast<int32_t*>(d_tri);
    p.t = const_cast<float*>(d_t);
    hipError_t e = tetrt::launch_gen_one(g, p, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "tm_request_rays: kernel launch");
    return TM_OK;
}

int tm_server_step(tm_server s, void* hip_stream, int64_t* launched) {
    tetrt::clear_error();
    if (!s) return fail(TM_ERR_ARG, "tm_server_step: NULL server");
    return step(s, static_cast<hipStream_t>(hip_stream), launched);
}

int tm_server_poll(tm_server s, tm_done* out, int32_t max, int32_t* n) {
    tetrt::clear_error();
    if (!s || !n || max < 0 || (max > 0 && !out)) return fail(TM_ERR_ARG, "tm_server_poll: bad argument");
    hipError_t e = retire(s, false);
    if (e != hipSuccess) return hip_fail(e, "tm_server_poll: a launch failed");
    int32_t k = 0;
    while (k < max && !s->finished.empty()) {
        out[k++] = s->finished.front();
        s->finished.pop_front();
    }
    *n = k;
    return TM_OK;
}

int tm_server_drain(tm_server s, void* hip_stream) {
    tetrt::clear_error();
    if (!s) return fail(TM_ERR_ARG, "tm_server_drain: NULL server");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    for (;;) {
        int64_t launched = 0;
        int rc = step(s, stream, &launched);
        if (rc != TM_OK) return rc;
        if (s->reqs.empty()) return TM_OK;
        if (launched == 0) {
            if (s->order.empty())
                return fail(TM_ERR_ARG, "tm_server_drain: requests left that cannot be scheduled");
            hipError_t e = retire(s, true);
            if (e != hipSuccess) return hip_fail(e, "tm_server_drain: a launch failed");
        }
    }
}

int tm_server_pending(tm_server s, int64_t* queued, int64_t* admitted, int64_t* finished) {
    tetrt::clear_error();
    if (!s) return fail(TM_ERR_ARG, "tm_server_pending: NULL server");
    if (queued) *queued = int64_t(s->queue.size());
    if (admitted) *admitted = s->admitted;
    if (finished) *finished = int64_t(s->finished.size());
    return TM_OK;
}

int tm_server_free(tm_server s) {
    tetrt::clear_error();
    if (!s) return TM_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != s->device) (void)hipSetDevice(s->device);
    hipError_t e = hipDeviceSynchronize();
    release(s);
    if (prev != s->device) (void)hipSetDevice(prev);
    delete s;
    if (e != hipSuccess) return hip_fail(e, "tm_server_free: device synchronize");
    return TM_OK;
}

}  // extern "C"
