// Host-side state of an uploaded mesh and the error helpers shared by the C-ABI
// translation units.
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"
#include "tetrt.h"

struct tm_mesh_s {
    tetrt::DevMesh dev{};
    int device = 0;
    int cus = 0;
    int64_t np = 0, nt = 0, ntri = 0;
    int32_t layout = 0, sfc = 0;
    int64_t n_regions = 0;
    int64_t hot_bytes = 0, cold_bytes = 0;
    std::vector<int32_t> tri_verts_user;  // host copy for tetmesh_tri_vertices
    std::vector<void*> allocations;
    float lo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};  // bounds of the points
    // The handle's own binning workspace (tm_upload_opts.bin_rays), fixed at
    // upload.  Traces that bin through it are ordered one after another: ws_done
    // is recorded on ws_stream after each, and a trace on another stream waits
    // for it on the device before its binning overwrites the permutation.
    std::mutex ws_mu;
    void* ws = nullptr;
    int64_t ws_bytes = 0;
    hipEvent_t ws_done = nullptr;
    hipStream_t ws_stream = nullptr;
    bool ws_used = false;
};

namespace tetrt {

void clear_error();
const char* last_error();
// Record a printf-style message for tm_last_error and return code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);
// Accelerator dies (XCDs) of a device with `cus` compute units: 32 CUs per XCD
// on MI355X (256 CUs, 8 XCDs).
inline int32_t xcd_count(int cus) { return cus >= 64 ? cus / 32 : 1; }
// Binning configuration of a trace of n rays; *on = false when they are not binned.
int sort_config(const tm_mesh_s* m, const tm_trace_opts& o, int64_t n, bool has_tmax, SortCfg* c,
                bool* on);

// Room beyond the binning permutation in a fixed workspace (the queue kernel's
// counters and job entry, the precision variant's tie list).
constexpr int64_t kFixedExtraBytes = 512 * 1024;

// The body of trace_closest.  fixed_ws (non-null): the binning workspace to
// use instead of the caller's or the handle's (fixed_ws_bytes long); `name`
// prefixes error messages.
int trace_impl(tm_mesh_s* m, int64_t n_rays, const float* d_orig, const float* d_dir,
               const float* d_tmax, const int32_t* d_start_tet, const int32_t* d_start_face,
               int32_t* d_tri, float* d_t, float* d_bary, int32_t* d_hit_tets, int32_t* d_steps,
               const tm_trace_opts* opts, void* hip_stream, void* fixed_ws, int64_t fixed_ws_bytes,
               const char* name);

}  // namespace tetrt
