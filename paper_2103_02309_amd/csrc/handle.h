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
    int64_t hot_bytes = 0, cold_bytes = 0;
    std::vector<int32_t> tri_verts_user;  // host copy for tetmesh_tri_vertices
    std::vector<void*> allocations;
    float lo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};  // bounds of the points
    std::mutex ws_mu;                   // the handle's workspace for ray binning
    void* ws = nullptr;
    int64_t ws_bytes = 0;
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

}  // namespace tetrt
