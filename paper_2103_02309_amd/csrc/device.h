// Device-side view of an uploaded mesh and the kernel launchers.
#pragma once
#include <cstdint>

#include <hip/hip_runtime_api.h>

namespace tetrt {

// Plain pointers into device memory owned by a tm_mesh handle; passed to the
// kernels by value.  Vector-typed arrays are stored as their scalar base type
// and reinterpreted in the kernels (int4 / float4 / int2, 16- or 8-byte aligned).
struct DevMesh {
    const int32_t* vx;        // [nt]      Tet20 xor field
    const int32_t* nb;        // [nt*4]    Tet20 neighbour fields (int4 per tet)
    const float* pts;         // [np*4]    float4 per point
    const int32_t* tetv;      // [nt*4]    ascending vertex ids (int4 per tet)
    const int32_t* cfv;       // [ntri*4]  constrained-face vertices (int4)
    const int32_t* cft;       // [ntri*2]  constrained-face tets (int2)
    const int32_t* t_new2old; // [nt]
    const int32_t* t_old2new; // [nt]
    const int32_t* seed;      // [G^3]
    float lo[3];
    float inv_cell[3];
    int32_t G;
    int32_t nt;
    int32_t np;
    int32_t ntri;
};

struct RayArgs {
    const float* orig;
    const float* dir;
    const float* tmax;
    const int32_t* start_tet;
    const int32_t* start_face;
    int32_t* tri;
    float* t;
    float* bary;
    int32_t* hit_tets;
    int32_t* steps;
    int64_t n;
    int32_t max_steps;
};

hipError_t launch_trace(const DevMesh& m, const RayArgs& r, int block, hipStream_t s);
hipError_t launch_locate(const DevMesh& m, int64_t n, const float* pts, int32_t* out,
                         int32_t max_steps, hipStream_t s);

}  // namespace tetrt
