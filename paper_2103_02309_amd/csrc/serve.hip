// Ray generation for the serving loop: camera rays of a request, and the
// shadow or ambient-occlusion ray that leaves each camera ray's hit.  One
// launch covers every request of a scheduler step; a block finds its request
// in the entry table as the batched walk does.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.h"

namespace tetrt {

namespace {

// 32-bit permutation hash of the PCG family (Jarzynski and Olano, "Hash
// Functions for GPU Rendering", JCGT 9(3), 2020: the pcg hash).
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

// uniform in [0, 1) with 24 random bits
__device__ __forceinline__ float unit_float(uint32_t h) { return float(h >> 8) * (1.0f / 16777216.0f); }

__device__ __forceinline__ void tile_pixel(int64_t i, int W, int& px, int& py) {
    const int64_t tile = i >> 6;
    const int in = int(i & 63);
    const int tiles_x = W >> 3;
    px = int(tile % tiles_x) * 8 + (in & 7);
    py = int(tile / tiles_x) * 8 + (in >> 3);
}

__device__ void camera_ray(const GenEntry& g, int64_t i, RayPool p) {
    int px, py;
    tile_pixel(i, g.W, px, py);
    const float sx = 2.0f * (float(px) + 0.5f) / float(g.W) - 1.0f;
    const float sy = 1.0f - 2.0f * (float(py) + 0.5f) / float(g.H);
    float d[3];
    for (int a = 0; a < 3; ++a) d[a] = g.fwd[a] + sx * g.right[a] + sy * g.up[a];
    const float il = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const int64_t k = g.base + i;
    for (int a = 0; a < 3; ++a) {
        p.orig[3 * k + a] = g.eye[a];
        p.dir[3 * k + a] = d[a] * il;
    }
    p.tmax[k] = INFINITY;
    p.sf[k] = -1;
}

__device__ void secondary_ray(const GenEntry& g, int64_t i, RayPool p) {
    const int64_t k = g.base + i;
    const int32_t tri = p.tri[k];
    float o[3], d[3];
    for (int a = 0; a < 3; ++a) {
        o[a] = p.orig[3 * k + a];
        d[a] = p.dir[3 * k + a];
    }
    if (tri < 0) {
        // no hit to leave from: a zero direction, which the walk reports as invalid
        for (int a = 0; a < 3; ++a) p.dir[3 * k + a] = 0.0f;
        p.tmax[k] = 0.0f;
        p.sf[k] = -1;
        return;
    }
    const float t = p.t[k];
    float h[3];
    for (int a = 0; a < 3; ++a) h[a] = fmaf(t, d[a], o[a]);
    float nd[3];
    if (g.kind == kGenShadow) {
        for (int a = 0; a < 3; ++a) nd[a] = g.light[a] - h[a];
        p.tmax[k] = 1.0f;        // the light is at t = 1
    } else {
        const int4 v = reinterpret_cast<const int4*>(g.cfv)[tri];
        const float* pa = g.pts + 3 * int64_t(v.x);
        const float* pb = g.pts + 3 * int64_t(v.y);
        const float* pc = g.pts + 3 * int64_t(v.z);
        const float3 A = make_float3(pa[0], pa[1], pa[2]);
        const float3 B = make_float3(pb[0], pb[1], pb[2]);
        const float3 C = make_float3(pc[0], pc[1], pc[2]);
        const float e1x = B.x - A.x, e1y = B.y - A.y, e1z = B.z - A.z;
        const float e2x = C.x - A.x, e2y = C.y - A.y, e2z = C.z - A.z;
        float n[3] = {e1y * e2z - e1z * e2y, e1z * e2x - e1x * e2z, e1x * e2y - e1y * e2x};
        // the hemisphere on the side the camera ray came from
        const float s = (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]) > 0.0f ? -1.0f : 1.0f;
        const float nl = s / sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int a = 0; a < 3; ++a) n[a] *= nl;
        // tangent frame: cross with the axis least aligned with n
        float ax[3] = {0.0f, 0.0f, 0.0f};
        ax[fabsf(n[0]) < 0.9f ? 0 : 1] = 1.0f;
        float t1[3] = {ax[1] * n[2] - ax[2] * n[1], ax[2] * n[0] - ax[0] * n[2], ax[0] * n[1] - ax[1] * n[0]};
        const float tl = 1.0f / sqrtf(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
        for (int a = 0; a < 3; ++a) t1[a] *= tl;
        const float t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
        // cosine-weighted direction (Malley: a uniform disk point lifted to the hemisphere)
        const uint32_t r0 = pcg_hash(g.seed ^ pcg_hash(uint32_t(2 * i)));
        const uint32_t r1 = pcg_hash(g.seed ^ pcg_hash(uint32_t(2 * i + 1)));
        const float u1 = unit_float(r0), u2 = unit_float(r1);
        const float rad = sqrtf(u1), phi = 6.283185307179586f * u2;
        const float x = rad * cosf(phi), y = rad * sinf(phi), z = sqrtf(fmaxf(0.0f, 1.0f - u1));
        for (int a = 0; a < 3; ++a) nd[a] = x * t1[a] + y * t2[a] + z * n[a];
        p.tmax[k] = g.ao_tmax;
    }
    for (int a = 0; a < 3; ++a) {
        p.orig[3 * k + a] = h[a];
        p.dir[3 * k + a] = nd[a];
    }
    p.sf[k] = tri;
}

__device__ __forceinline__ void gen_ray(const GenEntry& g, int64_t i, RayPool p) {
    if (i >= int64_t(g.W) * g.H) return;
    if (g.kind == kGenCamera)
        camera_ray(g, i, p);
    else
        secondary_ray(g, i, p);
}

__global__ void __launch_bounds__(kGenBlock) k_gen(const GenEntry* __restrict__ gen, int32_t n, RayPool p) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gen[mid].block0 <= b) lo = mid; else hi = mid;
    }
    const GenEntry& g = gen[lo];
    gen_ray(g, (b - g.block0) * kGenBlock + threadIdx.x, p);
}

__global__ void __launch_bounds__(kGenBlock) k_gen_one(GenEntry g, RayPool p) {
    gen_ray(g, int64_t(blockIdx.x) * kGenBlock + threadIdx.x, p);
}

}  // namespace

hipError_t launch_gen(const GenEntry* d_gen, int32_t n, int64_t total_blocks, RayPool pool, hipStream_t s) {
    if (n <= 0 || total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen, dim3{unsigned(total_blocks)}, dim3{unsigned(kGenBlock)}, 0, s, d_gen, n, pool);
    return hipGetLastError();
}

hipError_t launch_gen_one(const GenEntry& g, RayPool pool, hipStream_t s) {
    const int64_t n = int64_t(g.W) * g.H;
    if (n <= 0) return hipSuccess;
    const unsigned blocks = unsigned((n + kGenBlock - 1) / kGenBlock);
    hipLaunchKernelGGL(k_gen_one, dim3{blocks}, dim3{unsigned(kGenBlock)}, 0, s, g, pool);
    return hipGetLastError();
}

}  // namespace tetrt
