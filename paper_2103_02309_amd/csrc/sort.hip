// Ray binning for coherent traversal: rays are grouped by the cell of their
// origin (Morton order of a 2^k grid over the mesh bounds) and then by a
// quantised direction, with a counting sort (count, exclusive scan, scatter).
// The walk then takes rays in this order through a permutation, so that the
// lanes of a wavefront start close together and head the same way, and visit
// the same tet records and points.  Order within a bin is not deterministic;
// results are per ray and do not depend on it.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace tetrt {

namespace {

constexpr int kScanBlock = 1024;   // bins per scan block (256 threads x 4)

__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    // bits of x (at most 10) to every third bit
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ int cell_of(float v, float lo, float inv, int G) {
    // clamped in float first, so NaN and infinities land in a valid cell
    const float g = fminf(fmaxf((v - lo) * inv, 0.0f), float(G - 1));
    return int(g);
}

__device__ __forceinline__ uint32_t ray_key(const SortCfg& c, float ox, float oy, float oz, float dx,
                                            float dy, float dz) {
    const int G = 1 << c.cells_log2;
    const uint32_t cx = uint32_t(cell_of(ox, c.lo[0], c.inv[0], G));
    const uint32_t cy = uint32_t(cell_of(oy, c.lo[1], c.inv[1], G));
    const uint32_t cz = uint32_t(cell_of(oz, c.lo[2], c.inv[2], G));
    const uint32_t cell = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
    const float il = rsqrtf(fmaxf(dx * dx + dy * dy + dz * dz, 1e-30f));
    const int q = c.dirq;
    const float h = 0.5f * float(q);
    const uint32_t bx = uint32_t(fminf(fmaxf((dx * il + 1.0f) * h, 0.0f), float(q - 1)));
    const uint32_t by = uint32_t(fminf(fmaxf((dy * il + 1.0f) * h, 0.0f), float(q - 1)));
    const uint32_t bz = uint32_t(fminf(fmaxf((dz * il + 1.0f) * h, 0.0f), float(q - 1)));
    return cell * uint32_t(q * q * q) + (bx * uint32_t(q) + by) * uint32_t(q) + bz;
}

__global__ void k_fill_zero(uint32_t* p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_count(SortCfg c, const float* orig, const float* dir, int64_t n, uint32_t* bins) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = ray_key(c, orig[3 * i], orig[3 * i + 1], orig[3 * i + 2], dir[3 * i],
                               dir[3 * i + 1], dir[3 * i + 2]);
    atomicAdd(&bins[k], 1u);
}

// Exclusive scan of kScanBlock bins per block, in place; the block's total goes
// to sums[blockIdx.x].
__global__ void __launch_bounds__(256) k_scan_block(uint32_t* bins, int64_t nbins, uint32_t* sums) {
    __shared__ uint32_t part[256];
    const int64_t base = int64_t(blockIdx.x) * kScanBlock + threadIdx.x * 4;
    uint32_t v[4];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < nbins ? bins[base + k] : 0u;
        acc += v[k];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive scan of the thread totals
        const uint32_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - acc;     // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < nbins) bins[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = part[255];
}

// Exclusive scan of the block totals in one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan_sums(uint32_t* sums, int32_t nsums) {
    __shared__ uint32_t part[1024];
    const int per = (nsums + 1023) / 1024;
    const int b = threadIdx.x * per;
    uint32_t acc = 0;
    for (int k = 0; k < per; ++k)
        if (b + k < nsums) acc += sums[b + k];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - acc;
    for (int k = 0; k < per; ++k)
        if (b + k < nsums) {
            const uint32_t x = sums[b + k];
            sums[b + k] = run;
            run += x;
        }
}

__global__ void k_scan_add(uint32_t* bins, int64_t nbins, const uint32_t* sums) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nbins) bins[i] += sums[i / kScanBlock];
}

__global__ void k_scatter(SortCfg c, const float* orig, const float* dir, int64_t n, uint32_t* bins,
                          int32_t* perm) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = ray_key(c, orig[3 * i], orig[3 * i + 1], orig[3 * i + 2], dir[3 * i],
                               dir[3 * i + 1], dir[3 * i + 2]);
    const uint32_t pos = atomicAdd(&bins[k], 1u);
    perm[pos] = int32_t(i);
}

}  // namespace

int64_t sort_workspace_bytes(int64_t n, int64_t nbins) {
    const int64_t nsums = (nbins + kScanBlock - 1) / kScanBlock;
    auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
    return up(4 * nbins) + up(4 * nsums) + up(4 * n);
}

hipError_t launch_sort(const SortCfg& c, const float* orig, const float* dir, int64_t n, void* ws,
                       int32_t** perm_out, hipStream_t s) {
    const int64_t nbins = c.nbins;
    const int64_t nsums = (nbins + kScanBlock - 1) / kScanBlock;
    auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
    char* p = static_cast<char*>(ws);
    uint32_t* bins = reinterpret_cast<uint32_t*>(p);
    uint32_t* sums = reinterpret_cast<uint32_t*>(p + up(4 * nbins));
    int32_t* perm = reinterpret_cast<int32_t*>(p + up(4 * nbins) + up(4 * nsums));
    const int B = 256;
    hipLaunchKernelGGL(k_fill_zero, dim3(unsigned((nbins + B - 1) / B)), dim3(B), 0, s, bins, nbins);
    hipLaunchKernelGGL(k_count, dim3(unsigned((n + B - 1) / B)), dim3(B), 0, s, c, orig, dir, n, bins);
    hipLaunchKernelGGL(k_scan_block, dim3(unsigned(nsums)), dim3(256), 0, s, bins, nbins, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, int32_t(nsums));
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned((nbins + B - 1) / B)), dim3(B), 0, s, bins, nbins, sums);
    hipLaunchKernelGGL(k_scatter, dim3(unsigned((n + B - 1) / B)), dim3(B), 0, s, c, orig, dir, n, bins,
                       perm);
    *perm_out = perm;
    return hipGetLastError();
}

}  // namespace tetrt
