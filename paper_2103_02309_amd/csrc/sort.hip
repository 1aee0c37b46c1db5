// Ray binning for coherent traversal.  The ray order a caller produces is
// usually already coherent in origin (pixel tiles, hit points of neighbouring
// pixels); what breaks a wavefront's coherence is secondary rays that leave a
// point in many directions.  So rays are regrouped inside chunks of 2^c
// consecutive rays: by quantised direction, then (optionally) by the low bits
// of the Morton index of their origin's cell in a grid over the mesh bounds.
// By default the origin is not used: a chunk of consecutive rays already comes
// from one small region, and reading the origins would double the bytes read.  Each
// chunk is counting-sorted by one workgroup in LDS (no global atomics, one pass
// over the rays), and the walk takes rays through the resulting permutation.
// The order within a bin is not deterministic; results are per ray and do not
// depend on it.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace tetrt {

namespace {

constexpr int kMinorBits = 4;   // origin-cell bits below the direction bin

__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    // bits of x (at most 10) to every third bit
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t cell_of(float v, float lo, float inv, int G) {
    // clamped in float first, so NaN and infinities land in a valid cell
    return uint32_t(fminf(fmaxf((v - lo) * inv, 0.0f), float(G - 1)));
}

__device__ __forceinline__ uint32_t qdir(float v, float h, int q) {
    return uint32_t(fminf(fmaxf((v + 1.0f) * h, 0.0f), float(q - 1)));
}

// key in [0, dirq^3 * 2^kMinorBits)
__device__ __forceinline__ uint32_t ray_key(const SortCfg& c, float ox, float oy, float oz, float dx,
                                            float dy, float dz) {
    const int G = 1 << c.cells_log2;
    const uint32_t cell = (spread3(cell_of(ox, c.lo[0], c.inv[0], G)) << 2) |
                          (spread3(cell_of(oy, c.lo[1], c.inv[1], G)) << 1) |
                          spread3(cell_of(oz, c.lo[2], c.inv[2], G));
    const float il = rsqrtf(fmaxf(dx * dx + dy * dy + dz * dz, 1e-30f));
    const int q = c.dirq;
    const float h = 0.5f * float(q);
    const uint32_t dirbin = (qdir(dx * il, h, q) * uint32_t(q) + qdir(dy * il, h, q)) * uint32_t(q) +
                            qdir(dz * il, h, q);
    return (dirbin << kMinorBits) | (cell & ((1u << kMinorBits) - 1u));
}

// Counting sort of one chunk (rays base .. base + 2^CHUNK_LOG2 - 1) by key.
template <int CHUNK_LOG2>
__device__ void sort_chunk(const SortCfg& c, const float* orig, const float* dir, int64_t n,
                           int32_t* perm, int64_t base) {
    constexpr int C = 1 << CHUNK_LOG2;
    constexpr int K = 64 << kMinorBits;            // dirq <= 4
    __shared__ uint32_t hist[K];
    __shared__ uint16_t keys[C];
    const int cnt = int(min<int64_t>(C, n - base));
    const int nb = c.dirq * c.dirq * c.dirq << kMinorBits;
    for (int k = threadIdx.x; k < K; k += 256) hist[k] = 0u;
    __syncthreads();
    for (int r = threadIdx.x; r < cnt; r += 256) {
        const int64_t i = base + r;
        // with no origin grid (cells_log2 = 0) the origins are not read at all
        const bool by_origin = c.cells_log2 > 0;
        const uint32_t key = ray_key(c, by_origin ? orig[3 * i] : 0.0f, by_origin ? orig[3 * i + 1] : 0.0f,
                                     by_origin ? orig[3 * i + 2] : 0.0f, dir[3 * i], dir[3 * i + 1],
                                     dir[3 * i + 2]);
        keys[r] = uint16_t(key);
        atomicAdd(&hist[key], 1u);
    }
    __syncthreads();
    // exclusive scan of the nb counters: 256 threads x (K / 256) each
    __shared__ uint32_t part[256];
    constexpr int per = K / 256;
    uint32_t v[per];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        const int b = threadIdx.x * per + k;
        v[k] = b < nb ? hist[b] : 0u;
        acc += v[k];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - acc;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        const int b = threadIdx.x * per + k;
        if (b < nb) hist[b] = run;
        run += v[k];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < cnt; r += 256) {
        const uint32_t pos = atomicAdd(&hist[keys[r]], 1u);
        perm[base + pos] = int32_t(base + r);
    }
}

template <int CHUNK_LOG2>
__global__ void __launch_bounds__(256) k_chunk_sort(SortCfg c, const float* orig, const float* dir,
                                                    int64_t n, int32_t* perm) {
    sort_chunk<CHUNK_LOG2>(c, orig, dir, n, perm, int64_t(blockIdx.x) << CHUNK_LOG2);
}

// Batched: chunk b belongs to the job whose chunk range holds it.
template <int CHUNK_LOG2>
__global__ void __launch_bounds__(256) k_chunk_sort_batch(const Job* __restrict__ jobs, int32_t n_jobs) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].chunk0 <= b) lo = mid; else hi = mid;
    }
    const RayArgs r = jobs[lo].r;
    if (!r.perm) return;
    const SortCfg c = jobs[lo].sc;
    const int64_t base = (b - jobs[lo].chunk0) << CHUNK_LOG2;
    if (base >= r.n) return;
    sort_chunk<CHUNK_LOG2>(c, r.orig, r.dir, r.n, const_cast<int32_t*>(r.perm), base);
}

}  // namespace

int64_t sort_workspace_bytes(int64_t n) { return (4 * n + 255) / 256 * 256; }

hipError_t launch_sort(const SortCfg& c, const float* orig, const float* dir, int64_t n, void* ws,
                       int32_t** perm_out, hipStream_t s) {
    int32_t* perm = static_cast<int32_t*>(ws);
    const int64_t C = int64_t(1) << c.chunk_log2;
    const unsigned grid = unsigned((n + C - 1) / C);
    switch (c.chunk_log2) {
        case 10: hipLaunchKernelGGL(k_chunk_sort<10>, dim3(grid), dim3(256), 0, s, c, orig, dir, n, perm); break;
        case 11: hipLaunchKernelGGL(k_chunk_sort<11>, dim3(grid), dim3(256), 0, s, c, orig, dir, n, perm); break;
        case 12: hipLaunchKernelGGL(k_chunk_sort<12>, dim3(grid), dim3(256), 0, s, c, orig, dir, n, perm); break;
        default: hipLaunchKernelGGL(k_chunk_sort<13>, dim3(grid), dim3(256), 0, s, c, orig, dir, n, perm); break;
    }
    *perm_out = perm;
    return hipGetLastError();
}

hipError_t launch_sort_batch(const Job* d_jobs, int32_t n_jobs, int64_t total_chunks,
                             int32_t chunk_log2, hipStream_t s) {
    if (total_chunks <= 0 || n_jobs <= 0) return hipSuccess;
    const dim3 g{unsigned(total_chunks)}, b{256u};
    switch (chunk_log2) {
        case 10: hipLaunchKernelGGL(k_chunk_sort_batch<10>, g, b, 0, s, d_jobs, n_jobs); break;
        case 11: hipLaunchKernelGGL(k_chunk_sort_batch<11>, g, b, 0, s, d_jobs, n_jobs); break;
        case 12: hipLaunchKernelGGL(k_chunk_sort_batch<12>, g, b, 0, s, d_jobs, n_jobs); break;
        default: hipLaunchKernelGGL(k_chunk_sort_batch<13>, g, b, 0, s, d_jobs, n_jobs); break;
    }
    return hipGetLastError();
}

}  // namespace tetrt
