// Calibration kernel for the benchmark, built into a library of its own
// (libtetrt_probe.so) beside the traversal library: the rate at which a CU's
// vector L1 serves wave loads whose lanes each read 16 bytes, for a chosen
// spread of the lanes' addresses over cache lines.
//
// The walk reads, per ray and step, one 16-byte record and one 12-byte point at
// addresses that differ from lane to lane; a wave's load then touches up to 64
// cache lines.  The L1 looks lines up at a fixed rate per cycle, so that rate,
// not the bytes moved, is what such loads are limited by.  This kernel
// measures it: every lane of every wave issues `iters` independent 16-byte
// loads whose addresses follow `mode` (independent loads, or in mode 3 a chain
// in which each load waits for the previous one), and the caller times the
// launch.
//
// C-ABI (declared here only; not part of the traversal library's header):
//   int tetrt_probe_l1(const void* d_buf, uint64_t buf_bytes, int32_t mode,
//                      uint32_t unit_bytes, uint32_t units, int32_t blocks,
//                      int32_t iters, void* d_out, void* hip_stream);
//     Every lane of `blocks` 256-thread blocks issues `iters` independent
//     16-byte loads from d_buf (device, buf_bytes bytes, read only) at the
//     start of unit u of `units` units of `unit_bytes` bytes:
//       mode 0  u pseudo-random per lane (a wave touches up to 64 units);
//       mode 1  eight consecutive lanes per unit (8 units per wave load);
//       mode 2  one unit per wave load;
//       mode 3  u pseudo-random per lane as in mode 0, but each load's address
//               also depends on the value the lane's previous load returned
//               (a dependent chain per lane, as in a walk).
//
//     d_out: device, blocks * 256 * 16 bytes, receives per-lane sums (so the
//     loads stay).  Enqueued on hip_stream (NULL = default stream).  Returns 0,
//     -1 for a bad argument (unknown mode, unit_bytes not a multiple of 16,
//     units not a power of two, units * unit_bytes > buf_bytes, blocks or iters
//     outside [1, 2^20], NULL buffers), or -4 when the launch fails;
//     tetrt_probe_last_error() then describes it (per calling thread).
//   const char* tetrt_probe_last_error(void);

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace {

constexpr int32_t kRandom = 0;
constexpr int32_t kEightLanes = 1;
constexpr int32_t kOneLine = 2;
constexpr int32_t kChain = 3;

thread_local std::string g_probe_error;

int probe_fail(int code, const char* msg) {
    g_probe_error = msg;
    return code;
}

__global__ void __launch_bounds__(256) k_probe_l1(const uint4* __restrict__ buf, uint32_t units,
                                                  uint32_t unit_u4, int32_t mode, int32_t iters,
                                                  uint4* __restrict__ out) {
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t x = g * 2654435761u + 12345u;   // per-lane linear congruential sequence
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    if (mode == kChain) {
        uint32_t dep = 0u;
        for (int32_t k = 0; k < iters; ++k) {
            x = x * 1664525u + 1013904223u;
            const uint32_t u = ((x ^ dep) >> 8) & (units - 1u);
            const uint4 v = buf[size_t(u) * unit_u4];
            acc.x += v.x; acc.y ^= v.y; acc.z += v.z; acc.w ^= v.w;
            dep = v.x;
        }
        out[g] = acc;
        return;
    }
    for (int32_t k = 0; k < iters; ++k) {
        x = x * 1664525u + 1013904223u;
        uint32_t u;
        if (mode == kRandom) u = (x >> 8) & (units - 1u);
        else if (mode == kEightLanes) u = ((uint32_t(k) * 64u + lane) >> 3) & (units - 1u);
        else u = uint32_t(k) & (units - 1u);
        const uint4 v = buf[size_t(u) * unit_u4];
        acc.x += v.x; acc.y ^= v.y; acc.z += v.z; acc.w ^= v.w;
    }
    out[g] = acc;
}

}  // namespace

extern "C" const char* tetrt_probe_last_error(void) { return g_probe_error.c_str(); }

extern "C" int tetrt_probe_l1(const void* d_buf, uint64_t buf_bytes, int32_t mode, uint32_t unit_bytes,
                              uint32_t units, int32_t blocks, int32_t iters, void* d_out, void* hip_stream) {
    g_probe_error.clear();
    if (mode != kRandom && mode != kEightLanes && mode != kOneLine && mode != kChain)
        return probe_fail(-1, "tetrt_probe_l1: unknown mode");
    if (unit_bytes < 16 || unit_bytes % 16 || units == 0 || (units & (units - 1u)))
        return probe_fail(-1, "tetrt_probe_l1: unit_bytes must be a multiple of 16, units a power of 2");
    if (uint64_t(units) * unit_bytes > buf_bytes)
        return probe_fail(-1, "tetrt_probe_l1: units * unit_bytes exceeds the buffer");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
        return probe_fail(-1, "tetrt_probe_l1: blocks and iters must be in [1, 2^20]");
    if (!d_buf || !d_out) return probe_fail(-1, "tetrt_probe_l1: NULL buffer");
    hipLaunchKernelGGL(k_probe_l1, dim3(unsigned(blocks)), dim3(256), 0, hipStream_t(hip_stream),
                       static_cast<const uint4*>(d_buf), units, unit_bytes / 16u, mode, iters,
                       static_cast<uint4*>(d_out));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char buf[256];
        snprintf(buf, sizeof buf, "tetrt_probe_l1: launch: %s", hipGetErrorString(e));
        return probe_fail(-4, buf);
    }
    return 0;
}
