// trace_closest_noalloc: trace_closest for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  Its scratch --
// the ray-binning permutation, the queue kernel's counters, the precision
// variant's tie list -- lives in `scratch` below, a fixed array of the code
// object: each device the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to a
// kernel (in host code it names a host-side stand-in, not device memory): the
// device address is looked up once per device with hipGetSymbolAddress and
// that pointer is what the binning and walk kernels receive.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "device.h"
#include "handle.h"
#include "tetrt.h"

namespace {

constexpr int64_t kScratchRays = TM_NOALLOC_MAX_BINNED_RAYS;
constexpr int kMaxDevices = 64;

// the binning permutation (4 bytes per binned ray), then room for the queue
// kernel's counters and job entry and the precision variant's tie list
constexpr int64_t kScratchWords = kScratchRays + tetrt::kFixedExtraBytes / 4;
static __device__ __align__(256) int32_t scratch[kScratchWords];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there, with that device current).
int scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return tetrt::hip_fail(e, "trace_closest_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return tetrt::fail(TM_ERR_ARG, "trace_closest_noalloc: device %d beyond the %d supported", dev,
                           kMaxDevices);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return tetrt::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                   "trace_closest_noalloc: hipGetSymbolAddress(scratch)");
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TM_OK;
}

}  // namespace

extern "C" int trace_closest_noalloc(tm_mesh m, int64_t n_rays, const float* d_orig, const float* d_dir,
                                     const float* d_tmax, const int32_t* d_start_tet,
                                     const int32_t* d_start_face, int32_t* d_tri, float* d_t,
                                     float* d_bary, int32_t* d_hit_tets, int32_t* d_steps,
                                     const tm_trace_opts* opts, void* hip_stream) {
    tetrt::clear_error();
    void* ws = nullptr;
    if (int rc = scratch_ptr(&ws)) return rc;
    return tetrt::trace_impl(m, n_rays, d_orig, d_dir, d_tmax, d_start_tet, d_start_face, d_tri, d_t,
                             d_bary, d_hit_tets, d_steps, opts, hip_stream, ws,
                             kScratchWords * int64_t(sizeof(int32_t)), "trace_closest_noalloc");
}
