// rt_noalloc.hip -- the fused forward + L2 loss + adjoint without any
// allocation, for callers that cannot allocate device memory.
//
// Everything the call needs beyond the caller's inputs and outputs (the
// partition-function table, the gradient accumulators and the adjoint's
// sample tape and cotangents for one band of image rows) is carved from one
// file-scope device array.  The array exists once per GPU, for the life of
// the process, and every call on that GPU shares it: calls that overlap on one
// GPU (from different streams or threads) race.  Each call clears what must
// start at zero (the accumulators, the loss) with kernels before using it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rt_host.h"

namespace rt {

// Size of the fixed region: the table (8 KiB), the accumulators (0.8 MB on a
// 256 x 128 grid) and the band scratch (16 B per pixel-sample for the tape
// plus 16 B per pixel-sample and cotangent slice: one 512-pixel row of a
// 64-channel, 512-sample image is 8.4 MB, so a band is ~30 such rows).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};

// The array's device address on the current device, looked up once per
// device (the host-side name is only a stand-in for the symbol).
rt_status scratch_ptr(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RT_EDEVICE, "device %d beyond the library's device table", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = (char *)p;
    }
    *out = g_ptr[dev];
    return RT_OK;
}
} // namespace

} // namespace rt

using namespace rt;

extern "C" rt_status rt_render_cube_l2_adjoint_noalloc(const rt_problem *p, const float *target, const rt_grads *g,
                                                       float *cube, double *loss, void *stream) {
    rt_status st = validate(p);
    if (st != RT_OK) return st;
    if (!target || !cube) return fail(RT_EINVAL, "target and cube must not be NULL");
    if (!g) return fail(RT_EINVAL, "grads is NULL");
    if (p->mlp || g->d_mlp) return fail(RT_EINVAL, "the allocation-free adjoint takes grid fields only (no network)");
    if (p->spec.nch > kLaunchChannels)
        return fail(RT_EINVAL, "the fused L2 adjoint takes at most %d channels per call", kLaunchChannels);
    if (fixed_scratch_min_bytes(p) > kNoAllocScratchBytes)
        return fail(RT_ETOOBIG, "the call needs %llu bytes of scratch for one row of pixels; the fixed region "
                                "holds %llu", (unsigned long long)fixed_scratch_min_bytes(p),
                    (unsigned long long)kNoAllocScratchBytes);
    char *base = nullptr;
    st = scratch_ptr(&base);
    if (st != RT_OK) return st;
    const FixedScratch fx{base, kNoAllocScratchBytes};
    hipStream_t s = (hipStream_t)stream;
    st = adjoint_core(p, nullptr, g, cube, s, nullptr, nullptr, target, &fx);
    if (st != RT_OK || !loss) return st;
    const size_t n = (size_t)p->spec.nch * p->cam.nx * p->cam.ny;
    const hipError_t e = launch_l2_value(cube, target, n, loss, s);
    return e == hipSuccess ? RT_OK : fail_hip(e, "loss");
}

extern "C" uint64_t rt_noalloc_scratch_bytes(void) { return (uint64_t)kNoAllocScratchBytes; }
