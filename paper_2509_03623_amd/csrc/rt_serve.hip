// rt_serve.hip -- device side of the render server: a persistent forward
// launch over the work items of every request in a batch, and the fused L2
// loss / cotangent of forward+adjoint requests.
//
// A batch holds up to max_slots requests; its work items are (request,
// 8 x 8 pixel tile, 16-channel block) in request order.  The four adjacent
// lanes of a pixel march consecutive quarters of its ray and compose them by
// shuffles at the end (front-to-back composition is associative), so an
// item's latency is a quarter of its ray.  The launch has a fixed number of
// workgroups; each pulls the next item index from a device counter until the
// batch is exhausted, so items of small and large requests of the batch share
// the GPU.  Every wave exits once the counter passes the item count.
#include "rt_host.h"
#include "rt_serve.h"

namespace rt {

constexpr int kServeCB = 16;
static_assert(kServeTile * kServeTile * kServeSplit == 256, "one item per 256-lane workgroup");

__global__ __launch_bounds__(256) void serve_fwd(const ServeDesc *__restrict__ descs, int nreq, uint32_t nitems,
                                                 uint32_t *__restrict__ counter) {
    __shared__ float4 ztab[kZTableNodes - 1];
    __shared__ uint32_t s_item;
    __shared__ const float4 *s_tab;
    if (threadIdx.x == 0) s_tab = nullptr;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: scalar from here on
        if (item >= nitems) break;
        // request of this item: last descriptor whose first item <= item
        int lo = 0, hi = nreq - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (descs[mid].item0 <= item) lo = mid; else hi = mid - 1;
        }
        // the request index is the same for every lane: keep its descriptor in
        // scalar registers for the whole item
        const ServeDesc D = descs[__builtin_amdgcn_readfirstlane(lo)];
        if (s_tab != D.s.ztab) {     // uniform: every lane reads the same s_tab
            __syncthreads();
            for (int i = threadIdx.x; i < kZTableNodes - 1; i += 256) ztab[i] = D.s.ztab[i];
            __syncthreads();
            if (threadIdx.x == 0) s_tab = D.s.ztab;
        }
        const uint32_t local = item - D.item0;
        const int blk = (int)(local % (uint32_t)D.nblk);
        const int tile = (int)(local / (uint32_t)D.nblk);
        const Geometry &g = D.g;
        const int split = threadIdx.x % kServeSplit, slot = threadIdx.x / kServeSplit;
        const int p = (tile % D.tiles_x) * kServeTile + slot % kServeTile;
        const int q = (tile / D.tiles_x) * kServeTile + slot / kServeTile;
        const int c0 = blk * kServeCB;
        const bool inside = p < g.nx && q < g.ny;
        float I[kServeCB], Tr[kServeCB];
#pragma unroll
        for (int c = 0; c < kServeCB; ++c) { I[c] = 0.0f; Tr[c] = 1.0f; }
        float vc[kServeCB];
#pragma unroll
        for (int c = 0; c < kServeCB; ++c) vc[c] = D.vch[c0 + c];
        const RaySetup r = ray_setup(g, inside ? p : 0, inside ? q : 0);
        if (inside && r.live) {
            const float half = 0.5f * (float)g.nsamp;
            const int len = (g.nsamp + kServeSplit - 1) / kServeSplit;
            const int k0 = split * len, k1 = min(g.nsamp, k0 + len);
            for (int k = k0; k < k1; ++k) {
                const float t = ((float)k + 0.5f - half) * r.ds;
                const SampleQ sq = shade_sample<false>(D.s, ztab, r.px, fmaf(t, r.wy, r.pmy),
                                                       fmaf(t, r.wz, r.pmz), r.ds, 0);
                // no ray of the wave with opacity at this sample: no channel changes
                if (__ballot(sq.K > 0.0f) == 0) continue;
                march_sample<kServeCB, true>(I, Tr, sq, [&](int c) { return vc[c]; });
            }
        }
        // compose the quarters front to back (every lane takes part in the shuffles)
#pragma unroll
        for (int d = 1; d < kServeSplit; d <<= 1) {
#pragma unroll
            for (int c = 0; c < kServeCB; ++c) {
                const float Ib = __shfl_down(I[c], d, kServeSplit);
                const float Tb = __shfl_down(Tr[c], d, kServeSplit);
                if ((split & (2 * d - 1)) == 0) {
                    I[c] = fmaf(Tr[c], Ib, I[c]);
                    Tr[c] *= Tb;
                }
            }
        }
        if (inside && split == 0) {
            const size_t plane = (size_t)g.nx * g.ny, pix = (size_t)q * g.nx + p;
#pragma unroll
            for (int c = 0; c < kServeCB; ++c)
                if (c0 + c < D.nch) D.cube[(size_t)(c0 + c) * plane + pix] = I[c];
        }
    }
}

hipError_t launch_serve_fwd(const ServeDesc *descs, int nreq, uint32_t nitems, uint32_t *counter, int nwg,
                            hipStream_t st) {
    hipLaunchKernelGGL(serve_fwd, dim3(nwg), dim3(256), 0, st, descs, nreq, nitems, counter);
    return hipGetLastError();
}

// dl = 2 (cube - target); L += sum (cube - target)^2 (double atomics)
__global__ __launch_bounds__(256) void l2_loss(const float *__restrict__ cube, const float *__restrict__ target,
                                               float *__restrict__ dl, size_t n, double *__restrict__ loss) {
    __shared__ double part[256];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float r = cube[i] - target[i];
        dl[i] = 2.0f * r;
        acc += (double)r * (double)r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, part[0]);
}

__global__ void zero_double(double *p) { *p = 0.0; }

// L = sum (cube - target)^2 (double atomics)
__global__ __launch_bounds__(256) void l2_value(const float *__restrict__ cube, const float *__restrict__ target,
                                                size_t n, double *__restrict__ loss) {
    __shared__ double part[256];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double r = (double)cube[i] - (double)target[i];
        acc += r * r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, part[0]);
}

hipError_t launch_l2_value(const float *cube, const float *target, size_t n, double *loss, hipStream_t st) {
    hipLaunchKernelGGL(zero_double, dim3(1), dim3(1), 0, st, loss);
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(l2_value, dim3(blocks), dim3(256), 0, st, cube, target, n, loss);
    return hipGetLastError();
}

__global__ void zero_doubles(double *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// blockIdx.y = request of the batch; each request's elements grid-strided
// over blockIdx.x, block partial sums added with FP64 atomics
__global__ __launch_bounds__(256) void l2_batch(const ServeDesc *__restrict__ descs) {
    const ServeDesc &D = descs[blockIdx.y];
    if (!D.target) return;
    __shared__ double part[256];
    const size_t n = (size_t)D.nch * D.g.nx * D.g.ny;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double r = (double)D.cube[i] - (double)D.target[i];
        acc += r * r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(D.loss, part[0]);
}

hipError_t launch_l2_batch(const ServeDesc *descs, int nreq, double *losses, size_t max_n, hipStream_t st) {
    hipLaunchKernelGGL(zero_doubles, dim3(1), dim3(256), 0, st, losses, nreq);
    const int blocks = (int)std::min<size_t>((max_n + 255) / 256, 256);
    hipLaunchKernelGGL(l2_batch, dim3(blocks, nreq), dim3(256), 0, st, descs);
    return hipGetLastError();
}

hipError_t launch_l2_loss(const float *cube, const float *target, float *dl, size_t n, double *loss, hipStream_t st) {
    hipLaunchKernelGGL(zero_double, dim3(1), dim3(1), 0, st, loss);
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(l2_loss, dim3(blocks), dim3(256), 0, st, cube, target, dl, n, loss);
    return hipGetLastError();
}

} // namespace rt
