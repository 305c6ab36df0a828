// rt_census.hip -- work accounting of a render: which rays cross the grid's
// bounding volume (the others have no samples: zero intensity, no work), how
// many pixel-samples they hold, how many of those are optically thin in the
// march's sense (line-centre depth below the series threshold), how many
// have any opacity at all (K > 0: the others change no channel), and how many
// lie inside the grid's edge taper (the others are not shaded at all).  Uses the
// march's own ray set-up and shading, so the counts are those of the render.
#include "rt_host.h"
#include "rt_kernels.h"

namespace rt {

// blockIdx.y: a chunk of the samples of each ray
__global__ __launch_bounds__(256) void census(Geometry g, Shade s, uint8_t *__restrict__ mask,
                                              unsigned long long *__restrict__ counts, int shade) {
    __shared__ float4 ztab[kZTableNodes - 1];
    __shared__ unsigned long long part[4];
    if (shade) stage_ztab(s, ztab);
    if (threadIdx.x < 4) part[threadIdx.x] = 0ull;
    __syncthreads();
    const int npix = g.nx * g.ny;
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix < npix) {
        const RaySetup r = ray_setup(g, pix % g.nx, pix / g.nx);
        if (blockIdx.y == 0) {
            if (mask) mask[pix] = r.live ? 1 : 0;
            if (r.live) atomicAdd(&part[0], 1ull);
        }
        if (r.live && shade) {
            const float half = 0.5f * (float)g.nsamp;
            const int len = (g.nsamp + gridDim.y - 1) / gridDim.y;
            const int k0 = blockIdx.y * len, k1 = min(g.nsamp, k0 + len);
            unsigned thin = 0, emit = 0, inside = 0;
            for (int k = k0; k < k1; ++k) {
                const float t = ((float)k + 0.5f - half) * r.ds;
                const float py = fmaf(t, r.wy, r.pmy), pz = fmaf(t, r.wz, r.pmz);
                const SampleQ q = shade_sample<false>(s, ztab, r.px, py, pz, r.ds, 0);
                thin += q.K < kThinK ? 1u : 0u;
                emit += q.K > 0.0f ? 1u : 0u;
                inside += locate(s, r.px, py, pz).taper > 0.0f ? 1u : 0u;
            }
            if (thin) atomicAdd(&part[1], (unsigned long long)thin);
            if (emit) atomicAdd(&part[2], (unsigned long long)emit);
            if (inside) atomicAdd(&part[3], (unsigned long long)inside);
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 && part[threadIdx.x]) atomicAdd(counts + threadIdx.x, part[threadIdx.x]);
}

__global__ void zero_counts(unsigned long long *c) {
    if (threadIdx.x < 4) c[threadIdx.x] = 0ull;
}

} // namespace rt

using namespace rt;

extern "C" rt_status rt_render_census(const rt_problem *p, uint8_t *mask, int64_t *counts, void *stream) {
    rt_status st = validate(p);
    if (st != RT_OK) return st;
    if (!counts) return fail(RT_EINVAL, "counts is NULL");
    Geometry g;
    Shade s;
    st = build_launch(p, &g, &s);
    if (st != RT_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e;
    unsigned long long *d = (unsigned long long *)stream_workspace(hs, kWsCensus, 4 * sizeof(unsigned long long), &e);
    if (!d) return fail_hip(e, "census counters");
    // the shading needs the network's outputs when there is a network: count rays only
    const int shade = p->mlp ? 0 : 1;
    const int npix = p->cam.nx * p->cam.ny;
    int chunks = 1;
    while (shade && chunks < 64 && (long)((npix + 255) / 256) * chunks < 4096 && p->nsamp >= 16 * chunks) chunks *= 2;
    hipLaunchKernelGGL(zero_counts, dim3(1), dim3(64), 0, hs, d);
    hipLaunchKernelGGL(census, dim3((npix + 255) / 256, chunks), dim3(256), 0, hs, g, s, mask, d, shade);
    unsigned long long h[4] = {0, 0, 0, 0};
    if ((e = hipGetLastError()) == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return fail_hip(e, "census");
    counts[0] = (int64_t)h[0];
    counts[1] = (int64_t)h[0] * p->nsamp;
    counts[2] = shade ? (int64_t)h[1] : -1;
    counts[3] = shade ? (int64_t)h[2] : -1;
    counts[4] = shade ? (int64_t)h[3] : -1;
    return RT_OK;
}
