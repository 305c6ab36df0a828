// rt_mlp_host.cpp -- render and adjoint entry points with the neural CO
// layer: prepare the weights, evaluate the network at every (pixel, sample)
// point, march with its outputs, and (adjoint) backpropagate into the weights.
#include <hip/hip_runtime.h>

#include "rt_adjoint.h"
#include "rt_host.h"
#include "rt_mlp.h"

namespace rt {

namespace {
struct Scratch {
    void *p = nullptr;
    hipStream_t st = nullptr;
    ~Scratch() { if (p) (void)hipFreeAsync(p, st); }
};
} // namespace

// prepared weights + network outputs for every point of the render
static rt_status mlp_setup(const rt_problem *p, Geometry *geo, Shade *sh, MlpDev *w, Scratch *ws, float4 **out,
                           size_t extra_point_bytes, void **extra, hipStream_t st) {
    rt_status rs = build_launch(p, geo, sh);
    if (rs != RT_OK) return rs;
    const int prec = p->mlp->precision;
    const size_t M = (size_t)p->cam.nx * p->cam.ny * p->nsamp;
    const size_t prep = (mlp_prep_bytes(prec) + 255) / 256 * 256;
    const size_t ob = sizeof(float4) * M;
    // with the per-point extra (the backward's dL/do) comes the backward's pass list
    const size_t list_b = extra ? mlp_backward_list_bytes(M) : 0;
    ws->st = st;
    hipError_t e = hipMallocAsync(&ws->p, prep + ob + extra_point_bytes * M + list_b, st);
    if (e != hipSuccess) { ws->p = nullptr; return fail_hip(e, "network scratch"); }
    *out = (float4 *)((char *)ws->p + prep);
    if (extra) *extra = (char *)ws->p + prep + ob;
    if ((e = mlp_prepare(p->mlp->weights, prec, ws->p, w, st)) != hipSuccess) return fail_hip(e, "network weights");
    if ((e = mlp_forward(*geo, *sh, *w, prec, M, *out, st)) != hipSuccess) return fail_hip(e, "network forward");
    return RT_OK;
}

rt_status render_cube_mlp(const rt_problem *p, float *cube, hipStream_t st) {
    Geometry geo;
    Shade sh;
    MlpDev w;
    Scratch ws;
    float4 *o = nullptr;
    rt_status rs = mlp_setup(p, &geo, &sh, &w, &ws, &o, 0, nullptr, st);
    if (rs != RT_OK) return rs;
    sh.mlp_o = o;
    return march_cube(p, geo, sh, cube, st);
}

rt_status adjoint_mlp(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st,
                      const float *target) {
    if (p->spec.nch > kLaunchChannels)
        return fail(RT_EINVAL, "the neural CO layer adjoint takes at most %d channels per call", kLaunchChannels);
    // the backward lists its points with 32-bit indices
    if ((uint64_t)p->cam.nx * p->cam.ny * p->nsamp >= 0xFFFFFFFFull)
        return fail(RT_EINVAL, "the neural CO layer adjoint takes fewer than 2^32 - 1 pixel-samples per call");
    Geometry geo;
    Shade sh;
    MlpDev w;
    Scratch ws;
    float4 *o = nullptr;
    void *dO = nullptr;
    rt_status rs = mlp_setup(p, &geo, &sh, &w, &ws, &o, sizeof(float4), &dO, st);
    if (rs != RT_OK) return rs;
    rs = adjoint_core(p, dl, g, cube_opt, st, o, (float4 *)dO, target);
    if (rs != RT_OK) return rs;
    const size_t M = (size_t)p->cam.nx * p->cam.ny * p->nsamp;
    if (g->d_mlp) {
        hipError_t e = zero_async(g->d_mlp, RT_MLP_PARAMS, st);
        if (e == hipSuccess)
            e = mlp_backward(geo, sh, w, p->mlp->precision, M, (const float4 *)dO,
                             (uint32_t *)((float4 *)dO + M), g->d_mlp, st);
        if (e != hipSuccess) return fail_hip(e, "network backward");
    }
    return RT_OK;
}

} // namespace rt
