// rt_adjoint.h -- launch interface of the adjoint passes (internal).
#pragma once
#include "rt_kernels.h"

namespace rt {

struct GradOut {
    float *ln_n, *temp, *vphi, *zlo, *zup;
};
// double accumulators of the scatter (NULL = not requested)
struct GradAcc {
    double *ln_n, *temp, *vphi, *zlo, *zup;
};

hipError_t zero_async(float *p, size_t n, hipStream_t st);
hipError_t zero_async_d(double *p, size_t n, hipStream_t st);
hipError_t to_float_async(const double *src, float *dst, size_t n, hipStream_t st);
hipError_t copy_float_async(const float *src, float *dst, size_t n, hipStream_t st);
// tape [nsamp][npix], ray records [npix], and each ray's run of samples with
// K > 0 as span [npix] = (nsamp - first, last + 1), (0, 0) when it has none;
// span_only: the tape holds valid entries only inside each ray's run (when
// one chunk covers a ray), which the checkpoint-free march is built for
hipError_t launch_adj_tape(const Geometry &g, const Shade &s, float4 *tape, float4 *rays, int2 *span, bool span_only,
                           hipStream_t st);
// reverse march.  kseg 0: the checkpoint-free march with `lanes` (1, 2 or 4)
// lanes per pixel over each ray's span alone (lanes = 4 needs the velocities
// uniformly spaced in groups of cb: lane g's = lane 0's + g shift); kseg > 0:
// the checkpointed march (one lane per pixel)
hipError_t launch_adj_march(int cb, int kseg, int lanes, int nsamp, int npix, int plane, const Channels &ch,
                            float shift, const float4 *tape, const int2 *span, const float *dl, const float *target,
                            float *ckpt, float4 *cot, float *cube_out, hipStream_t st);
// chain passes; both read the cotangents of the samples in each ray's span
hipError_t launch_adj_chain(const Geometry &g, const Shade &s, const float4 *rays, const int2 *span, const float4 *cot,
                            int nblk, const GradAcc &go, float4 *dO, hipStream_t st);
bool chain_lds_fits(int nr, int nz);
hipError_t launch_adj_chain_lds(const Geometry &g, const Shade &s, const float4 *rays, const int2 *span, float4 *cot,
                                int nblk, const GradAcc &go, float4 *dO, hipStream_t st);

} // namespace rt
