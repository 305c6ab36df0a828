// rt_host.h -- internal host helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/rtcube.h"
#include "rt_kernels.h"

namespace rt {

rt_status fail(rt_status st, const char *fmt, ...);
rt_status fail_hip(hipError_t e, const char *what);
rt_status validate(const rt_problem *p);
rt_status build_launch(const rt_problem *p, Geometry *g, Shade *s);
int channel_block_for(int nch, long npix);
void forward_shape(int nch, long npix, int nsamp, int *cb, int *nsplit);
bool thin_series();
int ckpt_segment_option();
bool grad_accum_double();

rt_status render_cube_mlp(const rt_problem *p, float *cube, hipStream_t st);
rt_status march_cube(const rt_problem *p, const Geometry &g, const Shade &s, float *cube, hipStream_t st);
rt_status adjoint_core(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st,
                       const float4 *mlp_o, float4 *dO);
rt_status adjoint_mlp(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st);
rt_status adjoint_grid(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st);

} // namespace rt
