// rt_host.h -- internal host helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/rtcube.h"
#include "rt_kernels.h"

namespace rt {

rt_status fail(rt_status st, const char *fmt, ...);
rt_status fail_hip(hipError_t e, const char *what);
rt_status validate(const rt_problem *p);
rt_status validate_view(const rt_line &l, const rt_camera &c, const rt_spectral &s, int32_t nsamp,
                        double intensity_scale, double max_incl_deg);
// Z(T) table of the line's levels on the current device (built once per level set)
rt_status partition_table(const rt_line &l, const float4 **out);
// the same table on the host: tab[kZTableNodes - 1]
void partition_table_host(const rt_line &l, float4 *tab);
// launch constants of a problem; ztab: a partition table already on the
// device (NULL: the library's cached table of the line)
rt_status build_launch(const rt_problem *p, Geometry *g, Shade *s, const float4 *ztab = nullptr);
int channel_block_for(int nch, long npix);
void forward_shape(int nch, long npix, int nsamp, int *cb, int *nsplit);
// channels per lane, lanes per pixel and samples per checkpoint segment (0:
// none) of the reverse march; cube: the march also forms the intensity (fused
// L2 loss or a requested cube)
void adjoint_shape(int nch, long npix, bool cube, int *cb, int *lanes, int *kseg);
// velocities v[n] uniformly spaced in groups of cb within blocks of G cb
// channels (lane m's = lane 0's + m shift)
bool group_shift(const double *v, int n, int G, int cb, double *shift);
bool thin_series();
int ckpt_segment_option();
int ray_split_option();
int channel_block_option();
int adjoint_block_option();
int adjoint_lanes_option();
bool grad_accum_double();

// Device scratch kept with a stream: the buffer of (current device, stream,
// slot) is grown on demand with stream-ordered allocation and reused by later
// calls on that stream, so steady-state calls allocate nothing.  Calls that
// share a stream must be issued from one host thread at a time.
void *stream_workspace(hipStream_t st, int slot, size_t bytes, hipError_t *err);
// bytes a workspace of `bytes` actually holds (the growth step rounds up)
size_t workspace_round(size_t bytes);
void release_stream_workspaces(hipStream_t st);
// return the current device's memory-pool blocks that nothing holds to the device
void trim_memory_pool();
// bytes the stream's workspaces hold
size_t stream_workspace_bytes(hipStream_t st);
constexpr int kWsAdjoint = 0, kWsGradAcc = 1, kWsChain = 2, kWsNeuralT = 3, kWsBeam = 4, kWsBeamCube = 5,
              kWsGradBatch = 6, kWsCensus = 7;
// default largest adjoint scratch (tape, checkpoints, cotangents) of one pass
// over a band of image rows; larger images are processed band by band
constexpr size_t kAdjointScratchCap = (size_t)8 << 30;
size_t adjoint_scratch_cap();
// bytes of adjoint scratch per pixel for nch channels and nsamp samples
size_t adjoint_bytes_per_pixel(int nch, long npix, int nsamp, bool cube);

rt_status render_cube_mlp(const rt_problem *p, float *cube, hipStream_t st);
// beam checks shared by rt_beam_convolve and the server's submit
rt_status validate_beam(const rt_beam &b);
// cube <- beam * cube through the stream's scratch (slot kWsBeamCube)
rt_status beam_in_place(float *cube, int nch, int ny, int nx, const rt_beam &b, hipStream_t st);
rt_status march_cube(const rt_problem *p, const Geometry &g, const Shade &s, float *cube, hipStream_t st);
// dl = dL/dcube; or dl == NULL and target != NULL: the cotangent of the L2
// loss sum (cube - target)^2, formed inside the reverse march from its own
// forward sweep (cube_opt then receives the cube)
// A fixed device region that replaces the library's allocations in an
// adjoint call: the partition table, the gradient accumulators and the band
// scratch are carved from it, and the image is processed in bands of rows
// whose scratch fits what is left.
struct FixedScratch {
    char *base;
    size_t bytes;
};
// bytes a FixedScratch must hold at least: table, accumulators and one row
size_t fixed_scratch_min_bytes(const rt_problem *p);
rt_status adjoint_core(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st,
                       const float4 *mlp_o, float4 *dO, const float *target = nullptr,
                       const FixedScratch *fx = nullptr);
rt_status adjoint_mlp(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st,
                      const float *target = nullptr);
rt_status adjoint_grid(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st,
                       const float *target = nullptr);
// sum (cube - target)^2 into loss (device double), after the cube is written
hipError_t launch_l2_value(const float *cube, const float *target, size_t n, double *loss, hipStream_t st);

} // namespace rt
