// rt_launch.h -- host-side entry points of the kernels (internal).
#pragma once
#include "rt_kernels.h"

namespace rt {

hipError_t launch_forward(const Geometry &g, const Shade &s, const Channels &ch, float *cube, int cb, bool thin,
                          int nsplit, hipStream_t st);
// paired-lane march of 64-channel blocks whose upper 32 velocities are the
// lower 32 plus `shift`
hipError_t launch_forward_pair(const Geometry &g, const Shade &s, const Channels &ch, float *cube, bool thin,
                               float shift, hipStream_t st);

} // namespace rt
