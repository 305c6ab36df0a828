// rt_launch.h -- host-side entry points of the kernels (internal).
#pragma once
#include "rt_kernels.h"

namespace rt {

hipError_t launch_forward(const Geometry &g, const Shade &s, const Channels &ch, float *cube, int cb, bool thin,
                          int nsplit, hipStream_t st);
// grouped-lane march of 64-channel blocks (lanes = 2 or 4 per pixel), lane
// h's channel velocities being lane 0's plus h `shift`
hipError_t launch_forward_group(const Geometry &g, const Shade &s, const Channels &ch, float *cube, bool thin,
                                int lanes, float shift, hipStream_t st);

} // namespace rt
