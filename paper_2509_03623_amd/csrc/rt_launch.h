// rt_launch.h -- host-side entry points of the kernels (internal).
#pragma once
#include "rt_kernels.h"

namespace rt {

hipError_t launch_forward(const Geometry &g, const Shade &s, const Channels &ch, float *cube, int cb, bool thin,
                          int nsplit, hipStream_t st);

} // namespace rt
