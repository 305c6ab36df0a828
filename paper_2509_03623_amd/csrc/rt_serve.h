// rt_serve.h -- device side of the render server (internal).
#pragma once
#include <algorithm>

#include "rt_kernels.h"

namespace rt {

// workgroups (256 lanes each) per compute unit of the persistent forward
// launch; an item covers kServeTile x kServeTile pixels with kServeSplit
// lanes per pixel
constexpr int kServeWorkgroupsPerCU = 4;
constexpr int kServeTile = 8;
constexpr int kServeSplit = 4;

// One request of a persistent forward batch.
struct ServeDesc {
    Geometry g;
    Shade s;
    const float *vch;     // channel velocities, padded to a multiple of 16
    float *cube;          // [nch][ny][nx]
    int32_t nch, nblk, tiles_x;   // channel blocks of 16, item tiles across
    uint32_t item0;       // first work item of this request in the batch
    const float *target;  // L = sum (cube - target)^2 into *loss (NULL: no loss)
    double *loss;
};

hipError_t launch_serve_fwd(const ServeDesc *descs, int nreq, uint32_t nitems, uint32_t *counter, int nwg,
                            hipStream_t st);
hipError_t launch_l2_loss(const float *cube, const float *target, float *dl, size_t n, double *loss, hipStream_t st);
// L of every request of a batch that has a target (descs on the device, losses zeroed first)
hipError_t launch_l2_batch(const ServeDesc *descs, int nreq, double *losses, size_t max_n, hipStream_t st);

} // namespace rt
