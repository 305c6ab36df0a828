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

// Batched gradient requests (forward + L2 loss + adjoint of grid fields):
// the reverse march runs kGradLanes lanes per pixel of kGradLaneCB channels
// each, so a cotangent slice covers kGradSlice channels (the requests'
// channels uniformly spaced in groups of kGradLaneCB: lane g's velocities are
// lane 0's plus g vshift); tape items split each tile's samples into
// kGradTapeChunks chunks; chain items are (field pass, chunk of about
// kGradChainChunk pixel-samples) of one request, accumulated by a 1024-lane
// workgroup in LDS and flushed once.
constexpr int kGradSlice = 32;
constexpr int kGradLanes = 4;
constexpr int kGradLaneCB = kGradSlice / kGradLanes;
constexpr int kGradTapeChunks = 4;
constexpr int kGradChainThreads = 1024;
constexpr long kGradChainChunk = 64L * kGradChainThreads;

struct GradDesc {
    Geometry g;
    Shade s;
    const float *vch;          // channel velocities, padded to a multiple of kGradSlice
    const float *target;       // [nch][ny][nx]
    float *cube;               // [nch][ny][nx] (written by the reverse march)
    float4 *tape, *rays, *cot; // scratch: [nsamp][npix], [npix], [nblk][nsamp][npix]
    int2 *span;                // scratch [npix]: each ray's run of samples with K > 0
                               // as (nsamp - first, last + 1), (0, 0) for none
    double *acc;               // accumulators [3 nr nz + 2 nr]: ln n, T, v_phi, z_lo, z_up (sized for
                               // double; float ones, the default, use the head of it)
    float *out[5];             // caller's gradient outputs in the same order (NULL: not requested)
    double *loss;              // L of this request
    int32_t nch, nblk;         // channels, cotangent slices (of kGradSlice channels)
    float vshift;              // velocity offset between adjacent lanes of a pixel (kGradLaneCB dv)
    uint32_t item0[3];         // first item of this request in the tape, march and chain passes
    int32_t nfp;               // chain field passes (>= 1; the first also takes the surfaces)
    int32_t fields[3];         // field of each pass: 0 ln n, 1 T, 2 v_phi, 3 none (surfaces only)
    uint32_t chunks;           // chain chunks per field pass
};

// scratch bytes of one batched gradient request (tape, rays, cotangents, spans, accumulators)
size_t grad_batch_scratch_bytes(int nch, long npix, int nsamp, long nr, long nz);
// items of one request in the three passes (nfp chain field passes)
void grad_batch_items(int nch, long npix, int nsamp, int nfp, uint32_t items[3], uint32_t *chunks);
// whether a grid's chain accumulators fit the LDS of one workgroup
bool grad_batch_grid_fits(int nr, int nz);
// zero -> tape -> reverse march -> chain -> outputs and losses, on one stream;
// counters: 3 device words
hipError_t launch_grad_batch(const GradDesc *descs, const GradDesc *host_descs, int nreq, const uint32_t nitems[3],
                             uint32_t *counters, int nwg, hipStream_t st);
hipError_t launch_l2_loss(const float *cube, const float *target, float *dl, size_t n, double *loss, hipStream_t st);
// L of every request of a batch that has a target (descs on the device, losses zeroed first)
hipError_t launch_l2_batch(const ServeDesc *descs, int nreq, double *losses, size_t max_n, hipStream_t st);

} // namespace rt
