// rt_serve_grad.hip -- batched gradient requests of the render server.
//
// Several forward + L2 loss + adjoint requests (grid fields, uneven sizes)
// share one sequence of launches: the accumulators of every request are
// cleared, then three persistent launches run the adjoint's passes over the
// work items of all requests of the batch, each workgroup pulling the next
// item from a device counter:
//   tape   -- (request, 256-pixel tile, chunk of samples): the shading of
//             every sample to the request's tape;
//   march  -- (request, 64-pixel tile, slice of 4 x 8 channels): the
//             checkpoint-free reverse march with the intensity formed in the
//             march, writing the cube and the per-sample cotangents;
//   chain  -- (request, field pass, chunk of pixel-samples): the shading's
//             local derivatives, accumulated in LDS by a 1024-lane workgroup
//             and flushed once into the request's accumulators (float, or
//             double by option);
// then one launch writes every request's gradients (as float) and one its
// loss (summed in double).  A request's items are those of its own problem and its results go
// to its own buffers, so what it gets does not depend on the rest of the
// batch beyond the order of the atomic additions.
#include "rt_adjoint_dev.h"
#include "rt_host.h"
#include "rt_serve.h"

namespace rt {

static_assert(kGradLanes == 4 && kGradLaneCB == 8, "the batched reverse march is instantiated for 4 x 8 channels");

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

size_t grad_batch_scratch_bytes(int nch, long npix, int nsamp, long nr, long nz) {
    const size_t nblk = (size_t)(nch + kGradSlice - 1) / kGradSlice;
    return al256(sizeof(float4) * (size_t)nsamp * npix) + al256(sizeof(float4) * (size_t)npix) +
           al256(sizeof(float4) * nblk * nsamp * npix) + al256(sizeof(int2) * (size_t)npix) +
           al256(sizeof(double) * (size_t)(3 * nr * nz + 2 * nr));
}

void grad_batch_items(int nch, long npix, int nsamp, int nfp, uint32_t items[3], uint32_t *chunks) {
    const long nblk = (nch + kGradSlice - 1) / kGradSlice;
    items[0] = (uint32_t)(((npix + 255) / 256) * kGradTapeChunks);
    items[1] = (uint32_t)(((npix + 256 / kGradLanes - 1) / (256 / kGradLanes)) * nblk);
    *chunks = (uint32_t)std::max<size_t>(1, ((size_t)nsamp * npix + kGradChainChunk - 1) / kGradChainChunk);
    items[2] = (uint32_t)nfp * *chunks;
}

// LDS of the chain pass: one field of the grid and the two surface vectors
// (float), beside the partition table
constexpr size_t kGradChainLdsMax = 160 * 1024 - sizeof(float4) * (kZTableNodes - 1) - 1024;

static size_t chain_lds_bytes(int nr, int nz) {
    return 2 * (size_t)nr * sizeof(float) + (size_t)nr * nz * sizeof(float);
}

bool grad_batch_grid_fits(int nr, int nz) { return chain_lds_bytes(nr, nz) <= kGradChainLdsMax; }

// the request owning item `item` of pass `pass`: the last whose first item is <= item
__device__ __forceinline__ int owner(const GradDesc *__restrict__ descs, int nreq, int pass, uint32_t item) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].item0[pass] <= item) lo = mid; else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// a wave-uniform pointer kept in scalar registers
template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

// next item of a persistent launch, the same for the whole workgroup
__device__ __forceinline__ uint32_t next_item(uint32_t *counter, uint32_t *s_item) {
    __syncthreads();
    if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1u);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*s_item);
}

// the request's partition table into LDS when it is not the one already there
__device__ __forceinline__ void stage_table(const float4 *tab, float4 *lds, const float4 **s_tab) {
    if (*s_tab != tab) {     // uniform: every lane reads the same s_tab
        __syncthreads();
        for (int i = threadIdx.x; i < kZTableNodes - 1; i += 256) lds[i] = tab[i];
        __syncthreads();
        if (threadIdx.x == 0) *s_tab = tab;
    }
}

// accumulators of type A (float, or double with RT_OPT_GRAD_ACCUM 1) at the
// head of the request's double-sized accumulator region
template <typename A>
__global__ __launch_bounds__(256) void grad_zero(const GradDesc *__restrict__ descs) {
    const GradDesc &D = descs[blockIdx.y];
    const size_t n = 3 * (size_t)D.s.nr * D.s.nz + 2 * (size_t)D.s.nr;
    A *acc = (A *)D.acc;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) acc[i] = (A)0;
    // the tape's chunks merge the rays' spans into a cleared record
    const size_t np = (size_t)D.g.nx * D.g.ny;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < np; i += (size_t)gridDim.x * 256)
        D.span[i] = make_int2(0, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) *D.loss = 0.0;
}

__global__ __launch_bounds__(256) void grad_tape(const GradDesc *__restrict__ descs, int nreq, uint32_t nitems,
                                                 uint32_t *__restrict__ counter) {
    __shared__ float4 ztab[kZTableNodes - 1];
    __shared__ uint32_t s_item;
    __shared__ const float4 *s_tab;
    if (threadIdx.x == 0) s_tab = nullptr;
    for (;;) {
        const uint32_t item = next_item(counter, &s_item);
        if (item >= nitems) break;
        const GradDesc D = descs[owner(descs, nreq, 0, item)];
        stage_table(D.s.ztab, ztab, &s_tab);
        const uint32_t local = item - D.item0[0];
        const int tile = (int)(local / kGradTapeChunks), chunk = (int)(local % kGradTapeChunks);
        const int npix = D.g.nx * D.g.ny, pix = tile * 256 + (int)threadIdx.x;
        if (pix < npix) {
            const int len = (D.g.nsamp + kGradTapeChunks - 1) / kGradTapeChunks;
            const int k0 = chunk * len, k1 = min(D.g.nsamp, k0 + len);
            tape_pixel(D.g, D.s, ztab, pix, k0, k1, chunk == 0, D.tape, D.rays, D.span, true);
        }
    }
}

__global__ __launch_bounds__(256) void grad_march(const GradDesc *__restrict__ descs, int nreq, uint32_t nitems, uint32_t *__restrict__ counter) {
    constexpr int CB = kGradLaneCB, G = kGradLanes, PX = 256 / kGradLanes;
    __shared__ uint32_t s_item;
    for (;;) {
        const uint32_t item = next_item(counter, &s_item);
        if (item >= nitems) break;
        const GradDesc *D = descs + owner(descs, nreq, 1, item);
        const uint32_t local = item - __builtin_amdgcn_readfirstlane(D->item0[1]);
        const int nblk = __builtin_amdgcn_readfirstlane(D->nblk);
        const int tile = (int)(local / (uint32_t)nblk), blk = (int)(local % (uint32_t)nblk);
        const int npix = __builtin_amdgcn_readfirstlane(D->g.nx * D->g.ny);
        const int nsamp = __builtin_amdgcn_readfirstlane(D->g.nsamp);
        const int nch = __builtin_amdgcn_readfirstlane(D->nch);
        const float vshift = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(D->vshift)));
        const int g = (int)(threadIdx.x % G);
        const int pix = tile * PX + (int)threadIdx.x / G;
        const int c0 = (blk * G + g) * CB;
        if (pix < npix) {   // the lanes of a pixel take the branch together
            // lane 0's velocities of the slice (wave-uniform), lane g's offset
            // folded into a by the march
            const float *vch = uniform_ptr(D->vch) + blk * kGradSlice;
            auto vel = [&](int c) -> float { return vch[c]; };
            const int2 ks = span_of(uniform_ptr(D->span)[pix], nsamp);
            march_tau_pixel<CB, G, true, true, true>(pix, blk, g, c0, nch, nsamp, npix, npix, ks.y >= ks.x, vel,
                                                     uniform_ptr(D->tape), nullptr, uniform_ptr(D->target),
                                                     uniform_ptr(D->cot), uniform_ptr(D->cube), (float)g * vshift, ks);
        }
    }
}

// Chain pass: each item is one field pass over a contiguous chunk of one
// request's pixel-samples.  The workgroup (1024 lanes, one per CU) clears
// that field's grid in LDS, adds every sample's bilinear contributions there
// (and, in the request's first field pass, the two surfaces'),
// then flushes the nodes it touched into the request's accumulators (type A).
// Every pass sums the request's cotangent slices itself, so passes of one
// request may run at the same time.
template <typename A>
__global__ __launch_bounds__(kGradChainThreads) void grad_chain(const GradDesc *__restrict__ descs, int nreq,
                                                               uint32_t nitems, uint32_t *__restrict__ counter) {
    extern __shared__ float dyn[];    // [2 nr] surfaces, then [nr nz] field
    __shared__ float4 ztab[kZTableNodes - 1];
    __shared__ uint32_t s_item;
    __shared__ const float4 *s_tab;
    if (threadIdx.x == 0) s_tab = nullptr;
    for (;;) {
        const uint32_t item = next_item(counter, &s_item);
        if (item >= nitems) break;
        const GradDesc &D = descs[owner(descs, nreq, 2, item)];   // uniform: scalar loads
        if (s_tab != D.s.ztab) {
            __syncthreads();
            for (int i = threadIdx.x; i < kZTableNodes - 1; i += kGradChainThreads) ztab[i] = D.s.ztab[i];
            __syncthreads();
            if (threadIdx.x == 0) s_tab = D.s.ztab;
        }
        const uint32_t local = item - D.item0[2];
        const int fp = (int)(local / D.chunks), chunk = (int)(local % D.chunks);
        const int field = D.fields[fp];
        const bool surf = fp == 0 && (D.out[3] || D.out[4]);
        const int nr = D.s.nr, nn = D.s.nr * D.s.nz;
        float *sl = dyn;
        float *fl = dyn + 2 * nr;
        if (surf)
            for (int i = threadIdx.x; i < 2 * nr; i += kGradChainThreads) sl[i] = 0.0f;
        if (field < 3)
            for (int i = threadIdx.x; i < nn; i += kGradChainThreads) fl[i] = 0.0f;
        __syncthreads();
        const int npix = D.g.nx * D.g.ny, nsamp = D.g.nsamp;
        const size_t total = (size_t)nsamp * npix;
        const size_t len = (total + D.chunks - 1) / D.chunks;
        const size_t i0 = (size_t)chunk * len, i1 = min(total, i0 + len);
        for (size_t idx = i0 + threadIdx.x; idx < i1; idx += kGradChainThreads) {
            const int k = (int)(idx / npix);
            const int pix = (int)(idx - (size_t)k * npix);
            // samples outside the ray's run of K > 0 have no cotangents
            const int2 ks = span_of(D.span[pix], nsamp);
            if (k < ks.x || k > ks.y) continue;
            const float4 rr = D.rays[pix];
            float4 c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            for (int b = 0; b < D.nblk; ++b) {
                const float4 t = D.cot[((size_t)b * nsamp + k) * npix + pix];
                c.x += t.x; c.y += t.y; c.z += t.z; c.w += t.w;
            }
            if (!(rr.w > 0.0f) || (c.x == 0.0f && c.y == 0.0f && c.z == 0.0f && c.w == 0.0f)) continue;
            const ChainTerms t = chain_terms(D.g, D.s, ztab, rr, c, k, pix);
            const float fu = t.fu, fv = t.fv;
            if (field < 3) {
                const float gv = field == 0 ? t.gn : (field == 1 ? t.gT : t.gV);
                if (gv != 0.0f) {
                    const int n00 = t.i0 * D.s.nz + t.j0, n10 = n00 + D.s.nz;
                    atomicAdd(fl + n00, gv * (1.0f - fu) * (1.0f - fv));
                    atomicAdd(fl + n00 + 1, gv * (1.0f - fu) * fv);
                    atomicAdd(fl + n10, gv * fu * (1.0f - fv));
                    atomicAdd(fl + n10 + 1, gv * fu * fv);
                }
            }
            if (surf) {
                if (t.gzl != 0.0f) {
                    atomicAdd(sl + t.i0, t.gzl * (1.0f - fu));
                    atomicAdd(sl + t.i0 + 1, t.gzl * fu);
                }
                if (t.gzu != 0.0f) {
                    atomicAdd(sl + nr + t.i0, t.gzu * (1.0f - fu));
                    atomicAdd(sl + nr + t.i0 + 1, t.gzu * fu);
                }
            }
        }
        __syncthreads();
        if (field < 3) {
            A *dst = (A *)D.acc + (size_t)field * nn;
            for (int i = threadIdx.x; i < nn; i += kGradChainThreads)
                if (fl[i] != 0.0f) atomicAdd(dst + i, (A)fl[i]);
        }
        if (surf) {
            A *zl = (A *)D.acc + 3 * (size_t)nn, *zu = zl + nr;
            for (int i = threadIdx.x; i < nr; i += kGradChainThreads) {
                if (D.out[3] && sl[i] != 0.0f) atomicAdd(zl + i, (A)sl[i]);
                if (D.out[4] && sl[nr + i] != 0.0f) atomicAdd(zu + i, (A)sl[nr + i]);
            }
        }
    }
}

// blockIdx.y = request: its accumulators to the caller's FP32 outputs
template <typename A>
__global__ __launch_bounds__(256) void grad_finish(const GradDesc *__restrict__ descs) {
    const GradDesc &D = descs[blockIdx.y];
    const A *acc = (const A *)D.acc;
    const size_t nn = (size_t)D.s.nr * D.s.nz, nr = (size_t)D.s.nr;
    const size_t off[5] = {0, nn, 2 * nn, 3 * nn, 3 * nn + nr};
    const size_t len[5] = {nn, nn, nn, nr, nr};
    for (int f = 0; f < 5; ++f) {
        float *o = D.out[f];
        if (!o) continue;
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < len[f]; i += (size_t)gridDim.x * 256)
            o[i] = (float)acc[off[f] + i];
    }
}

// blockIdx.y = request: L = sum (cube - target)^2 (block sums, FP64 atomics)
__global__ __launch_bounds__(256) void grad_loss(const GradDesc *__restrict__ descs) {
    const GradDesc &D = descs[blockIdx.y];
    __shared__ double part[256];
    const size_t n = (size_t)D.nch * D.g.nx * D.g.ny;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double r = (double)D.cube[i] - (double)D.target[i];
        acc += r * r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(D.loss, part[0]);
}

__global__ void zero_counters(uint32_t *c) {
    if (threadIdx.x < 3) c[threadIdx.x] = 0u;
}

template <typename A>
static hipError_t grad_batch_t(const GradDesc *descs, const GradDesc *host_descs, int nreq, const uint32_t nitems[3],
                              uint32_t *counters, int nwg, hipStream_t st) {
    size_t max_acc = 0, max_cube = 0;
    for (int i = 0; i < nreq; ++i) {
        const GradDesc &D = host_descs[i];
        max_acc = std::max(max_acc, 3 * (size_t)D.s.nr * D.s.nz + 2 * (size_t)D.s.nr);
        max_cube = std::max(max_cube, (size_t)D.nch * D.g.nx * D.g.ny);
    }
    hipLaunchKernelGGL(zero_counters, dim3(1), dim3(64), 0, st, counters);
    hipLaunchKernelGGL(grad_zero<A>, dim3((unsigned)std::min<size_t>((max_acc + 255) / 256, 64), nreq), dim3(256), 0, st,
                       descs);
    hipLaunchKernelGGL(grad_tape, dim3(nwg), dim3(256), 0, st, descs, nreq, nitems[0], counters);
    hipLaunchKernelGGL(grad_march, dim3(nwg), dim3(256), 0, st, descs, nreq, nitems[1], counters + 1);
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    size_t lds = 0;
    for (int i = 0; i < nreq; ++i) lds = std::max(lds, chain_lds_bytes(host_descs[i].s.nr, host_descs[i].s.nz));
    if ((e = hipFuncSetAttribute((const void *)grad_chain<A>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(grad_chain<A>, dim3(std::max<int>(1, std::min<int>(ncu, (int)nitems[2]))), dim3(kGradChainThreads),
                       lds, st, descs, nreq, nitems[2], counters + 2);
    hipLaunchKernelGGL(grad_finish<A>, dim3((unsigned)std::min<size_t>((max_acc + 255) / 256, 64), nreq), dim3(256), 0,
                       st, descs);
    hipLaunchKernelGGL(grad_loss, dim3((unsigned)std::min<size_t>((max_cube + 255) / 256, 128), nreq), dim3(256), 0,
                       st, descs);
    return hipGetLastError();
}

hipError_t launch_grad_batch(const GradDesc *descs, const GradDesc *host_descs, int nreq, const uint32_t nitems[3],
                             uint32_t *counters, int nwg, hipStream_t st) {
    return grad_accum_double() ? grad_batch_t<double>(descs, host_descs, nreq, nitems, counters, nwg, st)
                               : grad_batch_t<float>(descs, host_descs, nreq, nitems, counters, nwg, st);
}

} // namespace rt
