// rt_micro.hip -- register-only microbenchmarks of the instruction classes
// the ray march is made of (measurement aid, see include/rtcube_micro.h).
#include <hip/hip_runtime.h>

#include "../../include/rtcube_micro.h"
#include "rt_host.h"
#include "rt_kernels.h"

namespace rt {

constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(256) void micro(int64_t iters, float seed, float *sink) {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 0.001f * (threadIdx.x + c);
    const float a = 0.9999f + 1e-9f * seed, b = 1e-6f * seed;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (KIND == RT_MICRO_FMA) {
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
            } else if (KIND == RT_MICRO_EXP2) {
                x[c] = fexp2(-x[c]); x[c] = fexp2(-x[c]);
                x[c] = fexp2(-x[c]); x[c] = fexp2(-x[c]);
            } else if (KIND == RT_MICRO_RCP) {
                x[c] = frcp(x[c] + 1.0f); x[c] = frcp(x[c] + 1.0f);
                x[c] = frcp(x[c] + 1.0f); x[c] = frcp(x[c] + 1.0f);
            } else if (KIND == RT_MICRO_LOG2) {
                x[c] = flog2(x[c] + 2.0f); x[c] = flog2(x[c] + 2.0f);
                x[c] = flog2(x[c] + 2.0f); x[c] = flog2(x[c] + 2.0f);
            } else if (KIND == RT_MICRO_EXP_FMA) {
                x[c] = fexp2(-x[c]);
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (s == 1234.5f) sink[threadIdx.x] = s;
}

// The channel-loop body of the forward march on 32 channels held in
// registers, driven by a per-iteration sample (S, K, a, b) like the real
// kernel: THIN keeps K below the thin-sample threshold (series form), else
// above it (1 - 2^-x).
template <bool THIN>
__global__ __launch_bounds__(256) void micro_loop(int64_t iters, float seed, float *sink) {
    constexpr int CB = 32;
    float I[CB], Tr[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) { I[c] = 0.0f; Tr[c] = 1.0f; }
    SampleQ q;
    q.a = seed * (float)threadIdx.x;
    q.b = 1.2f + seed;
    q.K = THIN ? 0.5f * kThinK : 0.05f + seed;
    q.S = 1.0f + seed;
    for (int64_t it = 0; it < iters; ++it) {
        q.a += 0.001f;
        march_sample<CB, true>(I, Tr, q, [](int c) { return (float)(c - 16) * 0.1f; });
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < CB; ++c) s += I[c] + Tr[c];
    if (s == 1234.5f) sink[threadIdx.x] = s;
}

} // namespace rt

using namespace rt;

extern "C" int32_t rt_microbench(int32_t kind, int64_t iters, double *out) {
    if (!out || iters < 1) return fail(RT_EINVAL, "bad microbenchmark arguments");
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail_hip(e, "device query");
    float *sink = nullptr;
    e = hipMalloc(&sink, 256 * sizeof(float));
    if (e != hipSuccess) return fail_hip(e, "hipMalloc");
    const int blocks = ncu * 16;   // 16 waves of 64 per CU
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    double lane_ops = 0.0;
    const double lanes = (double)blocks * 256;
    for (int rep = 0; rep < 2; ++rep) {   // first pass warms up clocks
        (void)hipEventRecord(t0, 0);
        switch (kind) {
        case RT_MICRO_FMA: hipLaunchKernelGGL(micro<RT_MICRO_FMA>, dim3(blocks), dim3(256), 0, 0, iters, 0.5f, sink);
            lane_ops = lanes * iters * kChains * 4; break;
        case RT_MICRO_EXP2: hipLaunchKernelGGL(micro<RT_MICRO_EXP2>, dim3(blocks), dim3(256), 0, 0, iters, 0.5f, sink);
            lane_ops = lanes * iters * kChains * 4; break;
        case RT_MICRO_RCP: hipLaunchKernelGGL(micro<RT_MICRO_RCP>, dim3(blocks), dim3(256), 0, 0, iters, 0.5f, sink);
            lane_ops = lanes * iters * kChains * 4; break;
        case RT_MICRO_LOG2: hipLaunchKernelGGL(micro<RT_MICRO_LOG2>, dim3(blocks), dim3(256), 0, 0, iters, 0.5f, sink);
            lane_ops = lanes * iters * kChains * 4; break;
        case RT_MICRO_EXP_FMA: hipLaunchKernelGGL(micro<RT_MICRO_EXP_FMA>, dim3(blocks), dim3(256), 0, 0, iters, 0.5f, sink);
            lane_ops = lanes * iters * kChains * 5; break;
        case RT_MICRO_LOOP_PLAIN: hipLaunchKernelGGL(micro_loop<false>, dim3(blocks), dim3(256), 0, 0, iters, 0.5f, sink);
            lane_ops = lanes * iters * 32; break;
        case RT_MICRO_LOOP_THIN: hipLaunchKernelGGL(micro_loop<true>, dim3(blocks), dim3(256), 0, 0, iters, 0.5f, sink);
            lane_ops = lanes * iters * 32; break;
        default:
            (void)hipFree(sink);
            return fail(RT_EINVAL, "unknown microbenchmark %d", kind);
        }
        (void)hipEventRecord(t1, 0);
        e = hipEventSynchronize(t1);
        if (e != hipSuccess) break;
    }
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(sink);
    if (e != hipSuccess) return fail_hip(e, "microbenchmark");
    *out = lane_ops / (ms * 1e-3);
    return 0;
}
