/*
 * rtcube_micro.h -- measurement aid of librtcube: register-only
 * microbenchmarks that pin the issue rates behind the renderer's roofline on
 * the GPU in use (not part of the rendering API).
 */
#ifndef RTCUBE_MICRO_H
#define RTCUBE_MICRO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
    RT_MICRO_FMA = 0,          /* v_fma_f32, independent chains */
    RT_MICRO_EXP2 = 1,         /* v_exp_f32 */
    RT_MICRO_RCP = 2,          /* v_rcp_f32 */
    RT_MICRO_LOG2 = 3,         /* v_log_f32 */
    RT_MICRO_LOOP_PLAIN = 4,   /* the march's channel-loop body on a thick sample (1 - e^-x direct) */
    RT_MICRO_LOOP_THIN = 5,    /* the same body on an optically thin sample (series form) */
    RT_MICRO_EXP_FMA = 6       /* one v_exp_f32 per four v_fma_f32 */
};

/* Runs microbenchmark `kind` on the current device (synchronously) and
 * stores its rate in *out: lane-instructions per second for kinds 0-3 and 6
 * (all instructions counted), ray-samples per second for kinds 4-5.
 * Returns 0 or a negative rt_status. */
int32_t rt_microbench(int32_t kind, int64_t iters, double *out);

#ifdef __cplusplus
}
#endif
#endif
