// rt_kernels.h -- device-side argument blocks and shared math of the ray
// march kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rt {

// channels carried in one launch's kernel arguments
constexpr int kLaunchChannels = 256;
// partition-function table: nodes uniform in log2 T over [log2 0.1, log2 1e4]
constexpr int kZTableNodes = 1024;
constexpr float kLog2E = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Per-launch geometry.  Per-ray set-up runs in double (once per ray), the
// samples themselves in float.
struct Geometry {
    double d_pix;            // pixel size [au]
    double cpa, spa;         // position-angle rotation
    double si, ci;           // sin / cos inclination
    double rc, zc;           // bounding cylinder radius and half height [au]
    int32_t nx, ny, nsamp;
    int32_t pad_;
};

// Fields and the channel-independent shading constants.
struct Shade {
    const float *ln_n, *temp, *vphi, *zlo, *zup;   // caller's arrays
    const float4 *ztab;      // [kZTableNodes-1] {Z_i, h Z'_i, Z_i+1, h Z'_i+1}
    int32_t nr, nz;
    float u_scale;           // u = (log2 rho - log2_rmin) * u_scale
    float log2_rmin;
    float inv_dzr;           // v = (|z| / rho) * inv_dzr
    float fnr, fnz;          // nr, nz as float
    float inv_w;             // mask argument = (z_s - |z|) * inv_w / rho  (log2e folded in)
    float zt_l2t0, zt_scale; // table index = (log2 T - zt_l2t0) * zt_scale
    float el_log2e;          // e^(-E_l/T) = exp2(-el_log2e / T)
    float theta;             // h nu0 / k [K]
    float c_s;               // intensity_scale * 2 h nu0^3 / c^2
    float c_k;               // x_co (h nu0/4pi) g_l B_lu (c/nu0) au / (sqrt(pi) 1e5) * log2e
    float c_alpha;           // alpha^2 [(km/s)^2] = T * c_alpha
    float sqrt_log2e;
    float vrot;              // sin i
    float vsys;              // systemic velocity [km/s]
    float thin_thr;          // dtau (log2 units) below which 1 - e^-dtau uses the series
};

struct Channels {
    int32_t n;               // channels in this launch
    int32_t pad_;
    float v[kLaunchChannels];
};

// ---------------------------------------------------------------- math
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float clampf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// e^x - 1 for 0 <= x: Taylor series through x^9/9! below 1/2 (truncation
// < 1e-8 relative), e^x - 1 above (relative error ~ 1 ulp / (1 - e^-x)).
__device__ __forceinline__ float expm1_pos(float x) {
    float p = 1.0f / 362880.0f;
    p = fmaf(p, x, 1.0f / 40320.0f);
    p = fmaf(p, x, 1.0f / 5040.0f);
    p = fmaf(p, x, 1.0f / 720.0f);
    p = fmaf(p, x, 1.0f / 120.0f);
    p = fmaf(p, x, 1.0f / 24.0f);
    p = fmaf(p, x, 1.0f / 6.0f);
    p = fmaf(p, x, 0.5f);
    p = fmaf(p, x, 1.0f);
    const float series = p * x;
    const float direct = fexp2(x * kLog2E) - 1.0f;
    return x < 0.5f ? series : direct;
}

// 1 - 2^-x for small x >= 0 (x in log2 units): series in y = x ln 2 through
// y^5 (first omitted term y^6/720).
__device__ __forceinline__ float one_minus_exp2_neg_series(float x) {
    constexpr float c1 = 0.6931471805599453f;             //  ln2
    constexpr float c2 = -0.2402265069591007f;            // -ln2^2/2
    constexpr float c3 = 0.05550410866482158f;            //  ln2^3/6
    constexpr float c4 = -0.009618129107628477f;          // -ln2^4/24
    constexpr float c5 = 0.0013333558146428443f;          //  ln2^5/120
    float p = fmaf(c5, x, c4);
    p = fmaf(p, x, c3);
    p = fmaf(p, x, c2);
    p = fmaf(p, x, c1);
    return p * x;
}

// Z(T) by cubic Hermite interpolation of the table in log2 T.
__device__ __forceinline__ float partition_fn(const Shade &s, float log2t) {
    float t = (log2t - s.zt_l2t0) * s.zt_scale;
    t = clampf(t, 0.0f, (float)(kZTableNodes - 1));
    int i = (int)t;
    i = i > kZTableNodes - 2 ? kZTableNodes - 2 : i;
    const float f = t - (float)i;
    const float4 n = s.ztab[i];
    const float g = 1.0f - f;
    const float h00 = (1.0f + 2.0f * f) * g * g;
    const float h10 = f * g * g;
    const float h01 = f * f * (3.0f - 2.0f * f);
    const float h11 = -f * f * g;
    return h00 * n.x + h10 * n.y + h01 * n.z + h11 * n.w;
}

} // namespace rt
