// rt_mlp.hip -- neural CO layer on the matrix cores.
//
// Network: 16 Fourier frequencies on the two normalised grid coordinates of a
// sample (64 features) -> 4 SiLU layers of width 128 -> 3 outputs.  It is
// evaluated at every (pixel, sample) point of the render, point index
// m = k * npix + pix.
//
// mlp_fwd<T, P>: a workgroup of 8 waves evaluates a tile of P points.  Layer
//   outputs are 16 x 16 MFMA tiles: wave w owns output columns [16w, 16w+16)
//   for every 16-point row tile; activations go through LDS between layers
//   (row-major, the A-operand layout); weights are read as B operands
//   straight from the prepared layout.  Bias + SiLU are fused on the
//   accumulators.  T = bf16 (v_mfma_f32_16x16x32_bf16) or float
//   (v_mfma_f32_16x16x4f32), FP32 accumulation in both.
// mlp_bwd<T, P>: persistent workgroups; each recomputes the forward of its
//   tiles (keeping pre-activations and transposed activations in LDS),
//   backpropagates dL/do through the layers on MFMA, and accumulates the
//   weight gradient of the whole network in its own MFMA accumulators
//   (wave w owns rows [16w, 16w+16) of every hidden layer's dW), flushing
//   them with atomics once at the end.
#include <algorithm>
#include <cmath>

#include "rt_mlp.h"

namespace rt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kW = 128;     // hidden width
constexpr int kF = 64;      // features
constexpr int kLayerIn[4] = {kF, kW, kW, kW};

template <typename T> struct MM;
template <> struct MM<__bf16> {
    static constexpr int KCH = 32;   // K per MFMA
    static constexpr int EPL = 8;    // elements per lane per fragment
    typedef bf16x8 frag;
    static __device__ __forceinline__ frag load(const __bf16 *p) { return *(const bf16x8 *)p; }
    static __device__ __forceinline__ floatx4 mfma(frag a, frag b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct MM<float> {
    static constexpr int KCH = 4;
    static constexpr int EPL = 1;
    typedef float frag;
    static __device__ __forceinline__ frag load(const float *p) { return *p; }
    static __device__ __forceinline__ floatx4 mfma(frag a, frag b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

__device__ __forceinline__ float silu(float z) { return z * sigmoidf_(z); }
__device__ __forceinline__ float silu_d(float z) {
    const float s = sigmoidf_(z);
    return s * (1.0f + z * (1.0f - s));
}

// Normalised grid coordinates of point m (same positions as the march).
__device__ __forceinline__ void point_coords(const Geometry &g, const Shade &s, size_t m, float *rh, float *zh) {
    const int npix = g.nx * g.ny;
    const int k = (int)(m / npix);
    const int pix = (int)(m - (size_t)k * npix);
    const RaySetup r = ray_setup(g, pix % g.nx, pix / g.nx);
    const float t = ((float)k + 0.5f - 0.5f * (float)g.nsamp) * r.ds;
    const Locus L = locate(s, r.px, fmaf(t, r.wy, r.pmy), fmaf(t, r.wz, r.pmz));
    *rh = clampf(L.u, -1.0f, s.fnr) / (s.fnr - 1.0f);
    *zh = clampf(L.v, 0.0f, s.fnz) / (s.fnz - 1.0f);
}

// sin(pi f c), cos(pi f c) with the phase reduced in double
template <typename T>
__device__ __forceinline__ void write_features(T *row, const MlpDev &w, float rh, float zh) {
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
        double xr = (double)w.freq[q] * (double)rh;
        double xz = (double)w.freq[q] * (double)zh;
        xr -= 2.0 * floor(0.5 * xr);
        xz -= 2.0 * floor(0.5 * xz);
        float sr, cr, sz, cz;
        sincospif((float)xr, &sr, &cr);
        sincospif((float)xz, &sz, &cz);
        row[q] = (T)sr;
        row[16 + q] = (T)cr;
        row[32 + q] = (T)sz;
        row[48 + q] = (T)cz;
    }
}

template <typename T> struct Pad { static constexpr int v = 16 / (int)sizeof(T); };

// LDS layout of one tile (P points).
template <typename T, int P, bool BWD> struct alignas(16) TileLds {
    static constexpr int PD = Pad<T>::v;
    static constexpr int S0 = kF + PD, S1 = kW + PD, ST = P + PD;
    T h0[P * S0];
    T h[4][P * S1];                          // post-activations of the hidden layers
    T z[BWD ? 4 : 1][BWD ? P * S1 : 1];      // pre-activations
    T hT0[BWD ? kF * ST : 1];                // transposed features
    T hT[BWD ? 3 : 1][BWD ? kW * ST : 1];    // transposed activations of layers 1..3
    T d[BWD ? P * S1 : 1];                   // dL/dz of the current layer
    T dT[BWD ? kW * ST : 1];
    float d5[BWD ? P * 3 : 1];
};

// Forward of one tile: features of points m0..m0+P-1, hidden layers, and
// (when out != NULL) the 3 outputs.  Caller syncs before reusing LDS.
template <typename T, int P, bool BWD>
__device__ void tile_forward(TileLds<T, P, BWD> &L, const Geometry &g, const Shade &s, const MlpDev &w, size_t m0,
                             size_t M, float4 *out) {
    typedef MM<T> mm;
    constexpr int S0 = TileLds<T, P, BWD>::S0, S1 = TileLds<T, P, BWD>::S1, ST = TileLds<T, P, BWD>::ST;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < P) {
        const size_t m = m0 + tid;
        float rh = 0.0f, zh = 0.0f;
        if (m < M) point_coords(g, s, m, &rh, &zh);
        write_features<T>(L.h0 + tid * S0, w, rh, zh);
    }
    __syncthreads();
    if (BWD) {
        for (int i = tid; i < P * kF; i += 512) {
            const int mm_ = i / kF, k = i - mm_ * kF;
            L.hT0[k * ST + mm_] = L.h0[mm_ * S0 + k];
        }
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int K = kLayerIn[l];
        const T *hin = l == 0 ? L.h0 : L.h[l - 1];
        const int SI = l == 0 ? S0 : S1;
        const T *W = (const T *)w.W[l];
        const int n = 16 * wv + (lane & 15);
        const float bias = w.b[l][n];
#pragma unroll
        for (int mt = 0; mt < P / 16; ++mt) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int kc = 0; kc < K / mm::KCH; ++kc) {
                const int k0 = kc * mm::KCH + (lane >> 4) * mm::EPL;
                acc = mm::mfma(mm::load(hin + (mt * 16 + (lane & 15)) * SI + k0), mm::load(W + n * K + k0), acc);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = mt * 16 + 4 * (lane >> 4) + i;
                const float zv = acc[i] + bias;
                const float hv = silu(zv);
                L.h[l][m * S1 + n] = (T)hv;
                if (BWD) {
                    L.z[l][m * S1 + n] = (T)zv;
                    if (l < 3) L.hT[l][n * ST + m] = (T)hv;
                }
            }
        }
        __syncthreads();
    }
    if (out && tid < P) {
        const size_t m = m0 + tid;
        float o0 = w.b5[0], o1 = w.b5[1], o2 = w.b5[2];
        const T *hr = L.h[3] + tid * S1;
        for (int k = 0; k < kW; ++k) {
            const float hv = (float)hr[k];
            o0 = fmaf(hv, w.W5[k], o0);
            o1 = fmaf(hv, w.W5[kW + k], o1);
            o2 = fmaf(hv, w.W5[2 * kW + k], o2);
        }
        if (m < M) out[m] = make_float4(o0, o1, o2, 0.0f);
    }
}

template <typename T, int P>
__global__ __launch_bounds__(512) void mlp_fwd(Geometry g, Shade s, MlpDev w, size_t M, float4 *__restrict__ out) {
    __shared__ TileLds<T, P, false> L;
    tile_forward<T, P, false>(L, g, s, w, (size_t)blockIdx.x * P, M, out);
}

template <typename T, int P>
__global__ __launch_bounds__(512) void mlp_bwd(Geometry g, Shade s, MlpDev w, size_t M, const float4 *__restrict__ dO,
                                               float *__restrict__ dW) {
    typedef MM<T> mm;
    __shared__ TileLds<T, P, true> L;
    constexpr int S1 = TileLds<T, P, true>::S1, ST = TileLds<T, P, true>::ST;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // weight-gradient accumulators: wave wv owns rows [16 wv, 16 wv + 16) of
    // every hidden layer; k-tiles of 16 columns
    floatx4 a0[kF / 16], a1[kW / 16], a2[kW / 16], a3[kW / 16];
#pragma unroll
    for (int i = 0; i < kF / 16; ++i) a0[i] = floatx4{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < kW / 16; ++i) { a1[i] = floatx4{0, 0, 0, 0}; a2[i] = a1[i]; a3[i] = a1[i]; }
    float db[4] = {0, 0, 0, 0};   // bias gradients, thread tid < 128 owns row tid
    float dw5 = 0.0f, db5 = 0.0f; // thread tid < 384 owns W5[tid / 128][tid % 128]; tid < 3 owns b5
    const size_t ntiles = (M + P - 1) / P;
    for (size_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const size_t m0 = tile * P;
        tile_forward<T, P, true>(L, g, s, w, m0, M, nullptr);
        // output layer
        if (tid < P) {
            const size_t m = m0 + tid;
            const float4 d = m < M ? dO[m] : make_float4(0, 0, 0, 0);
            L.d5[tid * 3 + 0] = d.x; L.d5[tid * 3 + 1] = d.y; L.d5[tid * 3 + 2] = d.z;
        }
        __syncthreads();
        if (tid < 3 * kW) {
            const int j = tid / kW, k = tid - j * kW;
            float acc = 0.0f;
            for (int m = 0; m < P; ++m) acc = fmaf(L.d5[m * 3 + j], (float)L.h[3][m * S1 + k], acc);
            dw5 += acc;
        }
        if (tid < 3) {
            float acc = 0.0f;
            for (int m = 0; m < P; ++m) acc += L.d5[m * 3 + tid];
            db5 += acc;
        }
        for (int i = tid; i < P * kW; i += 512) {
            const int m = i / kW, n = i - m * kW;
            const float gz = L.d5[m * 3] * w.W5[n] + L.d5[m * 3 + 1] * w.W5[kW + n] + L.d5[m * 3 + 2] * w.W5[2 * kW + n];
            const T dv = (T)(gz * silu_d((float)L.z[3][m * S1 + n]));
            L.d[m * S1 + n] = dv;
            L.dT[n * ST + m] = dv;
        }
        __syncthreads();
#pragma unroll
        for (int l = 3; l >= 0; --l) {
            // dW_l[n][k] += sum_m d[m][n] h_{l-1}[m][k]   (rows n of this wave)
            const int K = kLayerIn[l];
            const T *hT = l == 0 ? L.hT0 : L.hT[l - 1];
            const T *arow = L.dT + (16 * wv + (lane & 15)) * ST;
#pragma unroll
            for (int kt = 0; kt < K / 16; ++kt) {
                floatx4 acc = l == 0 ? a0[kt % (kF / 16)] : (l == 1 ? a1[kt] : (l == 2 ? a2[kt] : a3[kt]));
                const T *brow = hT + (16 * kt + (lane & 15)) * ST;
                for (int mc = 0; mc < P / mm::KCH; ++mc) {
                    const int k0 = mc * mm::KCH + (lane >> 4) * mm::EPL;
                    acc = mm::mfma(mm::load(arow + k0), mm::load(brow + k0), acc);
                }
                if (l == 0) a0[kt % (kF / 16)] = acc;
                else if (l == 1) a1[kt] = acc;
                else if (l == 2) a2[kt] = acc;
                else a3[kt] = acc;
            }
            if (tid < kW) {
                float acc = 0.0f;
                for (int m = 0; m < P; ++m) acc += (float)L.dT[tid * ST + m];
                db[l] += acc;
            }
            if (l == 0) break;
            // g_{l-1}[m][k] = sum_n d[m][n] W_l[n][k]   (columns k of this wave)
            floatx4 gacc[P / 16];
            const T *WT = (const T *)w.WT[l];
            const int k = 16 * wv + (lane & 15);
#pragma unroll
            for (int mt = 0; mt < P / 16; ++mt) {
                floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int nc = 0; nc < kW / mm::KCH; ++nc) {
                    const int n0 = nc * mm::KCH + (lane >> 4) * mm::EPL;
                    acc = mm::mfma(mm::load(L.d + (mt * 16 + (lane & 15)) * S1 + n0), mm::load(WT + k * kW + n0), acc);
                }
                gacc[mt] = acc;
            }
            __syncthreads();   // every wave is done reading d / dT of layer l
#pragma unroll
            for (int mt = 0; mt < P / 16; ++mt) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = mt * 16 + 4 * (lane >> 4) + i;
                    const T dv = (T)(gacc[mt][i] * silu_d((float)L.z[l - 1][m * S1 + k]));
                    L.d[m * S1 + k] = dv;
                    L.dT[k * ST + m] = dv;
                }
            }
            __syncthreads();
        }
        __syncthreads();
    }
    // flush: flat layout per layer W [out][in] then b [out]
    const int n_base = 16 * wv + 4 * (lane >> 4);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int K = kLayerIn[l];
        float *Wg = dW + w.off[l];
        for (int kt = 0; kt < K / 16; ++kt) {
            const floatx4 acc = l == 0 ? a0[kt % (kF / 16)] : (l == 1 ? a1[kt] : (l == 2 ? a2[kt] : a3[kt]));
            const int k = 16 * kt + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (acc[i] != 0.0f) atomicAdd(Wg + (n_base + i) * K + k, acc[i]);
        }
        if (tid < kW && db[l] != 0.0f) atomicAdd(dW + w.off[l] + kW * K + tid, db[l]);
    }
    if (tid < 3 * kW && dw5 != 0.0f) atomicAdd(dW + w.off[4] + tid, dw5);
    if (tid < 3 && db5 != 0.0f) atomicAdd(dW + w.off[4] + 3 * kW + tid, db5);
}

// Prepared weights from the flat float32 layout (W [out][in], b [out] per
// layer): row-major and transposed copies in T, float biases, float output layer.
template <typename T>
__global__ void mlp_prep(const float *__restrict__ flat, MlpDev w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int l = 0; l < 4; ++l) {
        const int K = kLayerIn[l];
        if (i < kW * K) {
            const int n = i / K, k = i - n * K;
            const float v = flat[w.off[l] + i];
            ((T *)w.W[l])[i] = (T)v;
            ((T *)w.WT[l])[k * kW + n] = (T)v;
        }
        if (i < kW) ((float *)w.b[l])[i] = flat[w.off[l] + kW * K + i];
    }
    if (i < 3 * kW) ((float *)w.W5)[i] = flat[w.off[4] + i];
    if (i < 3) ((float *)w.b5)[i] = flat[w.off[4] + 3 * kW + i];
}

size_t mlp_prep_bytes(int precision) {
    const size_t es = precision == RT_MLP_BF16 ? 2 : 4;
    size_t n = 0;
    for (int l = 0; l < 4; ++l) n += 2 * es * (size_t)kW * kLayerIn[l] + 4 * kW;
    return n + 4 * (3 * kW + 3) + 256 * 8;
}

hipError_t mlp_prepare(const float *flat, int precision, void *buf, MlpDev *w, hipStream_t st) {
    const size_t es = precision == RT_MLP_BF16 ? 2 : 4;
    char *p = (char *)buf;
    auto take = [&](size_t b) { char *q = p; p += (b + 255) / 256 * 256; return q; };
    int off = 0;
    for (int l = 0; l < 4; ++l) {
        w->off[l] = off;
        off += kW * kLayerIn[l] + kW;
        w->W[l] = take(es * kW * kLayerIn[l]);
        w->WT[l] = take(es * kW * kLayerIn[l]);
        w->b[l] = (const float *)take(4 * kW);
    }
    w->off[4] = off;
    w->W5 = (const float *)take(4 * 3 * kW);
    w->b5 = (const float *)take(4 * 3);
    for (int q = 0; q < 16; ++q) w->freq[q] = (float)std::exp2(3.0 * q / 15.0);
    const int n = kW * kW;
    if (precision == RT_MLP_BF16)
        hipLaunchKernelGGL(mlp_prep<__bf16>, dim3((n + 255) / 256), dim3(256), 0, st, flat, *w);
    else
        hipLaunchKernelGGL(mlp_prep<float>, dim3((n + 255) / 256), dim3(256), 0, st, flat, *w);
    return hipGetLastError();
}

hipError_t mlp_forward(const Geometry &g, const Shade &s, const MlpDev &w, int precision, size_t M, float4 *out,
                       hipStream_t st) {
    if (precision == RT_MLP_BF16) {
        constexpr int P = 64;
        hipLaunchKernelGGL((mlp_fwd<__bf16, P>), dim3((unsigned)((M + P - 1) / P)), dim3(512), 0, st, g, s, w, M, out);
    } else {
        constexpr int P = 32;
        hipLaunchKernelGGL((mlp_fwd<float, P>), dim3((unsigned)((M + P - 1) / P)), dim3(512), 0, st, g, s, w, M, out);
    }
    return hipGetLastError();
}

hipError_t mlp_backward(const Geometry &g, const Shade &s, const MlpDev &w, int precision, size_t M,
                        const float4 *dO, float *dW, hipStream_t st) {
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (precision == RT_MLP_BF16) {
        constexpr int P = 32;
        const size_t ntiles = (M + P - 1) / P;
        const unsigned grid = (unsigned)std::min<size_t>(ntiles, (size_t)ncu);
        hipLaunchKernelGGL((mlp_bwd<__bf16, P>), dim3(grid), dim3(512), 0, st, g, s, w, M, dO, dW);
    } else {
        constexpr int P = 16;
        const size_t ntiles = (M + P - 1) / P;
        const unsigned grid = (unsigned)std::min<size_t>(ntiles, (size_t)ncu);
        hipLaunchKernelGGL((mlp_bwd<float, P>), dim3(grid), dim3(512), 0, st, g, s, w, M, dO, dW);
    }
    return hipGetLastError();
}

} // namespace rt
