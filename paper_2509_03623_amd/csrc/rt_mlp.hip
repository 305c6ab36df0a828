// rt_mlp.hip -- neural CO layer on the matrix cores.
//
// Network: 16 Fourier frequencies on the two normalised grid coordinates of a
// sample (64 features) -> 4 SiLU layers of width 128 -> 3 outputs.  It is
// evaluated at every (pixel, sample) point of the render, point index
// m = k * npix + pix.
//
// The BF16 path runs mlp_fwd_rr and mlp_bwd_rr; the FP32 reference path runs
// mlp_fwd<float> and mlp_bwd<float>.
//
// mlp_fwd<T, P>: a workgroup of 8 waves evaluates a tile of P points.  Layer
//   outputs are 16 x 16 MFMA tiles: wave w owns output columns [16w, 16w+16)
//   for every 16-point row tile; activations go through LDS between layers
//   (row-major, the A-operand layout); weights are read as B operands
//   straight from the prepared layout.  Bias + SiLU are fused on the
//   accumulators.  T = bf16 (v_mfma_f32_16x16x32_bf16) or float
//   (v_mfma_f32_16x16x4f32), FP32 accumulation in both.
// mlp_fwd_rr (BF16): persistent workgroups holding all hidden weights in LDS;
//   each wave evaluates 64 points at a time with the transposed product
//   Z^T = W H^T, output neurons as MFMA rows and points as columns.  The
//   accumulator of a 16-neuron output tile leaves every lane with 4
//   consecutive neurons of one point; two such tiles are exactly the 8
//   operand values a lane supplies for one 32-deep K chunk of the next layer,
//   once that layer's input order is permuted to match (done when the
//   weights are prepared).  Activations therefore never leave registers; the
//   output layer is evaluated in FP32 on the VALU and reduced across the
//   four lane groups by shuffles.
// mlp_bwd_rr (BF16): see its definition below.
// mlp_bwd<T, P>: persistent workgroups; each recomputes the forward of its
//   tiles (keeping pre-activations and transposed activations in LDS),
//   backpropagates dL/do through the layers on MFMA, and accumulates the
//   weight gradient of the whole network in its own MFMA accumulators
//   (wave w owns rows [16w, 16w+16) of every hidden layer's dW), flushing
//   them with atomics once at the end.
#include <algorithm>
#include <cmath>

#include "rt_adjoint.h"
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

// Phase f c reduced to (-2, 2) in float: the product is split exactly into
// hi + lo with an FMA (Ogita, Rump and Oishi's TwoProduct), hi loses its even
// integer part exactly (|hi| < 2^23), and lo is added back with one rounding,
// so the reduced phase is the exact one rounded once.
__device__ __forceinline__ float phase2(float f, float c) {
    const float hi = f * c;
    const float lo = fmaf(f, c, -hi);
    return (hi - 2.0f * floorf(0.5f * hi)) + lo;
}

// sin(pi f c), cos(pi f c)
template <typename T>
__device__ __forceinline__ void write_features(T *row, const MlpDev &w, float rh, float zh) {
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
        float sr, cr, sz, cz;
        sincospif(phase2(w.freq[q], rh), &sr, &cr);
        sincospif(phase2(w.freq[q], zh), &sz, &cz);
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

// ---------------------------------------------------------------- register-resident BF16 forward
constexpr int kRrRow0 = kF + 8;        // padded row of layer 0 (bf16 elements)
constexpr int kRrRow = kW + 8;         // padded row of layers 1..3
// 16-point column tiles per wave and lanes per workgroup (one workgroup per
// CU, the weights filling most of its LDS); 4 x 512 measured fastest of
// 2 x 1024, 2 x 768 and 4 x 512, and the same as 3 x 512 (which spills no
// registers where 4 x 512 spills 31: the spills cost nothing measurable)
constexpr int kRrTiles = 4;
constexpr int kRrThreads = 512;
constexpr size_t kRrWeightElems = (size_t)kW * kRrRow0 + 3 * (size_t)kW * kRrRow;
constexpr size_t kRrLds = kRrWeightElems * 2 + 4 * (4 * kW) + 4 * (3 * kW) + 16;

// input slot s of a 32-deep K chunk -> neuron of the previous layer: lane
// group g holds slots 8g..8g+7 = neurons 4g..4g+3 of the chunk's first
// 16-neuron output tile and 4g..4g+3 of its second
__host__ __device__ constexpr int rr_perm(int s) {
    return (s & ~31) + 16 * ((s & 7) >> 2) + 4 * ((s >> 3) & 3) + (s & 3);
}

// Layer 0 is scaled by log2(e) so that its pre-activation comes out as
// log2(e) z; layers 1..3 take log2(e) SiLU(z) as input and need no scale.
__global__ void mlp_prep_rr(const float *__restrict__ flat, MlpDev w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    __bf16 *Wr = (__bf16 *)w.Wr;
    if (i < kW * kRrRow0) {
        const int o = i / kRrRow0, k = i - o * kRrRow0;
        Wr[i] = (__bf16)(k < kF ? kLog2E * flat[w.off[0] + o * kF + k] : 0.0f);
    }
    __bf16 *WrT = (__bf16 *)w.WrT;
    for (int l = 1; l < 4; ++l) {
        if (i < kW * kRrRow) {
            const int o = i / kRrRow, k = i - o * kRrRow;
            Wr[(size_t)kW * kRrRow0 + (size_t)(l - 1) * kW * kRrRow + i] =
                (__bf16)(k < kW ? flat[w.off[l] + o * kW + rr_perm(k)] : 0.0f);
            // transposed: row = input neuron o, column = output slot k
            WrT[(size_t)(l - 1) * kW * kRrRow + i] = (__bf16)(k < kW ? flat[w.off[l] + rr_perm(k) * kW + o] : 0.0f);
        }
    }
}

// One hidden layer of the register-resident forward for the NP column tiles
// of a wave: z' = W h' + b' (the weights and biases carry the log2(e) scale
// of the prepared layout, so z' = log2(e) z), h' = z' sigma(z) -- i.e.
// log2(e) SiLU(z), the scale being absorbed by the next layer's prepared
// weights.  The accumulators start from the biases.  The last layer feeds
// the FP32 output layer instead of the next operands.
template <int NP>
__device__ __forceinline__ void rr_layer(const bf16x8 (&hin)[4][NP], bf16x8 (&hout)[4][NP], float (&o)[3][NP],
                                         const __bf16 *sW, const float *sB, const float *sW5, int l, int lg, int lc,
                                         bool last) {
    typedef MM<__bf16> mm;
    const int nk = l == 0 ? kF / 32 : kW / 32;
    const int row = l == 0 ? kRrRow0 : kRrRow;
    const __bf16 *Wl = sW + (l == 0 ? 0 : (size_t)kW * kRrRow0 + (size_t)(l - 1) * kW * kRrRow);
    const float *bl = sB + l * kW;
#pragma unroll
    for (int cp = 0; cp < 4; ++cp) {           // output tiles 2cp, 2cp+1
        floatx4 acc[2][NP];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const floatx4 b4 = *(const floatx4 *)(bl + 32 * cp + 16 * h + 4 * lg);
#pragma unroll
            for (int tp = 0; tp < NP; ++tp) acc[h][tp] = b4;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= nk) break;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bf16x8 a = *(const bf16x8 *)(Wl + (size_t)(32 * cp + 16 * h + lc) * row + 32 * c + 8 * lg);
#pragma unroll
                for (int tp = 0; tp < NP; ++tp) acc[h][tp] = mm::mfma(a, hin[c][tp], acc[h][tp]);
            }
        }
        if (!last) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int tp = 0; tp < NP; ++tp)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float z = acc[h][tp][i];
                        hout[cp][tp][4 * h + i] = (__bf16)(z * frcp(1.0f + fexp2(-z)));
                    }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int n = 32 * cp + 16 * h + 4 * lg;
                const floatx4 w0 = *(const floatx4 *)(sW5 + n), w1 = *(const floatx4 *)(sW5 + kW + n),
                              w2 = *(const floatx4 *)(sW5 + 2 * kW + n);
#pragma unroll
                for (int tp = 0; tp < NP; ++tp)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float z = acc[h][tp][i];
                        const float hv = z * frcp(1.0f + fexp2(-z));
                        o[0][tp] = fmaf(hv, w0[i], o[0][tp]);
                        o[1][tp] = fmaf(hv, w1[i], o[1][tp]);
                        o[2][tp] = fmaf(hv, w2[i], o[2][tp]);
                    }
            }
        }
    }
}

template <int NP, int NT>
__global__ __launch_bounds__(NT) void mlp_fwd_rr(Geometry g, Shade s, MlpDev w, size_t M, float4 *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char rr_lds[];
    __bf16 *sW = (__bf16 *)rr_lds;                                  // layer 0, then layers 1..3
    float *sB = (float *)(rr_lds + kRrWeightElems * 2);             // [4][128]
    float *sW5 = sB + 4 * kW;                                       // [3][128]
    float *sB5 = sW5 + 3 * kW;                                      // [3]
    constexpr int PTS = NT / 64 * NP * 16;                          // points per workgroup pass
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lg = lane >> 4, lc = lane & 15;
    {
        const uint4 *src = (const uint4 *)w.Wr;
        uint4 *dst = (uint4 *)sW;
        for (size_t i = tid; i < kRrWeightElems / 8; i += NT) dst[i] = src[i];
        for (int i = tid; i < 4 * kW; i += NT) sB[i] = kLog2E * w.b[i / kW][i % kW];
        for (int i = tid; i < 3 * kW; i += NT) sW5[i] = kLn2 * w.W5[i];
        if (tid < 3) sB5[tid] = w.b5[tid];
    }
    __syncthreads();
    typedef MM<__bf16> mm;
    for (size_t base = (size_t)blockIdx.x * PTS; base < M; base += (size_t)gridDim.x * PTS) {
        const size_t mw = base + (size_t)wv * (NP * 16);     // this wave's points
        float rh = 0.0f, zh = 0.0f;
        if (lane < NP * 16 && mw + lane < M) point_coords(g, s, mw + lane, &rh, &zh);
        // layer-0 operands: features of chunk c (0: r, 1: z); lane group g
        // supplies slots 8g..8g+7 = sin (g < 2) or cos (g >= 2) of
        // frequencies 8 (g & 1) .. 8 (g & 1) + 7.  Lanes g and g ^ 2 share
        // the work: each evaluates four frequencies (hardware sine and cosine
        // of the phase reduced to one period) and passes the partner the half
        // it needs.
        bf16x8 hin[4][NP];
        const int fb = 8 * (lg & 1) + (lg < 2 ? 0 : 4);
#pragma unroll
        for (int tp = 0; tp < NP; ++tp) {
            const float cr = __shfl(rh, tp * 16 + lc), cz = __shfl(zh, tp * 16 + lc);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float own[4], sent[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // sin(pi f x) = sin(2 pi t) with t = (f x mod 2) / 2 in [0, 1)
                    const float x = w.freq[fb + q] * (c == 0 ? cr : cz);
                    const float t = 0.5f * (x - 2.0f * floorf(0.5f * x));
                    const float sv = __builtin_amdgcn_sinf(t), cv = __builtin_amdgcn_cosf(t);
                    own[q] = lg < 2 ? sv : cv;
                    sent[q] = lg < 2 ? cv : sv;
                }
                bf16x8 f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float r = __shfl_xor(sent[q], 32);
                    f[q] = (__bf16)(lg < 2 ? own[q] : r);
                    f[4 + q] = (__bf16)(lg < 2 ? r : own[q]);
                }
                hin[c][tp] = f;
            }
        }
        float o[3][NP];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int tp = 0; tp < NP; ++tp) o[j][tp] = 0.0f;
        bf16x8 hb[4][NP];
        // layers in pairs, activations ping-ponging between hin and hb
#pragma unroll 1
        for (int lp = 0; lp < 2; ++lp) {
            rr_layer<NP>(hin, hb, o, sW, sB, sW5, 2 * lp, lg, lc, false);
            rr_layer<NP>(hb, hin, o, sW, sB, sW5, 2 * lp + 1, lg, lc, lp == 1);
        }
        // sum the four lane groups' partial outputs; group 0 writes
#pragma unroll
        for (int tp = 0; tp < NP; ++tp) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                o[j][tp] += __shfl_xor(o[j][tp], 16);
                o[j][tp] += __shfl_xor(o[j][tp], 32);
            }
            const size_t m = mw + (size_t)tp * 16 + lc;
            if (lg == 0 && m < M) out[m] = make_float4(o[0][tp] + sB5[0], o[1][tp] + sB5[1], o[2][tp] + sB5[2], 0.0f);
        }
    }
}

// ---------------------------------------------------------------- register-resident BF16 backward
// mlp_bwd_rr: one workgroup of four waves per CU, each wave with the full
// register file of its SIMD.  A wave takes 16 points per pass (the workgroup
// 64): it recomputes the forward with the transposed product (weights read
// as A operands from LDS, where the workgroup stages each layer's weights
// from L2: one copy per pass for the four waves, written by loads that go
// to LDS directly and are issued one stage ahead into a free buffer -- the
// forward's layers alternate between the weight buffer and the point-major
// rows, which the forward does not use; the backward's transposed weights
// are issued before the weight-gradient products that precede them -- so
// their latency overlaps the matrix work), keeping z' of every layer as BF16;
// walks back through the layers (dL/dh' of the layer below by the product
// with the transposed weights, the SiLU derivative recomputed from z'); and
// for the weight gradient, which sums over points, writes dL/dz' and h' of
// the pass into LDS as point-major rows, so that after a barrier each wave
// accumulates its own slice of every layer's gradient (32 output rows of the
// hidden layers, two 16-column tiles of the output layer) in MFMA
// accumulators over all 64 points.  Bias gradients are row sums of the same
// LDS rows.  Everything is flushed with atomics once, at the end.
constexpr int kBrPts = 64;                 // points per workgroup pass
// global-memory views (the pass loop launders the weight pointers, which
// would otherwise turn their loads into flat loads)
typedef const __attribute__((address_space(1))) __bf16 gbf16;
typedef const __attribute__((address_space(1))) bf16x8 gbf16x8;
constexpr int kBrStride = kBrPts + 8;      // LDS row of the point-major buffers (bf16)

__device__ __forceinline__ void br_features(bf16x8 (&feat)[2], const MlpDev &w, float cr, float cz, int lg) {
    const int fb = 8 * (lg & 1) + (lg < 2 ? 0 : 4);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        float own[4], sent[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float x = w.freq[fb + q] * (c == 0 ? cr : cz);
            const float t = 0.5f * (x - 2.0f * floorf(0.5f * x));
            const float sv = __builtin_amdgcn_sinf(t), cv = __builtin_amdgcn_cosf(t);
            own[q] = lg < 2 ? sv : cv;
            sent[q] = lg < 2 ? cv : sv;
        }
        bf16x8 f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float r = __shfl_xor(sent[q], 32);
            f[q] = (__bf16)(lg < 2 ? own[q] : r);
            f[4 + q] = (__bf16)(lg < 2 ? r : own[q]);
        }
        feat[c] = f;
    }
}

// h' = z' sigma(z) and dL/dz' = dL/dh' SiLU'(z) of one neuron, z = ln2 z'
__device__ __forceinline__ void br_act_grad(__bf16 zq16, float dh, bf16x8 &hp, bf16x8 &dz, int e) {
    const float zq = (float)zq16;
    const float sg = frcp(1.0f + fexp2(-zq));
    const float z = kLn2 * zq;
    hp[e] = (__bf16)(zq * sg);
    dz[e] = (__bf16)(dh * (sg * (1.0f + z * (1.0f - sg))));
}

// point-major write of 32 accumulator-layout values (neurons 16t + 4lg + i,
// t = 2cp + h, element 4h + i of pair cp) of the lane's point
__device__ __forceinline__ void br_write_rows(__bf16 *X, const bf16x8 (&v)[4], int lg, int col) {
#pragma unroll
    for (int cp = 0; cp < 4; ++cp)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) X[(32 * cp + 16 * h + 4 * lg + i) * kBrStride + col] = v[cp][4 * h + i];
}

// dW slice of one hidden layer: rows [32 wv, 32 wv + 32) of XD against the
// NI 16-row tiles of XH, over the 64 points
template <int NI>
__device__ __forceinline__ void br_dw(floatx4 (&acc)[2][NI], const __bf16 *XD, const __bf16 *XH, int wv, int lg,
                                      int lc) {
    typedef MM<__bf16> mm;
#pragma unroll
    for (int kc = 0; kc < kBrPts / 32; ++kc) {
        const bf16x8 a0 = *(const bf16x8 *)(XD + (32 * wv + lc) * kBrStride + 32 * kc + 8 * lg);
        const bf16x8 a1 = *(const bf16x8 *)(XD + (32 * wv + 16 + lc) * kBrStride + 32 * kc + 8 * lg);
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            const bf16x8 b = *(const bf16x8 *)(XH + (16 * it + lc) * kBrStride + 32 * kc + 8 * lg);
            acc[0][it] = mm::mfma(a0, b, acc[0][it]);
            acc[1][it] = mm::mfma(a1, b, acc[1][it]);
        }
    }
}

// sum over the 64 points of LDS row r (two lanes per row, 32 points each);
// two values per instruction, as a dot product with (1, 1)
__device__ __forceinline__ float br_rowsum(const __bf16 *X, int r, int half) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 one = {(__bf16)1.0f, (__bf16)1.0f};
    float sum = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bf16x8 v = *(const bf16x8 *)(X + r * kBrStride + 32 * half + 8 * q);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x2 p = {v[2 * j], v[2 * j + 1]};
            sum = __builtin_amdgcn_fdot2_f32_bf16(p, one, sum, false);
        }
    }
    return sum + __shfl_xor(sum, 1);
}

// copy n bf16 elements (a multiple of 8) of one layer's prepared weights
// from global memory into the workgroup's staging buffer (256 lanes): global
// loads that write LDS directly (16 B per lane, lane i of a wave to the
// wave's base + 16 i), so the copy holds no registers; every load is waited
// for (br_wait) before the barrier that precedes the first read
__device__ __forceinline__ void br_issue(__bf16 *dst, const gbf16 *src, int n, int tid) {
    typedef __attribute__((address_space(3))) void lds_void;
    typedef const __attribute__((address_space(1))) void g_void;
    const int nchunk = n / 8, wv = tid >> 6, lane = tid & 63;
    // (kept apart from the surrounding matrix code: interleaved with it, the
    // address arithmetic lengthens live ranges into spills)
    __builtin_amdgcn_sched_barrier(0);
    for (int c0 = 64 * wv; c0 < nchunk; c0 += 256) {
        const int c = c0 + lane;
        if (c < nchunk) __builtin_amdgcn_global_load_lds((g_void *)(src + 8 * c), (lds_void *)(dst + 8 * c0), 16, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void br_wait() { __builtin_amdgcn_s_waitcnt(0); }

// The points with any dL/do != 0, in order, for mlp_bwd_rr.  dL/do = 0 at a
// point (no opacity there) makes every layer's dL/dz' zero: the point adds
// nothing to any gradient, so the backward takes the others only, packed 64
// to a pass.  Three launches over kLiveChunks chunks of the points: the
// count of each chunk, a scan of the counts, then each chunk writing its
// points' indices (1024 consecutive points at a time, each lane's place from
// a ballot within its wave and the waves' counts in LDS).  list: [0] the
// number of points, [1 ...] their indices; then the chunks' counts and
// offsets.
constexpr int kLiveChunks = 4096;

__device__ __forceinline__ bool live_point(const float4 *dO, size_t m) {
    const float4 d = dO[m];
    return d.x != 0.0f || d.y != 0.0f || d.z != 0.0f;
}

__global__ __launch_bounds__(1024) void mlp_live_count(const float4 *__restrict__ dO, size_t M, size_t chunk,
                                                       uint32_t *__restrict__ counts) {
    __shared__ uint32_t tot;
    if (threadIdx.x == 0) tot = 0u;
    __syncthreads();
    const size_t b0 = (size_t)blockIdx.x * chunk, b1 = min(M, b0 + chunk);
    uint32_t n = 0;
    for (size_t i = b0 + threadIdx.x; i < b1; i += 1024) n += live_point(dO, i) ? 1u : 0u;
    if (n) atomicAdd(&tot, n);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// exclusive offsets of nb <= 4 * 1024 counts (one workgroup) and their total into list[0]
__global__ __launch_bounds__(1024) void mlp_live_scan(const uint32_t *__restrict__ counts, int nb,
                                                      uint32_t *__restrict__ offsets, uint32_t *__restrict__ list) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    uint32_t c[4], n = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        c[j] = 4 * t + j < nb ? counts[4 * t + j] : 0u;
        n += c[j];
    }
    part[t] = n;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t o = part[t] - n;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (4 * t + j < nb) offsets[4 * t + j] = o;
        o += c[j];
    }
    if (t == 1023) list[0] = part[1023];
}

__global__ __launch_bounds__(1024) void mlp_live_write(const float4 *__restrict__ dO, size_t M, size_t chunk,
                                                       const uint32_t *__restrict__ offsets,
                                                       uint32_t *__restrict__ list) {
    __shared__ uint32_t wsum[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const size_t b0 = (size_t)blockIdx.x * chunk, b1 = min(M, b0 + chunk);
    uint32_t done = offsets[blockIdx.x];   // the same in every lane
    for (size_t c0 = b0; c0 < b1; c0 += 1024) {
        const size_t i = c0 + t;
        const bool f = i < b1 && live_point(dO, i);
        const uint64_t mk = __ballot(f);
        if (lane == 0) wsum[wv] = (uint32_t)__popcll(mk);
        __syncthreads();
        uint32_t off = done, tot = 0;
        for (uint32_t j = 0; j < 16; ++j) {
            const uint32_t n = wsum[j];
            off += j < wv ? n : 0u;
            tot += n;
        }
        if (f) list[1 + off + (uint32_t)__popcll(mk & ((1ull << lane) - 1ull))] = (uint32_t)i;
        done += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void mlp_bwd_rr(
    Geometry g, Shade s, MlpDev w, size_t M, const float4 *__restrict__ dO, const uint32_t *__restrict__ list,
    float *__restrict__ dW) {
    typedef MM<__bf16> mm;
    // point-major rows of the backward: dL/dz' (or dL/do) rows x points, then
    // h' (or features) rows x points; in the forward, layers 1 and 3's weights
    __shared__ __attribute__((aligned(16))) __bf16 XU[2 * kW * kBrStride];
    static_assert(2 * kW * kBrStride >= kW * kRrRow, "a hidden layer's weights fit the row buffers");
    __bf16 *const XD = XU;
    __bf16 *const XH = XU + kW * kBrStride;
    __shared__ __attribute__((aligned(16))) float sB[4 * kW];
    __shared__ __attribute__((aligned(16))) float sW5[3 * kW];
    // lane-private parking of z' (4 layers x 4 operand packs) and the two
    // feature packs between the forward and the backward of a pass
    __shared__ bf16x8 ZP[18][256];
    // one layer's weights (forward) or transposed weights (backward)
    __shared__ __attribute__((aligned(16))) __bf16 SW[kW * kRrRow];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lg = lane >> 4, lc = lane & 15;
    for (int i = tid; i < 4 * kW; i += 256) sB[i] = kLog2E * w.b[i / kW][i % kW];
    for (int i = tid; i < 3 * kW; i += 256) sW5[i] = kLn2 * w.W5[i];
    floatx4 g0[2][4], g1[2][8], g2[2][8], g3[2][8], g4[2][1];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) g0[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < 8; ++b) { g1[a][b] = g0[a][0]; g2[a][b] = g0[a][0]; g3[a][b] = g0[a][0]; }
        g4[a][0] = g0[a][0];
    }
    float db0 = 0.0f, db1 = 0.0f, db2 = 0.0f, db3 = 0.0f, db5 = 0.0f;
    const int brow = 32 * wv + (lane >> 1), bhalf = lane & 1;     // bias row of this lane
    const int col = 16 * wv + lc;                                 // this lane's point within the pass
    // layer 0's weights for the first pass (each pass stages the next's)
    br_issue(SW, (const gbf16 *)(uint64_t)w.Wr, kW * kRrRow0, tid);
    br_wait();
    __syncthreads();
    // the points with any dL/do != 0, listed in order (list[0] of them), 64
    // to a pass
    const uint32_t npts = list[0];
    const uint32_t npass = (npts + kBrPts - 1) / kBrPts;
    for (uint32_t ip = blockIdx.x; ip < npass; ip += gridDim.x) {
        const uint32_t base = ip * kBrPts;
        // the weight operands are the same every pass: hide that from the
        // compiler, or it keeps all 208 fragments in registers across passes
        uint64_t wr_u = (uint64_t)w.Wr, wrt_u = (uint64_t)w.WrT;
        asm volatile("" : "+s"(wr_u), "+s"(wrt_u));
        const gbf16 *Wr = (const gbf16 *)wr_u;
        const gbf16 *WrT = (const gbf16 *)wrt_u;
        const size_t m = base + col < npts ? (size_t)list[1 + base + col] : M;   // M: no point
        float rh = 0.0f, zh = 0.0f;
        if (lane < 16 && m < M) point_coords(g, s, m, &rh, &zh);
        bf16x8 hin[4];
        {
            bf16x8 feat[2];
            br_features(feat, w, __shfl(rh, lc), __shfl(zh, lc), lg);
            ZP[16][tid] = feat[0];
            ZP[17][tid] = feat[1];
            hin[0] = feat[0];
            hin[1] = feat[1];
        }
        // ---- forward, parking z' of every layer
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int nk = l == 0 ? kF / 32 : kW / 32;
            const int row = l == 0 ? kRrRow0 : kRrRow;
            // layer l's weights are in place; the next stage goes into the
            // other buffer, free since the barrier that ended layer l - 1:
            // layer l + 1's weights, or after layer 3 the transposed weights
            // of the backward's first product
            if (l < 3) br_issue(l & 1 ? SW : XU, Wr + (size_t)kW * kRrRow0 + (size_t)l * kW * kRrRow, kW * kRrRow, tid);
            else br_issue(SW, WrT + (size_t)2 * kW * kRrRow, kW * kRrRow, tid);
            const __bf16 *Wl = l & 1 ? XU : SW;
            bf16x8 hout[4];
#pragma unroll
            for (int cp = 0; cp < 4; ++cp) {
                floatx4 acc[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[h] = *(const floatx4 *)(sB + l * kW + 32 * cp + 16 * h + 4 * lg);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c >= nk) break;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const bf16x8 a = *(const bf16x8 *)(Wl + (32 * cp + 16 * h + lc) * row + 32 * c + 8 * lg);
                        acc[h] = mm::mfma(a, hin[c], acc[h]);
                    }
                }
                bf16x8 zq;
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float z = acc[h][i];
                        zq[4 * h + i] = (__bf16)z;
                        if (l < 3) hout[cp][4 * h + i] = (__bf16)(z * frcp(1.0f + fexp2(-z)));
                    }
                ZP[4 * l + cp][tid] = zq;
            }
            if (l < 3) {
#pragma unroll
                for (int c = 0; c < 4; ++c) hin[c] = hout[c];
            }
            br_wait();
            __syncthreads();
        }
        // ---- output layer: dL/dh'_3 = W5'^T dL/do, then h'_3 and dL/dz'_3
        const float4 d = m < M ? dO[m] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        bf16x8 hp[4], dz[4], dzu[4];   // h' and dL/dz' of the current layer, dL/dz' of the layer above
#pragma unroll
        for (int cp = 0; cp < 4; ++cp) {
            const bf16x8 zq = ZP[12 + cp][tid];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int n = 32 * cp + 16 * (e >> 2) + 4 * lg + (e & 3);
                const float dh = fmaf(sW5[n], d.x, fmaf(sW5[kW + n], d.y, sW5[2 * kW + n] * d.z));
                br_act_grad(zq[e], dh, hp[cp], dz[cp], e);
            }
        }
#pragma unroll
        for (int l = 3; l >= 0; --l) {
            // gradient of the layer above (the output layer when l == 3):
            // its dL/dz' and this layer's h', point-major, into LDS
            br_write_rows(XH, hp, lg, col);
            if (l == 3) {
                if (lg == 0) {
                    XD[0 * kBrStride + col] = (__bf16)d.x;
                    XD[1 * kBrStride + col] = (__bf16)d.y;
                    XD[2 * kBrStride + col] = (__bf16)d.z;
                } else {
                    // rows 3..15 are zero padding of the 16-row tile
#pragma unroll
                    for (int r = 0; r < 5; ++r) {
                        const int rr = 3 + 5 * (lg - 1) + r;
                        if (rr < 16) XD[rr * kBrStride + col] = (__bf16)0.0f;
                    }
                }
            } else {
                br_write_rows(XD, dzu, lg, col);
            }
            __syncthreads();
            // SW is free (every wave's product with it came before its rows):
            // issue the transposed weights of the next product down, or after
            // the last one the next pass's layer-0 weights
            if (l == 2 || l == 1) br_issue(SW, WrT + (size_t)(l - 1) * kW * kRrRow, kW * kRrRow, tid);
            else if (l == 0) br_issue(SW, Wr, kW * kRrRow0, tid);
            if (l == 3) {
#pragma unroll
                for (int kc = 0; kc < kBrPts / 32; ++kc) {
                    const bf16x8 a = *(const bf16x8 *)(XD + lc * kBrStride + 32 * kc + 8 * lg);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const bf16x8 b = *(const bf16x8 *)(XH + (16 * (wv + 4 * q) + lc) * kBrStride + 32 * kc + 8 * lg);
                        g4[q][0] = mm::mfma(a, b, g4[q][0]);
                    }
                }
                if (wv == 0) {
                    const float v = br_rowsum(XD, lane >> 1, bhalf);   // rows 0..2 are dL/do
                    if (lane < 6) db5 += v;
                }
            } else if (l == 2) {
                br_dw<8>(g3, XD, XH, wv, lg, lc);
                db3 += br_rowsum(XD, brow, bhalf);
            } else if (l == 1) {
                br_dw<8>(g2, XD, XH, wv, lg, lc);
                db2 += br_rowsum(XD, brow, bhalf);
            } else {
                br_dw<8>(g1, XD, XH, wv, lg, lc);
                db1 += br_rowsum(XD, brow, bhalf);
            }
            if (l != 0) br_wait();
            __syncthreads();
#pragma unroll
            for (int c = 0; c < 4; ++c) dzu[c] = dz[c];
            // dL/dh' of the layer below through the transposed weights, and
            // at once its h' and dL/dz'
            if (l >= 1) {
                // (the transposed weights are in SW, waited for before the
                // barrier above)
                const __bf16 *WT = SW;
#pragma unroll
                for (int cp = 0; cp < 4; ++cp) {
                        floatx4 acc[2] = {floatx4{0.0f, 0.0f, 0.0f, 0.0f}, floatx4{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
                    for (int c = 0; c < 4; ++c)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const bf16x8 a = *(const bf16x8 *)(WT + (32 * cp + 16 * h + lc) * kRrRow + 32 * c + 8 * lg);
                            acc[h] = mm::mfma(a, dzu[c], acc[h]);
                        }
                    const bf16x8 zq = ZP[4 * (l - 1) + cp][tid];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int i = 0; i < 4; ++i) br_act_grad(zq[4 * h + i], acc[h][i], hp[cp], dz[cp], 4 * h + i);
                }
            }
        }
        // ---- layer 0: features and dz'_0
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const bf16x8 f = ZP[16 + c][tid];
#pragma unroll
            for (int j = 0; j < 8; ++j) XH[(32 * c + 8 * lg + j) * kBrStride + col] = f[j];
        }
        br_write_rows(XD, dz, lg, col);
        __syncthreads();
        br_dw<4>(g0, XD, XH, wv, lg, lc);
        db0 += br_rowsum(XD, brow, bhalf);
        br_wait();   // the next pass's layer-0 weights
        __syncthreads();
    }
    // ---- flush: flat layout per layer W [out][in] then b [out]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 32 * wv + 16 * a + 4 * lg + i;
#pragma unroll
            for (int it = 0; it < 4; ++it) atomicAdd(dW + w.off[0] + o * kF + 16 * it + lc, kLog2E * g0[a][it][i]);
#pragma unroll
            for (int it = 0; it < 8; ++it) {
                atomicAdd(dW + w.off[1] + o * kW + 16 * it + lc, g1[a][it][i]);
                atomicAdd(dW + w.off[2] + o * kW + 16 * it + lc, g2[a][it][i]);
                atomicAdd(dW + w.off[3] + o * kW + 16 * it + lc, g3[a][it][i]);
            }
        }
    if (bhalf == 0) {
        atomicAdd(dW + w.off[0] + kW * kF + brow, kLog2E * db0);
        atomicAdd(dW + w.off[1] + kW * kW + brow, kLog2E * db1);
        atomicAdd(dW + w.off[2] + kW * kW + brow, kLog2E * db2);
        atomicAdd(dW + w.off[3] + kW * kW + brow, kLog2E * db3);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 4 * lg + i;
            if (j < 3) atomicAdd(dW + w.off[4] + j * kW + 16 * (wv + 4 * q) + lc, kLn2 * g4[q][0][i]);
        }
    if (wv == 0 && lane < 6 && bhalf == 0) atomicAdd(dW + w.off[4] + 3 * kW + (lane >> 1), db5);
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
    if (precision == RT_MLP_BF16) n += 2 * kRrWeightElems + 256 + 2 * 3 * (size_t)kW * kRrRow + 256;
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
    w->Wr = precision == RT_MLP_BF16 ? take(2 * kRrWeightElems) : nullptr;
    w->WrT = precision == RT_MLP_BF16 ? take(2 * 3 * (size_t)kW * kRrRow) : nullptr;
    for (int q = 0; q < 16; ++q) w->freq[q] = (float)std::exp2(3.0 * q / 15.0);
    const int n = kW * kW;
    if (precision == RT_MLP_BF16) {
        hipLaunchKernelGGL(mlp_prep<__bf16>, dim3((n + 255) / 256), dim3(256), 0, st, flat, *w);
        const int nr = kW * kRrRow;
        hipLaunchKernelGGL(mlp_prep_rr, dim3((nr + 255) / 256), dim3(256), 0, st, flat, *w);
    } else
        hipLaunchKernelGGL(mlp_prep<float>, dim3((n + 255) / 256), dim3(256), 0, st, flat, *w);
    return hipGetLastError();
}

hipError_t mlp_forward(const Geometry &g, const Shade &s, const MlpDev &w, int precision, size_t M, float4 *out,
                       hipStream_t st) {
    if (precision == RT_MLP_BF16) {
        int dev = 0, ncu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        constexpr int NP = kRrTiles, NT = kRrThreads;
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)mlp_fwd_rr<NP, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kRrLds);
        if (e != hipSuccess) return e;
        constexpr size_t pts = NT / 64 * NP * 16;
        const unsigned grid = (unsigned)std::min<size_t>((M + pts - 1) / pts, (size_t)ncu);
        hipLaunchKernelGGL((mlp_fwd_rr<NP, NT>), dim3(grid), dim3(NT), kRrLds, st, g, s, w, M, out);
    } else {
        constexpr int P = 32;
        hipLaunchKernelGGL((mlp_fwd<float, P>), dim3((unsigned)((M + P - 1) / P)), dim3(512), 0, st, g, s, w, M, out);
    }
    return hipGetLastError();
}

size_t mlp_backward_list_bytes(size_t M) { return sizeof(uint32_t) * (1 + M + 2 * (size_t)kLiveChunks); }

hipError_t mlp_backward(const Geometry &g, const Shade &s, const MlpDev &w, int precision, size_t M,
                        const float4 *dO, uint32_t *list, float *dW, hipStream_t st) {
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (precision == RT_MLP_BF16) {
        const size_t passes = (M + kBrPts - 1) / kBrPts;
        // chunks of at least 1024 points, at most kLiveChunks of them
        const size_t chunk = std::max<size_t>(1024, (M + kLiveChunks - 1) / kLiveChunks);
        const int nb = (int)((M + chunk - 1) / chunk);
        uint32_t *counts = list + 1 + M, *offsets = counts + kLiveChunks;
        hipLaunchKernelGGL(mlp_live_count, dim3(nb), dim3(1024), 0, st, dO, M, chunk, counts);
        hipLaunchKernelGGL(mlp_live_scan, dim3(1), dim3(1024), 0, st, counts, nb, offsets, list);
        hipLaunchKernelGGL(mlp_live_write, dim3(nb), dim3(1024), 0, st, dO, M, chunk, offsets, list);
        const unsigned grid = (unsigned)std::min<size_t>(passes, (size_t)ncu);
        hipLaunchKernelGGL(mlp_bwd_rr, dim3(grid), dim3(256), 0, st, g, s, w, M, dO, list, dW);
    } else {
        constexpr int P = 16;
        const size_t ntiles = (M + P - 1) / P;
        const unsigned grid = (unsigned)std::min<size_t>(ntiles, (size_t)ncu);
        hipLaunchKernelGGL((mlp_bwd<float, P>), dim3(grid), dim3(512), 0, st, g, s, w, M, dO, dW);
    }
    return hipGetLastError();
}

} // namespace rt
