// rt_neural_t.hip -- the neural temperature field of Methods, "Neural
// Temperature Recovery" on the render grid's nodes, its vector-Jacobian
// product to the weights, and the Adam step.
//
// T(r, |z|) = 5 + 395 sigma(o), o = MLP(gamma(x_r, x_z)): sinusoidal encoding
// of degree 4 of the normalised node coordinates (16 features), four ReLU
// layers of 64 units, one output.  The grid has 3.3e4 nodes at 256 x 128 and
// the network 1.4e4 weights (4.4e8 multiply-adds per evaluation), so this is
// plain FP32 VALU work: a workgroup of 128 nodes keeps each node's
// activations in its own LDS column, and four lanes per node each accumulate
// a 16-output slice of every layer in registers against weights staged in
// LDS (read as broadcasts: the lanes of a wave share their slice).  Four
// lanes per node give 8 waves per CU where one lane per node gave 2, with
// the same LDS (weights + two activation buffers).  The weight
// gradient sums outer products over the nodes: per layer and chunk of 128
// nodes in LDS into partial sums, then reduced in a fixed order
// (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/rtcube.h"
#include "rt_host.h"

namespace rt {

namespace {

constexpr int kNtL = 4, kNtIn = 4 * kNtL, kNtW = 64;
// nodes per workgroup, lanes per node, outputs per lane
constexpr int kNtNodes = 128, kNtQ = 4, kNtBlock = kNtNodes * kNtQ, kNtSlice = kNtW / kNtQ;
// flat layout: per layer W [out][in] then b [out]
constexpr int layer_in(int l) { return l == 0 ? kNtIn : kNtW; }
constexpr int layer_out(int l) { return l == 4 ? 1 : kNtW; }
constexpr int layer_off(int l) {
    int o = 0;
    for (int k = 0; k < l; ++k) o += layer_in(k) * layer_out(k) + layer_out(k);
    return o;
}
static_assert(layer_off(5) == RT_NT_PARAMS, "neural temperature parameter count");
// activation rows per node: 16 features, 4 x 64 hidden, the output o
constexpr int kActRows = kNtIn + 4 * kNtW + 1;
constexpr int kDeltaRows = 4 * kNtW + 1;
constexpr int kNtChunk = 128;    // nodes per partial sum of the weight gradient

__device__ __forceinline__ void node_features(int n, int nr, int nz, float *f) {
    const int i = n / nz, j = n - i * nz;
    const float x[2] = {(float)i / (float)(nr - 1), (float)j / (float)(nz - 1)};
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < kNtL; ++k) {
            float s, co;
            sincospif((float)(1 << k) * x[c], &s, &co);
            f[8 * c + k] = s;
            f[8 * c + kNtL + k] = co;
        }
}

// LDS: per layer l the transposed weights WT_l [in][out] then b_l (forward),
// or W_l [out][in] (backward); then two activation buffers [64][kNtNodes].
__device__ __forceinline__ void stage_weights(const float *W, float *sw, bool transposed) {
    for (int p = threadIdx.x; p < RT_NT_PARAMS; p += blockDim.x) {
        int l = 0;
        while (l < 4 && p >= layer_off(l + 1)) ++l;
        const int q = p - layer_off(l), in = layer_in(l), out = layer_out(l);
        int dst = p;
        if (transposed && q < in * out) {
            const int a = q / in, b = q - a * in;     // W[a][b]
            dst = layer_off(l) + b * out + a;         // WT[b][a]
        }
        sw[dst] = W[p];
    }
}

// one dense layer, this lane's slice of outputs a = 16 q + c of node column
// j: out[a] = act(sum_b W[a][b] in[b] + b[a]), with WT [in][out] in LDS; the
// slice is also left in acc
template <int IN, bool RELU>
__device__ __forceinline__ void dense_slice(const float *wt, const float *bias, const float *hin, float *hout, int j,
                                            int q, float *acc) {
#pragma unroll
    for (int c = 0; c < kNtSlice; ++c) acc[c] = bias[q * kNtSlice + c];
#pragma unroll 4
    for (int b = 0; b < IN; ++b) {
        const float h = hin[b * kNtNodes + j];
#pragma unroll
        for (int c = 0; c < kNtSlice; ++c) acc[c] = fmaf(wt[b * kNtW + q * kNtSlice + c], h, acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kNtSlice; ++c) {
        if (RELU) acc[c] = fmaxf(acc[c], 0.0f);
        hout[(q * kNtSlice + c) * kNtNodes + j] = acc[c];
    }
}

// lane t: node column j = t mod 128, slice q = t / 128 (one slice per wave)
__global__ __launch_bounds__(kNtBlock) void nt_fwd(int nr, int nz, const float *__restrict__ W,
                                                   float *__restrict__ T, float *__restrict__ act) {
    extern __shared__ float sm[];
    float *sw = sm, *h0 = sm + RT_NT_PARAMS, *h1 = h0 + kNtW * kNtNodes;
    stage_weights(W, sw, true);
    const int N = nr * nz, t = threadIdx.x, j = t % kNtNodes;
    const int q = __builtin_amdgcn_readfirstlane(t / kNtNodes);
    const int n = blockIdx.x * kNtNodes + j;
    const int nn = n < N ? n : N - 1;   // lanes past the end compute a copy and store nothing
    const bool store = act && n < N;
    if (q == 0) {
        float f[kNtIn];
        node_features(nn, nr, nz, f);
#pragma unroll
        for (int b = 0; b < kNtIn; ++b) h0[b * kNtNodes + j] = f[b];
        if (store)
            for (int b = 0; b < kNtIn; ++b) act[(size_t)b * N + n] = f[b];
    }
    __syncthreads();
    float acc[kNtSlice];
    // hidden layer l reads one buffer and writes the other; act rows 16 + 64 l + a
    dense_slice<kNtIn, true>(sw + layer_off(0), sw + layer_off(0) + kNtIn * kNtW, h0, h1, j, q, acc);
    if (store)
        for (int c = 0; c < kNtSlice; ++c) act[(size_t)(kNtIn + q * kNtSlice + c) * N + n] = acc[c];
    __syncthreads();
    float *hin = h1, *hout = h0;
    for (int l = 1; l < 4; ++l) {
        dense_slice<kNtW, true>(sw + layer_off(l), sw + layer_off(l) + kNtW * kNtW, hin, hout, j, q, acc);
        if (store)
            for (int c = 0; c < kNtSlice; ++c)
                act[(size_t)(kNtIn + l * kNtW + q * kNtSlice + c) * N + n] = acc[c];
        __syncthreads();
        float *tmp = hin;
        hin = hout;
        hout = tmp;
    }
    // output unit (one lane per node): o = b_4 + sum_b W_4[0][b] h_4[b]
    if (q == 0) {
        const float *w4 = sw + layer_off(4);
        float o = w4[kNtW];
        for (int b = 0; b < kNtW; ++b) o = fmaf(w4[b], hin[b * kNtNodes + j], o);
        if (n < N) {
            T[n] = 5.0f + 395.0f / (1.0f + expf(-o));
            if (act) act[(size_t)(kActRows - 1) * N + n] = o;
        }
    }
}

// backward through the layers for node column j, slice q: delta rows (dL/dz
// of hidden layers 1..4, then dL/do) into `delta` [kDeltaRows][N]
__global__ __launch_bounds__(kNtBlock) void nt_delta(int N, const float *__restrict__ W,
                                                     const float *__restrict__ dT, const float *__restrict__ act,
                                                     float *__restrict__ delta) {
    extern __shared__ float sm[];
    float *sw = sm, *d0 = sm + RT_NT_PARAMS, *d1 = d0 + kNtW * kNtNodes;
    stage_weights(W, sw, false);
    __syncthreads();
    const int t = threadIdx.x, j = t % kNtNodes;
    const int q = __builtin_amdgcn_readfirstlane(t / kNtNodes);
    const int n = blockIdx.x * kNtNodes + j, nn = n < N ? n : N - 1;
    const float o = act[(size_t)(kActRows - 1) * N + nn];
    const float s = 1.0f / (1.0f + expf(-o));
    const float dlo = (n < N ? dT[n] : 0.0f) * 395.0f * s * (1.0f - s);
    if (q == 0 && n < N) delta[(size_t)(kDeltaRows - 1) * N + n] = dlo;
    // dL/dz_4 = W_4^T dL/do masked by h_4 > 0
    const float *w4 = sw + layer_off(4);
    for (int c = 0; c < kNtSlice; ++c) {
        const int a = q * kNtSlice + c;
        const float h = act[(size_t)(kNtIn + 3 * kNtW + a) * N + nn];
        const float v = h > 0.0f ? w4[a] * dlo : 0.0f;
        d0[a * kNtNodes + j] = v;
        if (n < N) delta[(size_t)(3 * kNtW + a) * N + n] = v;
    }
    __syncthreads();
    // dL/dz_l = W_l^T dL/dz_{l+1} masked by h_l > 0, for l = 3, 2, 1 (W_l maps h_l to z_{l+1})
    float *cur = d0, *nxt = d1;
    for (int l = 3; l >= 1; --l) {
        const float *wl = sw + layer_off(l);   // W_l [out][in]
        float acc[kNtSlice];
#pragma unroll
        for (int c = 0; c < kNtSlice; ++c) acc[c] = 0.0f;
#pragma unroll 4
        for (int a = 0; a < kNtW; ++a) {
            const float g = cur[a * kNtNodes + j];
#pragma unroll
            for (int c = 0; c < kNtSlice; ++c) acc[c] = fmaf(wl[a * kNtW + q * kNtSlice + c], g, acc[c]);
        }
#pragma unroll
        for (int c = 0; c < kNtSlice; ++c) {
            const int b = q * kNtSlice + c;
            const float h = act[(size_t)(kNtIn + (l - 1) * kNtW + b) * N + nn];
            const float v = h > 0.0f ? acc[c] : 0.0f;
            nxt[b * kNtNodes + j] = v;
            if (n < N) delta[(size_t)((l - 1) * kNtW + b) * N + n] = v;
        }
        __syncthreads();
        float *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
}

// partial weight gradient of layer blockIdx.y over one chunk of kNtChunk
// nodes: W_l[a][b] gets sum_n dz_{l+1}[a][n] in_l[b][n] and b_l[a] gets
// sum_n dz_{l+1}[a][n].  The chunk's rows of dz_{l+1} (delta rows l 64 + a,
// or dL/do for the output layer) and of in_l (the features, or h_l) are
// staged in LDS; each lane accumulates up to 16 (a, b) entries (a 4 x 4 tile
// in the 64 x 64 layers).
__global__ __launch_bounds__(256) void nt_wgrad(int N, const float *__restrict__ act, const float *__restrict__ delta,
                                                float *__restrict__ partial) {
    __shared__ float sA[kNtW][kNtChunk + 1], sB[kNtW][kNtChunk + 1];
    const int l = blockIdx.y, M = layer_out(l), K = layer_in(l);
    const int n0 = blockIdx.x * kNtChunk, t = threadIdx.x;
    for (int idx = t; idx < kNtW * kNtChunk; idx += 256) {
        const int r = idx / kNtChunk, k = idx - r * kNtChunk, n = n0 + k;
        if (r < M) sA[r][k] = n < N ? delta[(size_t)(l == 4 ? kDeltaRows - 1 : l * kNtW + r) * N + n] : 0.0f;
        if (r < K) sB[r][k] = n < N ? act[(size_t)(l == 0 ? r : kNtIn + (l - 1) * kNtW + r) * N + n] : 0.0f;
    }
    __syncthreads();
    float *out = partial + (size_t)blockIdx.x * RT_NT_PARAMS + layer_off(l);
    if (M == kNtW && K == kNtW) {
        // 64 x 64 layers: a 4 x 4 tile of (a, b) per lane, 8 LDS reads per 16 FMAs
        const int a0 = (t / 16) * 4, b0 = (t % 16) * 4;
        float acc[4][4], bias[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bias[i] = 0.0f;
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[i][c] = 0.0f;
        }
        for (int k = 0; k < kNtChunk; ++k) {
            float ga[4], gb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) { ga[i] = sA[a0 + i][k]; gb[i] = sB[b0 + i][k]; }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bias[i] += ga[i];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[i][c] = fmaf(ga[i], gb[c], acc[i][c]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) out[(a0 + i) * K + b0 + c] = acc[i][c];
            if (b0 == 0) out[M * K + a0 + i] = bias[i];
        }
        return;
    }
    // other layers: lane -> row a and a run of `per` consecutive columns b0..
    const int per = (M * K + 255) / 256;          // 4 (64 x 16), 1 (1 x 64)
    const int runs = K / per;
    const int a = t / runs, b0 = (t - a * runs) * per;
    if (a < M) {
        float acc[16], bias = 0.0f;
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
        for (int k = 0; k < kNtChunk; ++k) {
            const float g = sA[a][k];
            bias += g;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < per) acc[c] = fmaf(g, sB[b0 + c][k], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < per) out[a * K + b0 + c] = acc[c];
        if (b0 == 0) out[M * K + a] = bias;
    }
}

// dW[p] = sum over chunks of the partials: 64 parameters per workgroup, 8
// lanes per parameter each summing every 8th chunk, then the 8 partial sums
// added in a fixed order (deterministic)
constexpr int kNtRedGroups = 8;
__global__ __launch_bounds__(64 * kNtRedGroups) void nt_wreduce(int chunks, const float *__restrict__ partial,
                                                                float *__restrict__ dW) {
    __shared__ float part[kNtRedGroups][64];
    const int pl = threadIdx.x % 64, g = threadIdx.x / 64;
    const int p = blockIdx.x * 64 + pl;
    float s = 0.0f;
    if (p < RT_NT_PARAMS)
        for (int c = g; c < chunks; c += kNtRedGroups) s += partial[(size_t)c * RT_NT_PARAMS + p];
    part[g][pl] = s;
    __syncthreads();
    if (g == 0 && p < RT_NT_PARAMS) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < kNtRedGroups; ++k) t += part[k][pl];
        dW[p] = t;
    }
}

__global__ __launch_bounds__(256) void nt_adam(int64_t n, float *__restrict__ p, float *__restrict__ m,
                                               float *__restrict__ v, const float *__restrict__ g, float lr, float b1,
                                               float b2, float eps, float gscale, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] * gscale;
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

rt_status validate_nt_grid(const rt_grid *g) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (g->nr < 2 || g->nz < 2) return fail(RT_EINVAL, "grid needs nr, nz >= 2");
    if ((size_t)g->nr * g->nz > (size_t)1 << 26) return fail(RT_EINVAL, "grid too large for the neural temperature");
    return RT_OK;
}

constexpr size_t kNtLds = sizeof(float) * (RT_NT_PARAMS + 2 * kNtW * kNtNodes);

hipError_t nt_lds_attr() {
    hipError_t e = hipFuncSetAttribute((const void *)nt_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNtLds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)nt_delta, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNtLds);
    return e;
}

} // namespace

} // namespace rt

using namespace rt;

extern "C" rt_status rt_neural_temperature(const rt_grid *grid, const float *weights, float *temp_k, void *stream) {
    rt_status st = validate_nt_grid(grid);
    if (st != RT_OK) return st;
    if (!weights || !temp_k) return fail(RT_EINVAL, "weights and temp_k must not be NULL");
    hipError_t e = nt_lds_attr();
    if (e != hipSuccess) return fail_hip(e, "neural temperature attributes");
    const int N = grid->nr * grid->nz;
    hipLaunchKernelGGL(nt_fwd, dim3((N + kNtNodes - 1) / kNtNodes), dim3(kNtBlock), kNtLds, (hipStream_t)stream,
                       grid->nr, grid->nz, weights, temp_k, (float *)nullptr);
    e = hipGetLastError();
    return e == hipSuccess ? RT_OK : fail_hip(e, "neural temperature");
}

extern "C" rt_status rt_neural_temperature_adjoint(const rt_grid *grid, const float *weights, const float *d_temp_k,
                                                   float *d_weights, void *stream) {
    rt_status st = validate_nt_grid(grid);
    if (st != RT_OK) return st;
    if (!weights || !d_temp_k || !d_weights) return fail(RT_EINVAL, "weights, d_temp_k and d_weights must not be NULL");
    hipError_t e = nt_lds_attr();
    if (e != hipSuccess) return fail_hip(e, "neural temperature attributes");
    hipStream_t s = (hipStream_t)stream;
    const int N = grid->nr * grid->nz;
    const int chunks = (N + kNtChunk - 1) / kNtChunk;
    const size_t act_n = (size_t)kActRows * N, del_n = (size_t)kDeltaRows * N, part_n = (size_t)chunks * RT_NT_PARAMS;
    float *w = (float *)stream_workspace(s, kWsNeuralT, sizeof(float) * (act_n + del_n + part_n + N), &e);
    if (!w) return fail_hip(e, "neural temperature scratch");
    float *act = w, *del = w + act_n, *part = del + del_n, *Tn = part + part_n;
    const int blocks = (N + kNtNodes - 1) / kNtNodes;
    hipLaunchKernelGGL(nt_fwd, dim3(blocks), dim3(kNtBlock), kNtLds, s, grid->nr, grid->nz, weights, Tn, act);
    hipLaunchKernelGGL(nt_delta, dim3(blocks), dim3(kNtBlock), kNtLds, s, N, weights, d_temp_k, act, del);
    hipLaunchKernelGGL(nt_wgrad, dim3(chunks, 5), dim3(256), 0, s, N, act, del, part);
    hipLaunchKernelGGL(nt_wreduce, dim3((RT_NT_PARAMS + 63) / 64), dim3(64 * kNtRedGroups), 0, s, chunks, part, d_weights);
    e = hipGetLastError();
    return e == hipSuccess ? RT_OK : fail_hip(e, "neural temperature adjoint");
}

extern "C" rt_status rt_adam_step(float *params, float *m, float *v, const float *grad, int64_t n, const rt_adam *opt,
                                  int64_t step, void *stream) {
    if (!params || !m || !v || !grad || !opt) return fail(RT_EINVAL, "Adam arguments must not be NULL");
    if (n < 0) return fail(RT_EINVAL, "parameter count must be >= 0");
    if (step < 1) return fail(RT_EINVAL, "Adam steps count from 1");
    if (!(opt->beta1 >= 0.0 && opt->beta1 < 1.0) || !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) || !(opt->eps > 0.0))
        return fail(RT_EINVAL, "need 0 <= beta1, beta2 < 1 and eps > 0");
    if (n == 0) return RT_OK;
    const float c1 = (float)(1.0 / (1.0 - std::pow(opt->beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(opt->beta2, (double)step)));
    hipLaunchKernelGGL(nt_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, params, m, v,
                       grad, (float)opt->lr, (float)opt->beta1, (float)opt->beta2, (float)opt->eps,
                       (float)opt->grad_scale, c1, c2);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RT_OK : fail_hip(e, "Adam step");
}
