// rt_beam.hip -- restoring-beam convolution of a model cube (gfx950).
//
// A model cube is compared with an interferometric image only after both are
// at the same resolution: every channel map is convolved with the image's
// elliptical Gaussian beam (FWHM bmaj >= bmin in pixels, major axis at bpa
// from +y towards -x), sampled at integer offsets within |dx|, |dy| <= R =
// ceil(3 sigma_maj), normalised to unit sum, zero outside the image.  The
// kernel is point-symmetric and the padding is zeros, so the operator is its
// own adjoint: the backward of the convolution is the same call.
//
// beam_weights (one workgroup) evaluates the (2R+1)^2 weights in float,
// normalises them by their workgroup-reduced sum and stores them.  beam_conv: one
// workgroup per 64 x 32 output tile of one channel; the tile plus its R-wide
// halo is staged in LDS (zeros outside the image) with the weights; each lane
// forms 8 consecutive outputs of one row, sliding a window of 8 staged values
// along each kernel row 8 taps at a time, so a tap costs one LDS read of data,
// one broadcast read of the weight and 8 FMAs.  The 32 lanes of a half-wave take 32
// different rows at one column, and the row pitch is odd, so their reads fall
// in distinct banks.  The work is dense FMA, not HBM traffic: (2R+1)^2 FMAs per
// output against 8 bytes moved.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/rtcube.h"
#include "rt_host.h"

namespace rt {

constexpr int kBeamTX = 64, kBeamTY = 32, kBeamOut = 8;   // tile and outputs per lane

__global__ __launch_bounds__(256) void beam_weights(float *__restrict__ w, int R, float inv_smaj, float inv_smin,
                                                    float spa, float cpa) {
    __shared__ float part[256];
    const int n = 2 * R + 1, nn = n * n;
    auto weight = [&](int idx) {
        const float dy = (float)(idx / n - R), dx = (float)(idx % n - R);
        const float u = fmaf(-dx, spa, dy * cpa) * inv_smaj, v = fmaf(dx, cpa, dy * spa) * inv_smin;
        return expf(-0.5f * fmaf(u, u, v * v));
    };
    float s = 0.0f;
    for (int i = threadIdx.x; i < nn; i += blockDim.x) s += weight(i);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    const float inv = 1.0f / part[0];
    for (int i = threadIdx.x; i < nn; i += blockDim.x) w[i] = weight(i) * inv;
}

__global__ __launch_bounds__(256) void beam_conv(const float *__restrict__ in, float *__restrict__ out,
                                                 const float *__restrict__ w, int nx, int ny, int R) {
    extern __shared__ float lds[];
    const int n = 2 * R + 1;
    const int W = kBeamTX + 2 * R, H = kBeamTY + 2 * R;
    const int P = W | 1;                       // odd row pitch
    float *tile = lds;
    float *wk = lds + H * P;
    const int x0 = blockIdx.x * kBeamTX, y0 = blockIdx.y * kBeamTY;
    const size_t plane = (size_t)nx * ny;
    const float *src = in + blockIdx.z * plane;
    // the pad column (lx = W) is zeroed: the window's last refill reads it
    for (int i = threadIdx.x; i < H * P; i += blockDim.x) {
        const int ly = i / P, lx = i % P;
        const int gy = y0 - R + ly, gx = x0 - R + lx;
        tile[i] = (lx < W && gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? src[(size_t)gy * nx + gx] : 0.0f;
    }
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) wk[i] = w[i];
    __syncthreads();
    const int ty = threadIdx.x % kBeamTY;      // lanes of a half-wave: 32 rows
    const int tx = threadIdx.x / kBeamTY;      // 8 groups of 8 columns
    float acc[kBeamOut];
#pragma unroll
    for (int q = 0; q < kBeamOut; ++q) acc[q] = 0.0f;
    // out(y, x) = sum_{j, i} K[j][i] in(y + R - j, x + R - i) = sum K[j][i] tile[ty + 2R - j][lx + 2R - i];
    // K is point-symmetric (K[j][i] = K[2R-j][2R-i]), so equally sum K[j][i] tile[ty + j][lx + i].
    for (int j = 0; j < n; ++j) {
        const float *row = tile + (ty + j) * P + tx * kBeamOut;
        const float *kr = wk + j * n;
        float win[kBeamOut];
#pragma unroll
        for (int q = 0; q < kBeamOut; ++q) win[q] = row[q];
        int i = 0;
        // 8 taps at a time with the next 8 values in a second window: the
        // shifts become register renaming (row[i + 15] <= row[2R + 8], the pad)
        for (; i + kBeamOut <= n; i += kBeamOut) {
            float nxt[kBeamOut];
#pragma unroll
            for (int q = 0; q < kBeamOut; ++q) nxt[q] = row[i + kBeamOut + q];
#pragma unroll
            for (int t = 0; t < kBeamOut; ++t) {
                const float k = kr[i + t];
#pragma unroll
                for (int q = 0; q < kBeamOut; ++q)
                    acc[q] = fmaf(k, t + q < kBeamOut ? win[t + q] : nxt[t + q - kBeamOut], acc[q]);
            }
#pragma unroll
            for (int q = 0; q < kBeamOut; ++q) win[q] = nxt[q];
        }
        for (; i < n; ++i) {
            const float k = kr[i];
#pragma unroll
            for (int q = 0; q < kBeamOut; ++q) acc[q] = fmaf(k, win[q], acc[q]);
#pragma unroll
            for (int q = 0; q < kBeamOut - 1; ++q) win[q] = win[q + 1];
            win[kBeamOut - 1] = row[i + kBeamOut];
        }
    }
    const int y = y0 + ty;
    if (y >= ny) return;
    float *dst = out + blockIdx.z * plane + (size_t)y * nx;
#pragma unroll
    for (int q = 0; q < kBeamOut; ++q) {
        const int x = x0 + tx * kBeamOut + q;
        if (x < nx) dst[x] = acc[q];
    }
}

} // namespace rt

using namespace rt;

namespace rt {

rt_status validate_beam(const rt_beam &b) {
    if (!(std::isfinite(b.bmaj_px) && std::isfinite(b.bmin_px) && std::isfinite(b.bpa_deg) && b.bmin_px > 0.0 &&
          b.bmaj_px >= b.bmin_px))
        return fail(RT_EINVAL, "need 0 < bmin_px <= bmaj_px and a finite bpa_deg");
    const int R = (int)std::ceil(3.0 * b.bmaj_px / (2.0 * std::sqrt(2.0 * std::log(2.0))));
    if (R > RT_BEAM_MAX_RADIUS) return fail(RT_EINVAL, "beam support radius %d exceeds %d pixels", R, RT_BEAM_MAX_RADIUS);
    return RT_OK;
}

rt_status beam_in_place(float *cube, int nch, int ny, int nx, const rt_beam &b, hipStream_t st) {
    const size_t bytes = (size_t)nch * nx * ny * sizeof(float);
    hipError_t e;
    float *tmp = (float *)stream_workspace(st, kWsBeamCube, bytes, &e);
    if (!tmp) return fail_hip(e, "beam cube workspace");
    rt_status rs = rt_beam_convolve(cube, tmp, nch, ny, nx, &b, st);
    if (rs != RT_OK) return rs;
    e = hipMemcpyAsync(cube, tmp, bytes, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? RT_OK : fail_hip(e, "beam copy");
}

} // namespace rt

extern "C" rt_status rt_beam_convolve(const float *in, float *out, int32_t nch, int32_t ny, int32_t nx,
                                      const rt_beam *beam, void *stream) {
    if (!in || !out) return fail(RT_EINVAL, "in and out are required");
    if (!beam) return fail(RT_EINVAL, "beam is NULL");
    if (nch < 1 || ny < 1 || nx < 1) return fail(RT_EINVAL, "need nch, ny, nx >= 1");
    if (nch > 65535 || (int64_t)nx * ny > (int64_t)1 << 30) return fail(RT_EINVAL, "cube too large");
    rt_status vs = validate_beam(*beam);
    if (vs != RT_OK) return vs;
    const double bmaj = beam->bmaj_px, bmin = beam->bmin_px, bpa = beam->bpa_deg;
    const double fw = 2.0 * std::sqrt(2.0 * std::log(2.0));
    const double smaj = bmaj / fw, smin = bmin / fw;
    const int R = (int)std::ceil(3.0 * smaj);
    const size_t bytes = (size_t)nch * nx * ny * sizeof(float);
    const char *a = (const char *)in, *b = (const char *)out;
    if (a < b + bytes && b < a + bytes) return fail(RT_EINVAL, "in and out overlap");
    hipStream_t st = (hipStream_t)stream;
    const int n = 2 * R + 1;
    hipError_t e;
    float *w = (float *)stream_workspace(st, kWsBeam, sizeof(float) * n * n, &e);
    if (!w) return fail_hip(e, "beam workspace");
    const double pa = bpa * 3.14159265358979323846 / 180.0;
    hipLaunchKernelGGL(beam_weights, dim3(1), dim3(256), 0, st, w, R, (float)(1.0 / smaj), (float)(1.0 / smin),
                       (float)std::sin(pa), (float)std::cos(pa));
    if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e, "beam weights launch");
    const int W = kBeamTX + 2 * R, H = kBeamTY + 2 * R, P = W | 1;
    const size_t lds = sizeof(float) * ((size_t)H * P + (size_t)n * n);
    dim3 grid((nx + kBeamTX - 1) / kBeamTX, (ny + kBeamTY - 1) / kBeamTY, nch);
    hipLaunchKernelGGL(beam_conv, grid, dim3(256), lds, st, in, out, w, nx, ny, R);
    if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e, "beam convolution launch");
    return RT_OK;
}
