// rt_render3d.hip -- line emission of fields on a 3-D spherical grid (gfx950).
//
// The fields of a non-axisymmetric disk (a hydrodynamic snapshot: density,
// temperature, all three velocity components, CO abundance) live on nodes
// r_i (log-spaced), theta_j (uniform polar angle), phi_k (uniform, periodic).
// The march keeps them as one interleaved record of eight floats per node,
// {ln n_H2, T, x_CO, v_r, v_theta, v_phi, 0, 0}: a sample's eight corners are
// sixteen 16-byte loads, and the two phi neighbours of a corner sit in one
// 64-byte run, where six separate planes would cost 48 scalar loads touching
// six times as many cache lines.  rt_pack_fields3d writes that layout from
// six planes once per snapshot; renders of the same snapshot (other channel
// sets, inclinations, position angles) reuse it.
//
// Per sample: spherical coordinates of the point, trilinear weights of its
// cell (computed once, applied to all six fields), the density fading to
// zero one cell beyond the radial and polar node ranges, LTE populations and
// source function as in the axisymmetric march, and the line-of-sight
// velocity v . w from the three components and the local unit vectors.  The
// channel loop, the lanes-per-ray split and its front-to-back composition
// are those of the axisymmetric march.  A sample beyond the fade (density
// and depth exactly 0) stops after its indices, and a wave skips the channel
// loop of a sample where none of its rays has opacity; the cube is the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/rtcube.h"
#include "rt_host.h"
#include "rt_kernels.h"

namespace rt {

// Per-launch camera geometry (float, the per-ray set-up included).
struct Geometry3 {
    float d_pix, cpa, spa, si, ci;
    float rc2;               // squared radius of the bounding sphere r_max e^dln [au^2]
    float xc, yc;
    int32_t nx, ny, nsamp, pad_;
};

// The ray through pixel (p, q) in the sky frame (x', y'), and h^2 = rc^2 -
// x'^2 - y'^2: the chord through the bounding sphere is s in [-h, h], its
// midpoint at s = 0 on the sky plane.
struct Chord3 {
    float xp, yp, h2;
};

__device__ __forceinline__ Chord3 chord3(const Geometry3 &g, int p, int q) {
    const float X = ((float)p + 0.5f - g.xc) * g.d_pix;
    const float Y = ((float)q + 0.5f - g.yc) * g.d_pix;
    Chord3 c;
    c.xp = fmaf(g.cpa, X, -g.spa * Y);
    c.yp = fmaf(g.spa, X, g.cpa * Y);
    c.h2 = fmaf(-c.xp, c.xp, fmaf(-c.yp, c.yp, g.rc2));
    return c;
}

// Fields and channel-independent constants.
struct Shade3 {
    const float4 *node;      // [nr][nt][np] records, two float4 each
    const float4 *ztab;
    const float *inv_r2n;    // [nr] 1 / r_i^2 of the radial nodes [au^-2]
    int32_t nr, nt, np, pad_;
    float u_scale, log2_rmin;   // coarse radial index (log2 r - log2 r_min) u_scale
    float h_r;                  // u_scale / 2: cells per unit of log2 (r^2 / r_i^2)
    float cth_c, sth_c;         // cos, sin of the middle polar angle theta_c of the nodes
    float inv_dth, half_nt1;    // w = (theta - theta_c) inv_dth + (nt - 1) / 2
    float inv_dph, fnp;         // s = phi inv_dph, phi in [0, 2 pi)
    float fnr, fnt;
    float zt_l2t0, zt_scale;    // partition-function table index
    float el_log2e, theta, c_s;
    float c_k;                  // as the axisymmetric c_k, without x_CO (a field here)
    float c_alpha, sqrt_log2e;
    float si, ci, vsys;
};

// Z(T): the table lookup of the axisymmetric march reads only the table's
// index constants of its shading block.
__device__ __forceinline__ float partition3(const Shade3 &s, const float4 *tab, float log2t) {
    Shade z{};
    z.zt_l2t0 = s.zt_l2t0;
    z.zt_scale = s.zt_scale;
    return partition_fn(z, tab, log2t);
}

// Channel-independent shading of one sample (cf. physics() of the
// axisymmetric march): S, line-centre depth K (log2 units), and d = a - v b.
__device__ __forceinline__ SampleQ shade3(const Shade3 &s, const float4 *tab, float px, float py, float pz,
                                          float ds) {
    const float rho2 = fmaf(px, px, py * py);
    const float r2 = fmaf(pz, pz, rho2);
    const float rho = fsqrt(rho2);
    // Radial index.  A float index near 500 carries ~3e-5 of a cell of
    // rounding and log2 of r^2 ~ 1e5 an absolute error that the cell scale
    // multiplies; so the cell comes from the coarse index and the fraction
    // from log2 of r^2 / r_i^2, a ratio near 1.  The coarse index is within
    // 1e-4 of a cell: one re-centring step suffices.  r = 0 gives a fraction
    // of -inf: clamped fetch, zero taper, zero depth.
    const float uco = fmaf(0.5f, flog2(r2), -s.log2_rmin) * s.u_scale;
    int i0 = (int)clampf(uco, 0.0f, s.fnr - 2.0f);
    float fr = flog2(1.0f + fmaf(r2, s.inv_r2n[i0], -1.0f)) * s.h_r;
    if (fr < 0.0f && i0 > 0) { --i0; fr += 1.0f; }
    else if (fr >= 1.0f && i0 < s.nr - 2) { ++i0; fr -= 1.0f; }
    // Polar index from the angle to the middle node direction theta_c, which
    // is small over a wedge about the midplane (finer float spacing than theta).
    const float a1 = fmaf(rho, s.cth_c, -pz * s.sth_c);   // r sin(theta - theta_c)
    const float a2 = fmaf(pz, s.cth_c, rho * s.sth_c);    // r cos(theta - theta_c)
    const float w = fmaf(atan2f(a1, a2), s.inv_dth, s.half_nt1);
    // fade one cell beyond the node ranges (radially from the cell and its
    // fraction, exact near both ends); beyond the fade the density and the
    // depth are exactly 0: no azimuth, no fetch, no physics
    const float taper = clampf((float)i0 + fr + 1.0f, 0.0f, 1.0f) * clampf((s.fnr - (float)i0) - fr, 0.0f, 1.0f) *
                        clampf(w + 1.0f, 0.0f, 1.0f) * clampf(s.fnt - w, 0.0f, 1.0f);
    if (taper <= 0.0f) {
        SampleQ z;
        z.S = 0.0f; z.K = 0.0f; z.a = 0.0f; z.b = 0.0f;
        return z;
    }
    float sp = atan2f(py, px) * s.inv_dph;
    sp = sp < 0.0f ? sp + s.fnp : sp;
    const float fu = clampf(fr, 0.0f, 1.0f);
    const float wc = clampf(w, 0.0f, s.fnt - 1.0f);
    const int j0 = min((int)wc, s.nt - 2);
    const float fw = wc - (float)j0;
    int k0 = (int)sp;
    const float fs = sp - (float)k0;
    k0 = k0 >= s.np ? k0 - s.np : k0;       // sp may round up to np
    const int k1 = k0 + 1 >= s.np ? 0 : k0 + 1;
    const uint32_t np = (uint32_t)s.np, plane = (uint32_t)s.nt * np;
    const uint32_t b00 = ((uint32_t)i0 * (uint32_t)s.nt + (uint32_t)j0) * np;
    const uint32_t base[4] = {b00, b00 + np, b00 + plane, b00 + plane + np};   // (i,j), (i,j+1), (i+1,j), (i+1,j+1)
    float4 A[8], B[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const size_t n0 = 2 * (size_t)(base[c] + (uint32_t)k0), n1 = 2 * (size_t)(base[c] + (uint32_t)k1);
        A[2 * c] = s.node[n0];
        B[2 * c] = s.node[n0 + 1];
        A[2 * c + 1] = s.node[n1];
        B[2 * c + 1] = s.node[n1 + 1];
    }
    // trilinear weights, in the corner order of the loads
    const float gu = 1.0f - fu, gw = 1.0f - fw, gs = 1.0f - fs;
    const float cuw[4] = {gu * gw, gu * fw, fu * gw, fu * fw};
    float wt[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) { wt[2 * c] = cuw[c] * gs; wt[2 * c + 1] = cuw[c] * fs; }
    float ln_n = 0.0f, T = 0.0f, xco = 0.0f, vr = 0.0f, vt = 0.0f, vp = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        ln_n = fmaf(wt[c], A[c].x, ln_n);
        T = fmaf(wt[c], A[c].y, T);
        xco = fmaf(wt[c], A[c].z, xco);
        vr = fmaf(wt[c], A[c].w, vr);
        vt = fmaf(wt[c], B[c].x, vt);
        vp = fmaf(wt[c], B[c].y, vp);
    }
    const float nco = xco * fexp2(ln_n * kLog2E) * taper;
    // LTE populations and source function
    const float rT = frcp(T);
    const float Z = partition3(s, tab, flog2(T));
    const float el = fexp2(-s.el_log2e * rT);
    const float x = fminf(s.theta * rT, 80.0f);
    const float em1 = expm1_pos(x);
    SampleQ q;
    q.S = s.c_s * frcp(em1);
    const float inv_alpha = frsq(T * s.c_alpha);
    q.K = s.c_k * nco * el * em1 * frcp(Z * (1.0f + em1)) * ds * inv_alpha;
    q.b = s.sqrt_log2e * inv_alpha;
    // v . w with w = (0, sin i, -cos i): radial, polar and azimuthal unit
    // vectors at the sample (the polar and azimuthal terms vanish on the axis)
    const float inv_r = r2 > 0.0f ? frsq(r2) : 0.0f;
    const float inv_rho = rho2 > 0.0f ? frsq(rho2) : 0.0f;
    const float er = fmaf(py, s.si, -pz * s.ci) * inv_r;
    const float et = fmaf((pz * inv_r) * (py * inv_rho), s.si, rho * inv_r * s.ci);
    const float ep = px * inv_rho * s.si;
    const float vlos = fmaf(vp, ep, fmaf(vt, et, fmaf(vr, er, s.vsys)));
    q.a = vlos * q.b;
    return q;
}

// One lane = one pixel (or a sub-chord of it, NSPLIT lanes per ray) x CB
// channels.  Blocks are numbered XCD-aware: the dispatcher deals consecutive
// workgroup ids to the eight XCDs in turn, so id L runs on XCD L % 8; logical
// work item (L % 8) * per_xcd + L / 8 gives each XCD one contiguous run of
// tiles with all their channel blocks, which read the same grid cells from
// that XCD's L2.  Blocks of up to 24 channels are held to 128 VGPRs (4 waves
// per SIMD, no spills): at 24 channels the unconstrained kernel takes ~137
// and runs 3, and the extra resident waves are worth 14% at 512^2 pixels.
template <int CB, int NSPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CB <= 16 ? 4 : 1))) void march3_fwd(Geometry3 g, Shade3 s, Channels ch, float *__restrict__ cube,
                                                   int ch_stride, int nchb, int nwork, int per_xcd) {
    const int L = blockIdx.x;
    const int work = (L % 8) * per_xcd + L / 8;
    if (work >= nwork) return;                       // whole workgroup: padding of the grid to 8 x per_xcd
    __shared__ float4 ztab[kZTableNodes - 1];
    for (int i = threadIdx.x; i < kZTableNodes - 1; i += blockDim.x) ztab[i] = s.ztab[i];
    __syncthreads();
    constexpr int TW = NSPLIT <= 2 ? 16 : 8;
    constexpr int TH = 256 / NSPLIT / TW;
    const int tiles_x = (g.nx + TW - 1) / TW;
    const int tile = work / nchb, c0 = (work % nchb) * CB;
    const int split = threadIdx.x % NSPLIT;
    const int slot = threadIdx.x / NSPLIT;
    const int p = (tile % tiles_x) * TW + slot % TW;
    const int q = (tile / tiles_x) * TH + slot / TW;
    const bool inside = p < g.nx && q < g.ny;
    float I[CB], Tr[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) { I[c] = 0.0f; Tr[c] = 1.0f; }
    // ray set-up: chord through the bounding sphere, midpoint at s = 0
    const Chord3 cr = chord3(g, inside ? p : 0, inside ? q : 0);
    if (inside && cr.h2 > 0.0f) {
        const float ds = 2.0f * sqrtf(cr.h2) / (float)g.nsamp;
        const float pxr = cr.xp, pmy = cr.yp * g.ci, pmz = cr.yp * g.si;
        const float wy = g.si, wz = -g.ci;
        const float half = 0.5f * (float)g.nsamp;
        const int len = (g.nsamp + NSPLIT - 1) / NSPLIT;
        const int k0 = split * len;
        const int k1 = min(g.nsamp, k0 + len);
        for (int k = k0; k < k1; ++k) {
            const float t = ((float)k + 0.5f - half) * ds;
            const SampleQ sq = shade3(s, ztab, pxr, fmaf(t, wy, pmy), fmaf(t, wz, pmz), ds);
            // no ray of the wave with opacity at this sample: no channel changes
            if (__ballot(sq.K > 0.0f) == 0) continue;
            march_sample<CB, true>(I, Tr, sq, [&](int c) { return ch.v[c0 + c]; });
        }
    }
#pragma unroll
    for (int d = 1; d < NSPLIT; d <<= 1) {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const float Ib = __shfl_down(I[c], d, NSPLIT);
            const float Tb = __shfl_down(Tr[c], d, NSPLIT);
            if ((split & (2 * d - 1)) == 0) {
                I[c] = fmaf(Tr[c], Ib, I[c]);
                Tr[c] *= Tb;
            }
        }
    }
    if (!inside || split != 0) return;
    const size_t pix = (size_t)q * g.nx + p;
#pragma unroll
    for (int c = 0; c < CB; ++c)
        if (c0 + c < ch.n) cube[(size_t)(c0 + c) * ch_stride + pix] = I[c];
}

template <int CB, int NSPLIT>
static hipError_t launch3_t(const Geometry3 &g, const Shade3 &s, const Channels &ch, float *cube, hipStream_t st) {
    constexpr int TW = NSPLIT <= 2 ? 16 : 8;
    constexpr int TH = 256 / NSPLIT / TW;
    const int tiles = ((g.nx + TW - 1) / TW) * ((g.ny + TH - 1) / TH);
    const int nchb = (ch.n + CB - 1) / CB;
    const long nwork = (long)tiles * nchb;
    if (nwork > (1L << 30)) return hipErrorInvalidValue;
    const int per_xcd = (int)((nwork + 7) / 8);
    hipLaunchKernelGGL((march3_fwd<CB, NSPLIT>), dim3(8 * per_xcd), dim3(256), 0, st, g, s, ch, cube, g.nx * g.ny,
                       nchb, (int)nwork, per_xcd);
    return hipGetLastError();
}

template <int CB>
static hipError_t launch3_cb(const Geometry3 &g, const Shade3 &s, const Channels &ch, float *cube, int nsplit,
                             hipStream_t st) {
    switch (nsplit) {
    case 1: return launch3_t<CB, 1>(g, s, ch, cube, st);
    case 2: return launch3_t<CB, 2>(g, s, ch, cube, st);
    case 4: return launch3_t<CB, 4>(g, s, ch, cube, st);
    case 8: return launch3_t<CB, 8>(g, s, ch, cube, st);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_forward3(const Geometry3 &g, const Shade3 &s, const Channels &ch, float *cube, int cb,
                                  int nsplit, hipStream_t st) {
    switch (cb) {
    case 8: return launch3_cb<8>(g, s, ch, cube, nsplit, st);
    case 16: return launch3_cb<16>(g, s, ch, cube, nsplit, st);
    case 24: return launch3_cb<24>(g, s, ch, cube, nsplit, st);
    case 32: return launch3_cb<32>(g, s, ch, cube, nsplit, st);
    case 48: return launch3_cb<48>(g, s, ch, cube, nsplit, st);
    case 64: return launch3_cb<64>(g, s, ch, cube, nsplit, st);
    default: return hipErrorInvalidValue;
    }
}

// Six planes [nr][nt][np] -> interleaved records; NULL velocity planes are zero.
__global__ __launch_bounds__(256) void pack3(const float *__restrict__ ln_n, const float *__restrict__ temp,
                                             const float *__restrict__ xco, const float *__restrict__ vr,
                                             const float *__restrict__ vt, const float *__restrict__ vp,
                                             float4 *__restrict__ node, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        node[2 * (size_t)i] = make_float4(ln_n[i], temp[i], xco[i], vr ? vr[i] : 0.0f);
        node[2 * (size_t)i + 1] = make_float4(vt ? vt[i] : 0.0f, vp ? vp[i] : 0.0f, 0.0f, 0.0f);
    }
}

constexpr double kPI3 = 3.14159265358979323846;
constexpr int64_t kMaxNodes3 = (int64_t)1 << 28;

// 1 / r_i^2 of the radial nodes, in double then rounded once, kept per
// (device, grid) for the life of the process like the partition table.
static rt_status radius_table(const rt_grid3d &g, const float **out) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, double, double>, float *> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    const auto key = std::make_tuple(dev, (int)g.nr, g.r_min_au, g.r_max_au);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) { *out = it->second; return RT_OK; }
    std::vector<float> tab(g.nr);
    const double dln = std::log(g.r_max_au / g.r_min_au) / (g.nr - 1);
    for (int i = 0; i < g.nr; ++i) {
        const double r = g.r_min_au * std::exp(i * dln);
        tab[i] = (float)(1.0 / (r * r));
    }
    float *d = nullptr;
    e = hipMalloc(&d, sizeof(float) * g.nr);
    if (e != hipSuccess) return fail_hip(e, "hipMalloc(radius table)");
    e = hipMemcpy(d, tab.data(), sizeof(float) * g.nr, hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(d); return fail_hip(e, "hipMemcpy(radius table)"); }
    cache[key] = d;
    *out = d;
    return RT_OK;
}

// Launch shape of the 3-D march.  Its shading (two atan2, sixteen scattered
// loads, the physics) costs ~25 channels' worth of issue slots per sample, so
// a pixel's channels stay in one block (the smallest of 8..64 holding them,
// never split into two 32-channel blocks as the axisymmetric march does).
// Two lanes per ray (two half-chords in flight per pixel) were best at every
// image size measured; rays split further only while the launch stays at or
// under 1024 waves.  Measured on the 512 x 96 x 256 grid (ms): 256^2 x 20 ch
// (24, 2) 0.75 against (24, 4) 0.85; 256^2 x 64 (64, 2) 1.00 against (32, 2)
// 1.52; 256^2 x 128 (64, 2) 1.89 against (32, 1) 2.96; 512^2 x 20 (24, 2)
// 2.17 against (24, 1) 2.38; 128^2 x 20 (24, 4) 0.33 against (24, 8) 0.37.
static void forward_shape3(int nch, long npix, int nsamp, int *cb_out, int *split_out) {
    static const int cands[] = {8, 16, 24, 32, 48, 64};
    int cb = 64;
    for (int c : cands)
        if (c >= nch) { cb = c; break; }
    auto waves = [&](int ns) { return ((npix * ns + 63) / 64) * (long)((nch + cb - 1) / cb); };
    int ns = nsamp >= 128 ? 2 : 1;
    while (ns < 8 && waves(2 * ns) <= 1024 && nsamp >= 128 * ns) ns <<= 1;
    *cb_out = cb;
    *split_out = ns;
}

// camera and bounding sphere of a 3-D problem
static Geometry3 geometry3(const rt_problem3d *p) {
    const rt_grid3d &gr = p->grid;
    const double dln = std::log(gr.r_max_au / gr.r_min_au) / (gr.nr - 1);
    const double ang = p->cam.incl_deg * kPI3 / 180.0, pa = p->cam.pa_deg * kPI3 / 180.0;
    Geometry3 g;
    std::memset(&g, 0, sizeof g);
    g.d_pix = p->cam.fov_au / p->cam.nx;
    g.cpa = std::cos(pa);
    g.spa = std::sin(pa);
    g.si = std::sin(ang);
    g.ci = std::cos(ang);
    if (p->cam.incl_deg == 0.0) { g.si = 0.0; g.ci = 1.0; }
    if (p->cam.incl_deg == 90.0) { g.si = 1.0; g.ci = 0.0; }
    if (p->cam.incl_deg == 180.0) { g.si = 0.0; g.ci = -1.0; }
    const double rc = gr.r_max_au * std::exp(dln);
    g.rc2 = rc * rc;
    g.xc = 0.5 * p->cam.nx;
    g.yc = 0.5 * p->cam.ny;
    g.nx = p->cam.nx;
    g.ny = p->cam.ny;
    g.nsamp = p->nsamp;
    return g;
}

// Rays of a 3-D render that cross the bounding sphere (the march's own
// test) and, with shade, their pixel-samples that are thin in the march's
// sense, that have any opacity, and that lie inside the grid's fade (the
// march's own shading).  blockIdx.y: a chunk of the samples of each ray.
__global__ __launch_bounds__(256) void census3(Geometry3 g, Shade3 s, uint8_t *__restrict__ mask,
                                               unsigned long long *__restrict__ counts, int shade) {
    __shared__ float4 ztab[kZTableNodes - 1];
    __shared__ unsigned long long part[4];
    if (shade)
        for (int i = threadIdx.x; i < kZTableNodes - 1; i += blockDim.x) ztab[i] = s.ztab[i];
    if (threadIdx.x < 4) part[threadIdx.x] = 0ull;
    __syncthreads();
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix < g.nx * g.ny) {
        const int p = pix % g.nx, q = pix / g.nx;
        const Chord3 cr = chord3(g, p, q);
        const bool live = cr.h2 > 0.0f;
        if (blockIdx.y == 0) {
            if (mask) mask[pix] = live ? 1 : 0;
            if (live) atomicAdd(&part[0], 1ull);
        }
        if (live && shade) {
            const float ds = 2.0f * sqrtf(cr.h2) / (float)g.nsamp;
            const float pmy = cr.yp * g.ci, pmz = cr.yp * g.si, wy = g.si, wz = -g.ci;
            const float half = 0.5f * (float)g.nsamp;
            const int len = (g.nsamp + gridDim.y - 1) / gridDim.y;
            const int k0 = blockIdx.y * len, k1 = min(g.nsamp, k0 + len);
            unsigned thin = 0, emit = 0, inside = 0;
            for (int k = k0; k < k1; ++k) {
                const float t = ((float)k + 0.5f - half) * ds;
                const SampleQ sq = shade3(s, ztab, cr.xp, fmaf(t, wy, pmy), fmaf(t, wz, pmz), ds);
                thin += sq.K < kThinK ? 1u : 0u;
                emit += sq.K > 0.0f ? 1u : 0u;
                inside += sq.b > 0.0f ? 1u : 0u;   // b = 0 only for a sample beyond the fade
            }
            if (thin) atomicAdd(&part[1], (unsigned long long)thin);
            if (emit) atomicAdd(&part[2], (unsigned long long)emit);
            if (inside) atomicAdd(&part[3], (unsigned long long)inside);
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 && part[threadIdx.x]) atomicAdd(counts + threadIdx.x, part[threadIdx.x]);
}

__global__ void census3_zero(unsigned long long *c) {
    if (threadIdx.x < 4) c[threadIdx.x] = 0ull;
}

static rt_status validate_grid3(const rt_grid3d *g) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (g->nr < 2 || g->nt < 2 || g->np < 1)
        return fail(RT_EINVAL, "grid needs nr >= 2, nt >= 2, np >= 1 (got %d, %d, %d)", g->nr, g->nt, g->np);
    if ((int64_t)g->nr * g->nt * g->np > kMaxNodes3) return fail(RT_EINVAL, "grid has more than 2^28 nodes");
    if (!(std::isfinite(g->r_min_au) && std::isfinite(g->r_max_au) && g->r_min_au > 0 && g->r_max_au > g->r_min_au))
        return fail(RT_EINVAL, "need 0 < r_min_au < r_max_au");
    if (!(std::isfinite(g->th_min) && std::isfinite(g->th_max) && g->th_min >= 0 && g->th_max > g->th_min &&
          g->th_max <= kPI3))
        return fail(RT_EINVAL, "need 0 <= th_min < th_max <= pi");
    return RT_OK;
}

// Shading constants of a 3-D problem (grid, line, camera): shared by the
// render and its census.  Needs the validated problem.
static rt_status build_shade3(const rt_problem3d *p, Shade3 *s) {
    rt_status st = RT_OK;
    const rt_grid3d &gr = p->grid;
    const rt_line &l = p->line;
    const float4 *tab = nullptr;
    st = partition_table(l, &tab);
    if (st != RT_OK) return st;
    constexpr double kH = 6.62607015e-27, kKB = 1.380649e-16, kC = 2.99792458e10, kAMU = 1.66053906660e-24,
                     kAU = 1.495978707e13, kZT0 = 0.1, kZT1 = 1.0e4;
    const double dln = std::log(gr.r_max_au / gr.r_min_au) / (gr.nr - 1);
    const double dth = (gr.th_max - gr.th_min) / (gr.nt - 1);
    const Geometry3 g = geometry3(p);
    std::memset(s, 0, sizeof *s);
    s->node = (const float4 *)p->nodes;
    s->ztab = tab;
    s->nr = gr.nr;
    s->nt = gr.nt;
    s->np = gr.np;
    const float *inv_r2n = nullptr;
    st = radius_table(gr, &inv_r2n);
    if (st != RT_OK) return st;
    s->inv_r2n = inv_r2n;
    s->u_scale = (float)(std::log(2.0) / dln);
    s->h_r = (float)(0.5 * std::log(2.0) / dln);
    s->log2_rmin = (float)std::log2(gr.r_min_au);
    const double thc = 0.5 * (gr.th_min + gr.th_max);
    s->cth_c = (float)std::cos(thc);
    s->sth_c = (float)std::sin(thc);
    s->inv_dth = (float)(1.0 / dth);
    s->half_nt1 = 0.5f * (float)(gr.nt - 1);
    s->inv_dph = (float)(gr.np / (2.0 * kPI3));
    s->fnp = (float)gr.np;
    s->fnr = (float)gr.nr;
    s->fnt = (float)gr.nt;
    const double l0 = std::log2(kZT0), l1 = std::log2(kZT1), log2e = 1.0 / std::log(2.0);
    s->zt_l2t0 = (float)l0;
    s->zt_scale = (float)((kZTableNodes - 1) / (l1 - l0));
    s->el_log2e = (float)(l.e_l_k * log2e);
    const double nu = l.nu0_hz;
    s->theta = (float)(kH * nu / kKB);
    s->c_s = (float)(p->intensity_scale * 2.0 * kH * nu * nu * nu / (kC * kC));
    const double bul = l.a_ul * kC * kC / (2.0 * kH * nu * nu * nu);
    const double blu = l.g_u / l.g_l * bul;
    s->c_k = (float)((kH * nu / (4.0 * kPI3)) * blu * l.g_l * (kC / nu) * kAU / (std::sqrt(kPI3) * 1e5) * log2e);
    s->c_alpha = (float)((2.0 * kKB / (l.m_co_amu * kAMU) + p->v_turb * p->v_turb * 2.0 * kKB / (l.m_mol_amu * kAMU)) /
                        1e10);
    s->sqrt_log2e = (float)std::sqrt(log2e);
    s->si = (float)g.si;
    s->ci = (float)g.ci;
    s->vsys = (float)p->spec.v_sys_kms;
    return RT_OK;
}

} // namespace rt

using namespace rt;

extern "C" {

rt_status rt_pack_fields3d(const rt_grid3d *grid, const float *ln_nh2, const float *temp_k, const float *x_co,
                           const float *v_r, const float *v_theta, const float *v_phi, float *nodes, void *stream) {
    rt_status st = validate_grid3(grid);
    if (st != RT_OK) return st;
    if (!ln_nh2 || !temp_k || !x_co) return fail(RT_EINVAL, "ln_nh2, temp_k and x_co are required");
    if (!nodes) return fail(RT_EINVAL, "nodes is NULL");
    if (((uintptr_t)nodes & 15) != 0) return fail(RT_EINVAL, "nodes must be 16-byte aligned");
    const uint32_t n = (uint32_t)((int64_t)grid->nr * grid->nt * grid->np);
    const unsigned blocks = (unsigned)std::min<uint32_t>((n + 255) / 256, 16384u);
    hipLaunchKernelGGL(pack3, dim3(blocks), dim3(256), 0, (hipStream_t)stream, ln_nh2, temp_k, x_co, v_r, v_theta,
                       v_phi, (float4 *)nodes, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RT_OK : fail_hip(e, "pack launch");
}

rt_status rt_render_census_3d(const rt_problem3d *p, uint8_t *mask, int64_t *counts, void *stream) {
    if (!p) return fail(RT_EINVAL, "problem is NULL");
    rt_status st = validate_grid3(&p->grid);
    if (st != RT_OK) return st;
    st = validate_view(p->line, p->cam, p->spec, p->nsamp, p->intensity_scale, 180.0);
    if (st != RT_OK) return st;
    if (!counts) return fail(RT_EINVAL, "counts is NULL");
    const Geometry3 g = geometry3(p);
    // the shading counts need the node records
    const int shade = p->nodes && ((uintptr_t)p->nodes & 15) == 0 ? 1 : 0;
    Shade3 s;
    std::memset(&s, 0, sizeof s);
    if (shade && (st = build_shade3(p, &s)) != RT_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e;
    unsigned long long *d = (unsigned long long *)stream_workspace(hs, kWsCensus, 4 * sizeof(unsigned long long), &e);
    if (!d) return fail_hip(e, "census counters");
    const int npix = p->cam.nx * p->cam.ny;
    int chunks = 1;
    while (shade && chunks < 64 && (long)((npix + 255) / 256) * chunks < 4096 && p->nsamp >= 16 * chunks) chunks *= 2;
    hipLaunchKernelGGL(census3_zero, dim3(1), dim3(64), 0, hs, d);
    hipLaunchKernelGGL(census3, dim3((npix + 255) / 256, chunks), dim3(256), 0, hs, g, s, mask, d, shade);
    unsigned long long h[4] = {0, 0, 0, 0};
    if ((e = hipGetLastError()) == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return fail_hip(e, "3-D census");
    counts[0] = (int64_t)h[0];
    counts[1] = (int64_t)h[0] * p->nsamp;
    counts[2] = shade ? (int64_t)h[1] : -1;
    counts[3] = shade ? (int64_t)h[2] : -1;
    counts[4] = shade ? (int64_t)h[3] : -1;
    return RT_OK;
}

rt_status rt_render_cube_3d(const rt_problem3d *p, float *cube, void *stream) {
    if (!p) return fail(RT_EINVAL, "problem is NULL");
    rt_status st = validate_grid3(&p->grid);
    if (st != RT_OK) return st;
    if (!p->nodes) return fail(RT_EINVAL, "nodes is NULL");
    if (((uintptr_t)p->nodes & 15) != 0) return fail(RT_EINVAL, "nodes must be 16-byte aligned");
    if (!(std::isfinite(p->v_turb) && p->v_turb >= 0)) return fail(RT_EINVAL, "need v_turb >= 0");
    st = validate_view(p->line, p->cam, p->spec, p->nsamp, p->intensity_scale, 180.0);
    if (st != RT_OK) return st;
    if (!cube) return fail(RT_EINVAL, "cube is NULL");
    Shade3 s;
    st = build_shade3(p, &s);
    if (st != RT_OK) return st;
    const Geometry3 g = geometry3(p);
    int cb, nsplit;
    forward_shape3(std::min(p->spec.nch, kLaunchChannels), (long)p->cam.nx * p->cam.ny, p->nsamp, &cb, &nsplit);
    if (channel_block_option()) cb = channel_block_option();
    if (ray_split_option()) nsplit = ray_split_option();
    const size_t plane = (size_t)p->cam.nx * p->cam.ny;
    for (int c0 = 0; c0 < p->spec.nch; c0 += kLaunchChannels) {
        Channels ch;
        std::memset(&ch, 0, sizeof ch);
        ch.n = std::min(kLaunchChannels, p->spec.nch - c0);
        for (int c = 0; c < ch.n; ++c) ch.v[c] = (float)p->spec.v_kms[c0 + c];
        const hipError_t e = launch_forward3(g, s, ch, cube + (size_t)c0 * plane, cb, nsplit, (hipStream_t)stream);
        if (e != hipSuccess) return fail_hip(e, "3-D forward launch");
    }
    return RT_OK;
}

} // extern "C"
