// rt_forward.hip -- forward ray march for gfx950.
//
// One lane = one pixel x one block of CB channels; a workgroup of 256 lanes
// covers a 16 x 16 pixel tile; blockIdx.y selects the channel block, so the
// channel velocities of a wave are uniform and live in scalar registers.
// Per sample the lane evaluates the channel-independent shading once (grid
// fetch, density, CO mask, LTE populations, source function, line width,
// projected velocity) and then runs the channel loop entirely in registers:
// profile, optical depth, front-to-back accumulation of I and transmission.
// Every sample of a ray is shaded; a sample with no opacity (K = 0: outside
// the CO layer or the grid) changes no channel, so a wave skips the channel
// loop of a sample where none of its rays has opacity there (a ballot over
// the lanes marching).  The cube is the same either way.
#include <type_traits>

#include "rt_kernels.h"
#include "rt_launch.h"

namespace rt {

// Lane layout: a workgroup of 256 lanes covers a tile of 256 / NSPLIT pixels;
// the NSPLIT adjacent lanes of a pixel march consecutive sub-chords of its
// ray (samples [split L, (split+1) L)).  Front-to-back composition is
// associative -- (I, Tr) of segment A followed by B is (I_A + Tr_A I_B,
// Tr_A Tr_B) -- so the sub-chord results are combined by shuffles at the end.
template <int CB, bool THIN, int NSPLIT, bool NEURAL>
__global__ __launch_bounds__(256) void march_fwd(Geometry g, Shade s, Channels ch, float *__restrict__ cube,
                                                  int ch_stride) {
    __shared__ float4 ztab[kZTableNodes - 1];
    stage_ztab(s, ztab);
    constexpr int TW = NSPLIT <= 2 ? 16 : 8;          // tile width in pixels
    constexpr int TH = 256 / NSPLIT / TW;             // tile height
    const int tiles_x = (g.nx + TW - 1) / TW;
    const int split = threadIdx.x % NSPLIT;
    const int slot = threadIdx.x / NSPLIT;
    const int p = (blockIdx.x % tiles_x) * TW + slot % TW;
    const int q = (blockIdx.x / tiles_x) * TH + slot / TW;
    const int c0 = blockIdx.y * CB;
    const bool inside = p < g.nx && q < g.ny;
    float I[CB], Tr[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) { I[c] = 0.0f; Tr[c] = 1.0f; }
    const RaySetup r = ray_setup(g, inside ? p : 0, inside ? q : 0);
    if (inside && r.live) {
        const float half = 0.5f * (float)g.nsamp;
        const int len = (g.nsamp + NSPLIT - 1) / NSPLIT;
        const int k0 = split * len;
        const int k1 = min(g.nsamp, k0 + len);
        for (int k = k0; k < k1; ++k) {
            const float t = ((float)k + 0.5f - half) * r.ds;
            const SampleQ sq = shade_sample<NEURAL>(s, ztab, r.px, fmaf(t, r.wy, r.pmy), fmaf(t, r.wz, r.pmz), r.ds,
                                            o_index(s, k, q * g.nx + p));
            if (__ballot(sq.K > 0.0f) == 0) continue;
            march_sample<CB, THIN>(I, Tr, sq, [&](int c) { return ch.v[c0 + c]; });
        }
    }
    // compose the sub-chords front to back: pairs, then pairs of pairs, ...
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

// Lane j of this lane's group of G (2 or 4) adjacent lanes: a DPP quad
// permutation that gives every lane of the group the value of its member j.
template <int G, int J>
__device__ __forceinline__ float group_lane(float x) {
    constexpr int sel = G == 4 ? J * 0x55 : (J == 0 ? 0xA0 : 0xF5);   // (j,j,j,j) or (j,j,2+j,2+j)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), sel, 0xF, 0xF, false));
}

// Grouped-lane march of one 64-channel block: G adjacent lanes share one
// pixel, lane h holding channels c0 + h CB ... c0 + h CB + CB - 1 (CB =
// 64 / G) in registers.  Each lane shades one of every G consecutive samples
// (lane h sample k + h), and the group passes the shadings (S, log2 K, a, b
// and the thin-sample decision) around by DPP.  Each sample is still shaded
// once for all 64 channels, while a lane carries 1/G of the state of a
// 64-channel lane: 4 waves per SIMD at G = 2 and 7 at G = 4, against 3.
// Lane h's velocities must be lane 0's plus h `shift` (uniform channel
// spacing): the channel velocities stay wave-uniform scalars, and lane h
// folds its offset into a, since d_c = a - (v_c + h shift) b = (a - h shift b)
// - v_c b.
template <int G, bool THIN, bool NEURAL>
__global__ __launch_bounds__(256) void march_fwd_group(Geometry g, Shade s, Channels ch, float shift,
                                                        float *__restrict__ cube, int ch_stride) {
    __shared__ float4 ztab[kZTableNodes - 1];
    stage_ztab(s, ztab);
    constexpr int CB = 64 / G, TW = G == 2 ? 16 : 8, TH = 256 / G / TW;
    const int tiles_x = (g.nx + TW - 1) / TW;
    const int h = threadIdx.x % G;
    const int slot = threadIdx.x / G;
    const int p = (blockIdx.x % tiles_x) * TW + slot % TW;
    const int q = (blockIdx.x / tiles_x) * TH + slot / TW;
    const int c0 = blockIdx.y * 64;
    const bool inside = p < g.nx && q < g.ny;
    float I[CB], Tr[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) { I[c] = 0.0f; Tr[c] = 1.0f; }
    const RaySetup r = ray_setup(g, inside ? p : 0, inside ? q : 0);
    // the lanes of a group take this branch together (same pixel)
    if (inside && r.live) {
        const float half = 0.5f * (float)g.nsamp;
        const float vsh = (float)h * shift;
        const int pix = q * g.nx + p;
        auto vel = [&](int c) { return ch.v[c0 + c]; };
        for (int k = 0; k < g.nsamp; k += G) {
            const int kk = min(k + h, g.nsamp - 1);
            const float t = ((float)kk + 0.5f - half) * r.ds;
            const SampleQ own = shade_sample<NEURAL>(s, ztab, r.px, fmaf(t, r.wy, r.pmy), fmaf(t, r.wz, r.pmz), r.ds,
                                                     o_index(s, kk, pix));
            // the owner's log2 K and thin-sample decision travel with the shading
            const float own_lk = flog2(own.K);
            const float own_thin = own.K < kThinK ? 1.0f : 0.0f;
            auto step = [&](auto jc) {
                constexpr int J = decltype(jc)::value;
                const float S = group_lane<G, J>(own.S), lK = group_lane<G, J>(own_lk);
                const float b = group_lane<G, J>(own.b);
                const float a = fmaf(-vsh, b, group_lane<G, J>(own.a));
                const bool thin = group_lane<G, J>(own_thin) != 0.0f;
                // the wave skips the step when none of its rays has opacity
                // at it (a ballot counts only the lanes marching)
                const bool any = __ballot(lK > -__builtin_huge_valf()) != 0;
                if (any && (J == 0 || k + J < g.nsamp)) march_lk<CB, THIN>(I, Tr, S, lK, a, b, thin, vel);
            };
            step(std::integral_constant<int, 0>{});
            step(std::integral_constant<int, 1>{});
            if constexpr (G == 4) {
                step(std::integral_constant<int, 2>{});
                step(std::integral_constant<int, 3>{});
            }
        }
    }
    if (!inside) return;
    const size_t pix = (size_t)q * g.nx + p;
    const int cl = c0 + h * CB;
#pragma unroll
    for (int c = 0; c < CB; ++c)
        if (cl + c < ch.n) cube[(size_t)(cl + c) * ch_stride + pix] = I[c];
}

template <int CB, bool THIN, int NSPLIT>
static hipError_t launch_t(const Geometry &g, const Shade &s, const Channels &ch, float *cube, hipStream_t st) {
    constexpr int TW = NSPLIT <= 2 ? 16 : 8;
    constexpr int TH = 256 / NSPLIT / TW;
    const int tiles = ((g.nx + TW - 1) / TW) * ((g.ny + TH - 1) / TH);
    dim3 grid(tiles, (ch.n + CB - 1) / CB);
    if (s.mlp_o)
        hipLaunchKernelGGL((march_fwd<CB, THIN, NSPLIT, true>), grid, dim3(256), 0, st, g, s, ch, cube, g.nx * g.ny);
    else
        hipLaunchKernelGGL((march_fwd<CB, THIN, NSPLIT, false>), grid, dim3(256), 0, st, g, s, ch, cube, g.nx * g.ny);
    return hipGetLastError();
}

template <int CB, bool THIN>
static hipError_t launch_split(const Geometry &g, const Shade &s, const Channels &ch, float *cube, int nsplit,
                               hipStream_t st) {
    switch (nsplit) {
    case 1: return launch_t<CB, THIN, 1>(g, s, ch, cube, st);
    case 2: return launch_t<CB, THIN, 2>(g, s, ch, cube, st);
    case 4: return launch_t<CB, THIN, 4>(g, s, ch, cube, st);
    case 8: return launch_t<CB, THIN, 8>(g, s, ch, cube, st);
    default: return hipErrorInvalidValue;
    }
}

template <int CB>
static hipError_t launch_cb(const Geometry &g, const Shade &s, const Channels &ch, float *cube, bool thin, int nsplit,
                            hipStream_t st) {
    return thin ? launch_split<CB, true>(g, s, ch, cube, nsplit, st) : launch_split<CB, false>(g, s, ch, cube, nsplit, st);
}

hipError_t launch_forward(const Geometry &g, const Shade &s, const Channels &ch, float *cube, int cb, bool thin,
                          int nsplit, hipStream_t st) {
    switch (cb) {
    case 8: return launch_cb<8>(g, s, ch, cube, thin, nsplit, st);
    case 16: return launch_cb<16>(g, s, ch, cube, thin, nsplit, st);
    case 24: return launch_cb<24>(g, s, ch, cube, thin, nsplit, st);
    case 32: return launch_cb<32>(g, s, ch, cube, thin, nsplit, st);
    case 48: return launch_cb<48>(g, s, ch, cube, thin, nsplit, st);
    case 64: return launch_cb<64>(g, s, ch, cube, thin, nsplit, st);
    default: return hipErrorInvalidValue;
    }
}

template <int G>
static hipError_t launch_group_t(const Geometry &g, const Shade &s, const Channels &ch, float *cube, bool thin,
                                 float shift, hipStream_t st) {
    constexpr int TW = G == 2 ? 16 : 8, TH = 256 / G / TW;
    const int tiles = ((g.nx + TW - 1) / TW) * ((g.ny + TH - 1) / TH);
    dim3 grid(tiles, (ch.n + 63) / 64);
    const int cs = g.nx * g.ny;
    if (s.mlp_o) {
        if (thin) hipLaunchKernelGGL((march_fwd_group<G, true, true>), grid, dim3(256), 0, st, g, s, ch, shift, cube, cs);
        else hipLaunchKernelGGL((march_fwd_group<G, false, true>), grid, dim3(256), 0, st, g, s, ch, shift, cube, cs);
    } else {
        if (thin) hipLaunchKernelGGL((march_fwd_group<G, true, false>), grid, dim3(256), 0, st, g, s, ch, shift, cube, cs);
        else hipLaunchKernelGGL((march_fwd_group<G, false, false>), grid, dim3(256), 0, st, g, s, ch, shift, cube, cs);
    }
    return hipGetLastError();
}

hipError_t launch_forward_group(const Geometry &g, const Shade &s, const Channels &ch, float *cube, bool thin,
                                int lanes, float shift, hipStream_t st) {
    switch (lanes) {
    case 2: return launch_group_t<2>(g, s, ch, cube, thin, shift, st);
    case 4: return launch_group_t<4>(g, s, ch, cube, thin, shift, st);
    default: return hipErrorInvalidValue;
    }
}

} // namespace rt
