// rt_kernels.h -- device-side argument blocks and shared math of the ray
// march kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rt {

// channels carried in one launch's kernel arguments
constexpr int kLaunchChannels = 256;
// partition-function table: nodes uniform in log2 T over [log2 0.1, log2 1e4]
constexpr int kZTableNodes = 512;
constexpr float kLog2E = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Per-launch geometry.  Everything, the per-ray set-up included, is float.
struct Geometry {
    float d_pix;             // pixel size [au]
    float cpa, spa;          // position-angle rotation
    float si, ci;            // sin / cos inclination (0 and 1 exactly face-on, 1 and 0 edge-on)
    float rc, zc;            // bounding cylinder radius and half height [au]
    float xc, yc;            // image centre in pixels from the first column / row of this launch
    int32_t nx, ny, nsamp;   // pixels of this launch (a band of rows of the image when chunked)
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
    float zr_max;            // (z/r) of the top grid row
    const float4 *mlp_o;     // neural CO layer outputs [nsamp][image pixels] (o0, o1, o2, -); NULL = grid surfaces
    int64_t o_plane, o_pix0; // output of sample k, pixel pix of the launch: mlp_o[k o_plane + o_pix0 + pix]
};

// index of a launch's (sample, pixel) in the image-wide network outputs
__device__ __forceinline__ size_t o_index(const Shade &s, int k, int pix) {
    return (size_t)k * (size_t)s.o_plane + (size_t)s.o_pix0 + (size_t)pix;
}

// Velocities of one launch's channels.  A kernel's last channel block may
// extend past n (and past kLaunchChannels, e.g. 11 blocks of 24 for 256
// channels); those padding lanes read the zeros after the n velocities, so
// the array runs one largest block (64) beyond kLaunchChannels.  Filled by
// the host after zeroing the whole struct.
struct Channels {
    int32_t n;               // channels in this launch
    int32_t pad_;
    float v[kLaunchChannels + 64];
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

// Optically thin samples.  1 - fl(2^-x) keeps only about ulp(1) / (x ln 2)
// of its relative precision (at x ln 2 = 1e-4 the fourth digit; below
// x ~ 1e-7 it is 0), so a sample whose line-centre depth K is below kThinK
// takes 1 - 2^-x from its series in y = x ln 2 through y^3 for every channel
// (each channel's x <= K; truncation y^4/24, so at most 1.3e-6 relative at
// y = 1/32), while thicker samples keep 1 - 2^-x, accurate to 2e-6 relative
// at the threshold and better above.  The series needs one exp2 fewer per
// channel than the direct form.
constexpr float kThinK = 0.04508422002825536f;   // y = 1/32
__device__ __forceinline__ float om_series3(float x) {
    constexpr float c1 = 0.6931471805599453f;      //  ln2
    constexpr float c2 = -0.2402265069591007f;     // -ln2^2/2
    constexpr float c3 = 0.05550410866482158f;     //  ln2^3/6
    return fmaf(fmaf(c3, x, c2), x, c1) * x;
}

// Z(T) by cubic Hermite interpolation of the table in log2 T (tab: the
// table in global memory or its copy in LDS).
__device__ __forceinline__ float partition_fn(const Shade &s, const float4 *tab, float log2t) {
    float t = (log2t - s.zt_l2t0) * s.zt_scale;
    t = clampf(t, 0.0f, (float)(kZTableNodes - 1));
    int i = (int)t;
    i = i > kZTableNodes - 2 ? kZTableNodes - 2 : i;
    const float f = t - (float)i;
    const float4 n = tab[i];
    const float g = 1.0f - f;
    const float h00 = (1.0f + 2.0f * f) * g * g;
    const float h10 = f * g * g;
    const float h01 = f * f * (3.0f - 2.0f * f);
    const float h11 = -f * f * g;
    return h00 * n.x + h10 * n.y + h01 * n.z + h11 * n.w;
}

// ---------------------------------------------------------------- rays and shading
struct RaySetup {
    float px, pmy, pmz;  // image-plane x' and the chord midpoint (y, z)
    float ds;            // segment length [au]
    float wy, wz;        // ray direction (y, z) components
    bool live;
};

// Chord of the ray through the bounding cylinder rho <= rc, |z| <= zc.  On
// the ray (x', y', s) the disk-frame position is x = x', y = y' ci + s si,
// z = y' si - s ci, so the cylinder keeps s within qq/si of s_c = -y' ci/si
// (qq^2 = rc^2 - x'^2) and the slab within zc/ci of s_z = y' si/ci.  The
// set-up is float and works relative to the chord's midpoint: when one
// constraint bounds both ends, the midpoint lies on its symmetry plane
// (y = 0 or z = 0) exactly, its other coordinate is y'/si or y'/ci (one
// rounding), and the chord length is 2 qq/si or 2 zc/ci, free of the
// cancellation in (s_c + h) - (s_c - h).  Chords cut by both constraints use
// the end points directly.
__device__ __forceinline__ RaySetup ray_setup(const Geometry &g, int p, int q) {
    RaySetup r;
    const float X = ((float)p + 0.5f - g.xc) * g.d_pix;
    const float Y = ((float)q + 0.5f - g.yc) * g.d_pix;
    const float xp = fmaf(g.cpa, X, -g.spa * Y);
    const float yp = fmaf(g.spa, X, g.cpa * Y);
    const float q2 = fmaf(-xp, xp, g.rc * g.rc);
    const float qq = sqrtf(fmaxf(q2, 0.0f));
    bool ok = q2 > 0.0f;
    const float inf = __builtin_huge_valf();
    float loc = -inf, hic = inf, loz = -inf, hiz = inf;
    if (g.si > 0.0f) {
        loc = fmaf(-yp, g.ci, -qq) / g.si;
        hic = fmaf(-yp, g.ci, qq) / g.si;
    } else {
        ok = ok && fabsf(yp * g.ci) <= qq;
    }
    if (g.ci > 0.0f) {
        loz = fmaf(yp, g.si, -g.zc) / g.ci;
        hiz = fmaf(yp, g.si, g.zc) / g.ci;
    } else {
        ok = ok && fabsf(yp * g.si) <= g.zc;
    }
    const bool cyl_lo = loc >= loz, cyl_hi = hic <= hiz;
    const float lo = cyl_lo ? loc : loz, hi = cyl_hi ? hic : hiz;
    ok = ok && hi > lo;
    float len, pmy, pmz;
    if (cyl_lo && cyl_hi) {            // both ends on the cylinder wall
        len = 2.0f * qq / g.si;
        pmy = 0.0f;
        pmz = yp / g.si;
    } else if (!cyl_lo && !cyl_hi) {   // both ends on the slab faces
        len = 2.0f * g.zc / g.ci;
        pmy = yp / g.ci;
        pmz = 0.0f;
    } else {
        const float sm = 0.5f * (lo + hi);
        len = hi - lo;
        pmy = fmaf(sm, g.si, yp * g.ci);
        pmz = fmaf(-sm, g.ci, yp * g.si);
    }
    r.px = xp;
    r.pmy = ok ? pmy : 0.0f;
    r.pmz = ok ? pmz : 0.0f;
    r.ds = ok ? len / (float)g.nsamp : 0.0f;
    r.wy = g.si;
    r.wz = -g.ci;
    r.live = ok;
    return r;
}

// Where a sample falls on the grid.
struct Locus {
    float rho, inv_rho, az;  // cylindrical radius, 1/rho, |z| [au]
    float u, v;              // continuous grid index (ln r, z/r); u = -2 on the axis
    float fu, fv;            // bilinear weights inside the clamped cell
    int i0, j0;              // clamped cell corner
    float taper;             // density fade one cell beyond the grid
};

__device__ __forceinline__ Locus locate(const Shade &s, float px, float py, float pz) {
    Locus L;
    const float rho2 = px * px + py * py;
    const bool on = rho2 > 0.0f;
    L.rho = fsqrt(rho2);
    L.inv_rho = on ? frcp(L.rho) : 0.0f;
    L.az = fabsf(pz);
    float u = (flog2(L.rho) - s.log2_rmin) * s.u_scale;
    float v = L.az * L.inv_rho * s.inv_dzr;
    u = on ? u : -2.0f;
    v = on ? v : 0.0f;
    L.u = u;
    L.v = v;
    const float uc = clampf(u, 0.0f, s.fnr - 1.0f);
    const float vc = clampf(v, 0.0f, s.fnz - 1.0f);
    int i0 = (int)uc;
    int j0 = (int)vc;
    L.i0 = i0 > s.nr - 2 ? s.nr - 2 : i0;
    L.j0 = j0 > s.nz - 2 ? s.nz - 2 : j0;
    L.fu = uc - (float)L.i0;
    L.fv = vc - (float)L.j0;
    L.taper = clampf(u + 1.0f, 0.0f, 1.0f) * clampf(s.fnr - u, 0.0f, 1.0f) * clampf(s.fnz - v, 0.0f, 1.0f);
    return L;
}

// Primary fields interpolated at the sample.
struct Fields {
    float ln_n, T, vphi, zlo, zup;
};

// The 16 grid values a sample reads (loaded ahead of their use).
struct Corners {
    float l00, l01, l10, l11, t00, t01, t10, t11, v00, v01, v10, v11, zl0, zl1, zu0, zu1;
};

__device__ __forceinline__ Corners load_corners(const Shade &s, const Locus &L) {
    const int n00 = L.i0 * s.nz + L.j0;
    const int n10 = n00 + s.nz;
    Corners c;
    c.l00 = s.ln_n[n00]; c.l01 = s.ln_n[n00 + 1]; c.l10 = s.ln_n[n10]; c.l11 = s.ln_n[n10 + 1];
    c.t00 = s.temp[n00]; c.t01 = s.temp[n00 + 1]; c.t10 = s.temp[n10]; c.t11 = s.temp[n10 + 1];
    c.v00 = s.vphi[n00]; c.v01 = s.vphi[n00 + 1]; c.v10 = s.vphi[n10]; c.v11 = s.vphi[n10 + 1];
    c.zl0 = s.zlo[L.i0]; c.zl1 = s.zlo[L.i0 + 1]; c.zu0 = s.zup[L.i0]; c.zu1 = s.zup[L.i0 + 1];
    return c;
}

__device__ __forceinline__ Fields interpolate(const Corners &c, const Locus &L) {
    const float fu = L.fu, fv = L.fv;
    const float l00 = c.l00, l01 = c.l01, l10 = c.l10, l11 = c.l11;
    const float t00 = c.t00, t01 = c.t01, t10 = c.t10, t11 = c.t11;
    const float v00 = c.v00, v01 = c.v01, v10 = c.v10, v11 = c.v11;
    const float zl0 = c.zl0, zl1 = c.zl1, zu0 = c.zu0, zu1 = c.zu1;
    Fields F;
    const float la = fmaf(fv, l01 - l00, l00), lb = fmaf(fv, l11 - l10, l10);
    F.ln_n = fmaf(fu, lb - la, la);
    const float ta = fmaf(fv, t01 - t00, t00), tb = fmaf(fv, t11 - t10, t10);
    F.T = fmaf(fu, tb - ta, ta);
    const float va = fmaf(fv, v01 - v00, v00), vb = fmaf(fv, v11 - v10, v10);
    F.vphi = fmaf(fu, vb - va, va);
    F.zlo = fmaf(fu, zl1 - zl0, zl0);
    F.zup = fmaf(fu, zu1 - zu0, zu0);
    return F;
}

__device__ __forceinline__ Fields fetch(const Shade &s, const Locus &L) { return interpolate(load_corners(s, L), L); }

__device__ __forceinline__ float sigmoidf_(float x) { return frcp(1.0f + fexp2(-x * kLog2E)); }
__device__ __forceinline__ float tanhf_(float x) { return 1.0f - 2.0f * frcp(1.0f + fexp2(2.0f * kLog2E * x)); }

// Neural CO layer: the network's outputs at the sample replace the two
// surfaces (z = zr_max rho sigma(o)) and scale the temperature by
// exp(0.5 tanh(o2)).
__device__ __forceinline__ void apply_mlp(const Shade &s, Fields &F, const Locus &L, float4 o) {
    F.zup = s.zr_max * L.rho * sigmoidf_(o.x);
    F.zlo = s.zr_max * L.rho * sigmoidf_(o.y);
    F.T *= fexp2(0.5f * kLog2E * tanhf_(o.z));
}

// Channel-independent quantities of one sample.
struct SampleQ {
    float S;     // source function (times intensity_scale)
    float K;     // optical depth of the segment at line centre (log2 units)
    float a, b;  // d_c = a - v_c b is (v_los - v_c)/alpha scaled by sqrt(log2 e)
};

// Intermediates the adjoint needs from the physics of one sample.
struct PhysTape {
    float rT, x, em1, Z, dZ;   // 1/T, h nu/kT, e^x - 1, Z(T), dZ/dlog2 T
    float sa, sb, iw;          // logistic factors of the two surface terms, mask scale
    float vfac;                // sin i * x' / rho
};

__device__ __forceinline__ float partition_fn_d(const Shade &s, const float4 *tab, float log2t, float *dz) {
    float t = (log2t - s.zt_l2t0) * s.zt_scale;
    const bool inside = t > 0.0f && t < (float)(kZTableNodes - 1);
    t = clampf(t, 0.0f, (float)(kZTableNodes - 1));
    int i = (int)t;
    i = i > kZTableNodes - 2 ? kZTableNodes - 2 : i;
    const float f = t - (float)i;
    const float4 n = tab[i];
    const float g = 1.0f - f;
    const float d00 = 6.0f * f * (f - 1.0f), d10 = g * (1.0f - 3.0f * f), d01 = -d00, d11 = f * (3.0f * f - 2.0f);
    *dz = inside ? (d00 * n.x + d10 * n.y + d01 * n.z + d11 * n.w) * s.zt_scale : 0.0f;
    const float h00 = (1.0f + 2.0f * f) * g * g;
    const float h10 = f * g * g;
    const float h01 = f * f * (3.0f - 2.0f * f);
    const float h11 = -f * f * g;
    return h00 * n.x + h10 * n.y + h01 * n.z + h11 * n.w;
}

template <bool TAPE>
__device__ __forceinline__ SampleQ physics(const Shade &s, const float4 *tab, const Locus &L, const Fields &F,
                                           float px, float ds, PhysTape *tp) {
    // density, fading to zero one cell beyond the grid
    const float n = fexp2(F.ln_n * kLog2E) * L.taper;
    // logistic CO mask between the two surfaces
    const float iw = s.inv_w * L.inv_rho;
    const float ea = fexp2((L.az - F.zup) * iw);
    const float eb = fexp2((F.zlo - L.az) * iw);
    const float ra = frcp(1.0f + ea), rb = frcp(1.0f + eb);
    const float mask = ra * rb;
    // LTE populations and source function
    const float rT = frcp(F.T);
    float dZ = 0.0f;
    const float Z = TAPE ? partition_fn_d(s, tab, flog2(F.T), &dZ) : partition_fn(s, tab, flog2(F.T));
    const float el = fexp2(-s.el_log2e * rT);
    const float x = fminf(s.theta * rT, 80.0f);
    const float em1 = expm1_pos(x);
    SampleQ q;
    q.S = s.c_s * frcp(em1);
    const float inv_alpha = frsq(F.T * s.c_alpha);
    q.K = s.c_k * n * mask * el * em1 * frcp(Z * (1.0f + em1)) * ds * inv_alpha;
    q.b = s.sqrt_log2e * inv_alpha;
    const float vfac = s.vrot * px * L.inv_rho;
    const float vlos = fmaf(F.vphi, vfac, s.vsys);
    q.a = vlos * q.b;
    if (TAPE) {
        tp->rT = rT; tp->x = x; tp->em1 = em1; tp->Z = Z; tp->dZ = dZ;
        // 1 - sigma of each surface term; e^A overflowing means the term is 1
        tp->sa = ea < 1e30f ? ea * ra : 1.0f;
        tp->sb = eb < 1e30f ? eb * rb : 1.0f;
        tp->iw = iw; tp->vfac = vfac;
    }
    return q;
}

template <bool NEURAL>
__device__ __forceinline__ SampleQ shade_sample(const Shade &s, const float4 *tab, float px, float py, float pz,
                                                float ds, size_t m) {
    const Locus L = locate(s, px, py, pz);
    // beyond the grid's edge taper (inside the bounding cylinder but above
    // the top z/r row, inside the inner radius or outside the outer one) the
    // density, and with it K, is exactly 0: no fetch, no physics
    if (L.taper <= 0.0f) {
        SampleQ z;
        z.S = 0.0f; z.K = 0.0f; z.a = 0.0f; z.b = 0.0f;
        return z;
    }
    Fields F = fetch(s, L);
    if (NEURAL) apply_mlp(s, F, L, s.mlp_o[m]);
    return physics<false>(s, tab, L, F, px, ds, nullptr);
}

// Copy the partition-function table into LDS (whole workgroup; barrier).
__device__ __forceinline__ void stage_ztab(const Shade &s, float4 *lds_tab) {
    for (int i = threadIdx.x; i < kZTableNodes - 1; i += blockDim.x) lds_tab[i] = s.ztab[i];
    __syncthreads();
}

// 1 - 2^-x given att = 2^-x, per channel: the series below kThinK
__device__ __forceinline__ float om_select(float x, float att) { return x < kThinK ? om_series3(x) : 1.0f - att; }

// One sample of the forward channel loop over CB channels held in registers:
// d = a - v_c b, x = K 2^-d^2 = 2^(lK - d^2) with lK = log2 K (K = 0 gives
// -inf, x = 0), I_c += Tr_c (1 - 2^-x) S, Tr_c *= 2^-x, with the series form
// when `thin` (K below kThinK; THIN; a branch per lane).  vel(c) gives
// channel c's velocity.
template <int CB, bool THIN, class Vel>
__device__ __forceinline__ void march_lk(float (&I)[CB], float (&Tr)[CB], float S, float lK, float a, float b,
                                         bool thin, Vel vel) {
    if (THIN && thin) {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const float d = fmaf(-vel(c), b, a);
            const float x = fexp2(fmaf(-d, d, lK));
            const float t = Tr[c] * om_series3(x);
            I[c] = fmaf(t, S, I[c]);
            Tr[c] -= t;
        }
    } else {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const float d = fmaf(-vel(c), b, a);
            const float x = fexp2(fmaf(-d, d, lK));
            const float att = fexp2(-x);
            I[c] = fmaf(Tr[c] * (1.0f - att), S, I[c]);
            Tr[c] *= att;
        }
    }
}

template <int CB, bool THIN, class Vel>
__device__ __forceinline__ void march_sample(float (&I)[CB], float (&Tr)[CB], const SampleQ &sq, Vel vel) {
    march_lk<CB, THIN>(I, Tr, sq.S, flog2(sq.K), sq.a, sq.b, sq.K < kThinK, vel);
}

} // namespace rt
