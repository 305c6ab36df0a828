// rt_adjoint_dev.h -- per-pixel and per-sample device functions of the
// adjoint passes, shared by the single-problem kernels and the server's
// batched ones (internal).
#pragma once
#include "rt_kernels.h"

namespace rt {

// Pass A for one pixel: its ray set-up (to rays[pix] when write_ray) and the
// channel-independent quantities (S, K, a, b) of samples [k0, k1) to the
// sample-major tape [nsamp][npix].
// span[pix] (when given) records the ray's samples with K > 0 as
// (nsamp - first, last + 1), zero when there are none: written whole when one
// chunk holds all the samples (shared = false), otherwise merged with atomic
// maxima into a span cleared beforehand.  With span_only (one chunk per ray)
// only the tape entries of that run are written: a zero entry is held back
// until a later sample with K > 0 shows it lies inside the run, so nothing
// is written in front of it, behind it, or for a ray that misses the grid.
__device__ __forceinline__ void tape_pixel(const Geometry &g, const Shade &s, const float4 *ztab, int pix, int k0,
                                           int k1, bool write_ray, float4 *__restrict__ tape,
                                           float4 *__restrict__ rays, int2 *__restrict__ span = nullptr,
                                           bool shared = false, bool span_only = false) {
    const int npix = g.nx * g.ny;
    const RaySetup r = ray_setup(g, pix % g.nx, pix / g.nx);
    if (write_ray) rays[pix] = make_float4(r.px, r.pmy, r.pmz, r.live ? r.ds : 0.0f);
    const float half = 0.5f * (float)g.nsamp;
    int kf = g.nsamp, kl = -1;
    for (int k = k0; k < k1; ++k) {
        float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (r.live) {
            const float t = ((float)k + 0.5f - half) * r.ds;
            const SampleQ q = s.mlp_o ? shade_sample<true>(s, ztab, r.px, fmaf(t, r.wy, r.pmy), fmaf(t, r.wz, r.pmz),
                                                           r.ds, o_index(s, k, pix))
                                      : shade_sample<false>(s, ztab, r.px, fmaf(t, r.wy, r.pmy), fmaf(t, r.wz, r.pmz),
                                                            r.ds, 0);
            o = make_float4(q.S, q.K, q.a, q.b);
        }
        if (o.y > 0.0f) {
            if (span_only && kl >= 0)   // the zeros since the last sample with K > 0
                for (int j = kl + 1; j < k; ++j) tape[(size_t)j * npix + pix] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            kf = min(kf, k);
            kl = k;
        }
        if (!span_only || o.y > 0.0f) tape[(size_t)k * npix + pix] = o;
    }
    if (span) {
        if (!shared) {
            span[pix] = make_int2(g.nsamp - kf, kl + 1);
        } else if (kl >= 0) {
            atomicMax(&span[pix].x, g.nsamp - kf);
            atomicMax(&span[pix].y, kl + 1);
        }
    }
}

// Largest v (0 <= v < 2^21) over the wave's active lanes, one bit at a time
// from the top: a ballot counts only active lanes, so lanes that have left
// (or never held a pixel) take no part.  Wave-uniform; needs one active lane.
__device__ __forceinline__ int active_max(int v) {
    int r = 0;
#pragma unroll
    for (int b = 20; b >= 0; --b) {
        const int c = r | (1 << b);
        if (__ballot(v >= c) != 0) r = c;
    }
    return r;
}

// (first, last) sample with K > 0 from a span record; first > last when none
__device__ __forceinline__ int2 span_of(int2 sp, int nsamp) { return make_int2(nsamp - sp.x, sp.y - 1); }

// value of the other lane of an adjacent pair (DPP quad permutation 1,0,3,2)
__device__ __forceinline__ float swap_pair(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// value of the lane two places over in a quad (DPP quad permutation 2,3,0,1)
__device__ __forceinline__ float swap_half_quad(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, false));
}

// Pass B without checkpoints for one pixel and one block of CB channels per
// lane (G = 1, 2 or 4 lanes per pixel; this lane is g of its group and its
// channels start at c0; blk is the cotangent slice of the G CB channels).
// vel(c) gives the velocity of this lane's channel c, plus vsh when SHIFT:
// the lane then folds vsh into a (d_c = (a - vsh b) - vel(c) b) and the
// derivative in b takes -vsh times the one in a.  With CUBE the march forms
// the intensity, and with target != NULL dL/dI = 2 (I - D) from it;
// otherwise dL/dI is read from dl_dcube.  Only the samples with K > 0 (one
// run along the ray) change anything: outside it x = 0 in every channel.
// With SPAN the run comes from the tape's span record (kspan = (first,
// last)): both sweeps cover the union of the wave's runs, each lane taking
// its tape entries outside its own run as zero (the tape may hold nothing
// there), and the cotangents outside a run are left unwritten, since the
// chain passes read the same record; without, sweep 1 finds the run and the
// cotangents outside it are written as zeros.  A pixel whose
// ray misses the grid (live false) has zero intensity: it only clears its
// channels of the cube and leaves its cotangents unwritten (every chain pass
// skips rays with ds = 0).
template <int CB, int G, bool CUBE, bool SHIFT = false, bool SPAN = false, class Vel>
__device__ __forceinline__ void march_tau_pixel(int pix, int blk, int g, int c0, int nch, int nsamp, int npix,
                                                int plane, bool live, Vel vel, const float4 *__restrict__ tape,
                                                const float *__restrict__ dl_dcube, const float *__restrict__ target,
                                                float4 *__restrict__ cot, float *__restrict__ cube_out,
                                                float vsh = 0.0f, int2 kspan = make_int2(0, -1)) {
    if (!live) {
        if (CUBE && cube_out) {
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c0 + c < nch) cube_out[(size_t)(c0 + c) * plane + pix] = 0.0f;
        }
        return;
    }
    float th[CB], tl[CB], w[CB];
    int kf = nsamp, kl = -1;
    // this lane's own run: the tape may hold nothing valid outside it
    const int own_f = kspan.x, own_l = kspan.y;
    if constexpr (SPAN) {
        // the union of the spans of the wave's live pixels (the lanes still
        // active here): a wave-uniform range, so both sweeps are scalar
        // loops; a lane's samples outside its own span in it have x = 0 and
        // change nothing
        kf = __builtin_amdgcn_readfirstlane(nsamp - active_max(nsamp - kspan.x));
        kl = __builtin_amdgcn_readfirstlane(active_max(kspan.y + 1) - 1);
    }
    {
        // sweep 1, back to front: total depth and (CUBE) J, which reaches I
        float J[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            th[c] = 0.0f;
            tl[c] = 0.0f;
            J[c] = 0.0f;
        }
        // the next sample's tape entry is loaded one iteration ahead.  With
        // SPAN the loop starts at kl and skips the samples in front of kf
        // (a bound of kf itself makes the compiler spill)
        const int k_hi = SPAN ? kl : nsamp - 1;
        float4 qn = tape[(size_t)max(k_hi, 0) * npix + pix];
#pragma unroll 1
        for (int k = k_hi; k >= 0; --k) {
            if (SPAN && k < kf) continue;
            float4 q = qn;
            qn = tape[(size_t)max(k - 1, 0) * npix + pix];
            if (SPAN && (k < own_f || k > own_l)) q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (!SPAN && q.y > 0.0f) {
                kf = k;
                kl = max(kl, k);
            }
            if constexpr (SHIFT) q.z = fmaf(-vsh, q.w, q.z);
            const float lK = flog2(q.y);
            // J_k-1 = S (1 - att) + att J_k: as S - att (S - J_k), or on a thin
            // sample as J_k + (1 - att)(S - J_k) with the series of 1 - att
            auto channels = [&](auto thin) {
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const float d = fmaf(-vel(c), q.w, q.z);
                    const float x = fexp2(fmaf(-d, d, lK));
                    // the error of th + x, exact with the larger operand first
                    // (both are >= 0, so their bit patterns order like the values)
                    const float sum = th[c] + x;
                    const unsigned ut = __float_as_uint(th[c]), ux = __float_as_uint(x);
                    tl[c] += __uint_as_float(min(ut, ux)) - (sum - __uint_as_float(max(ut, ux)));
                    th[c] = sum;
                    if (CUBE) {
                        if constexpr (decltype(thin)::value) J[c] = fmaf(om_series3(x), q.x - J[c], J[c]);
                        else J[c] = fmaf(-fexp2(-x), q.x - J[c], q.x);
                    }
                }
            };
            if (CUBE && q.y < kThinK) channels(std::true_type{});
            else channels(std::false_type{});
        }
        // padding channels of the last block read a valid channel's plane and
        // get w = 0
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const bool valid = c0 + c < nch;
            const size_t i = (size_t)min(c0 + c, nch - 1) * plane + pix;
            if (CUBE && cube_out && valid) cube_out[i] = J[c];
            const float wc = CUBE && target ? 2.0f * (J[c] - target[i]) : dl_dcube[i];
            w[c] = valid ? wc : 0.0f;
        }
    }
    // sweep 2, back to front: (sh, sl) = -(prefix depth) in front of the
    // current sample; u = w Tr
    float J[CB], u[CB];
    float *const sh = th, *const sl = tl;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        sh[c] = -th[c];
        sl[c] = -tl[c];
        J[c] = 0.0f;
        u[c] = w[c] * fexp2(sh[c] + sl[c]);
    }
    if (!SPAN && g == 0) {
        const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int k = nsamp - 1; k > kl; --k) cot[((size_t)blk * nsamp + k) * npix + pix] = z;
        if (kl >= 0)
            for (int k = kf - 1; k >= 0; --k) cot[((size_t)blk * nsamp + k) * npix + pix] = z;
    }
    float4 qn = tape[(size_t)max(kl, 0) * npix + pix];
#pragma unroll 1
    for (int k = kl; k >= kf; --k) {
        float4 q = qn;
        qn = tape[(size_t)max(k - 1, 0) * npix + pix];
        if (SPAN && (k < own_f || k > own_l)) q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float S = q.x, b = q.w;
        const float a = SHIFT ? fmaf(-vsh, q.w, q.z) : q.z;
        const float lK = flog2(q.y);
        // channel sums in two interleaved halves (shorter dependency chains)
        float cS[2] = {0.0f, 0.0f}, cX[2] = {0.0f, 0.0f}, ca[2] = {0.0f, 0.0f}, cb[2] = {0.0f, 0.0f};
        // on a thin sample 1 - att comes from its series and J_k-1 =
        // J_k + (1 - att)(S - J_k); otherwise J_k-1 = S - att (S - J_k)
        auto channels = [&](auto thin) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int h = c & 1;
                const float vc = vel(c);
                const float d = fmaf(-vc, b, a);
                const float x = fexp2(fmaf(-d, d, lK));
                const float smj = S - J[c];
                const float gg = u[c] * smj * x;
                float om;
                if constexpr (decltype(thin)::value) {
                    om = om_series3(x);
                    J[c] = fmaf(om, smj, J[c]);
                } else {
                    const float att = fexp2(-x);
                    om = 1.0f - att;
                    J[c] = fmaf(-att, smj, S);
                }
                const float sum = sh[c] + x;
                sl[c] += x - (sum - sh[c]);
                sh[c] = sum;
                const float u0 = w[c] * fexp2(sum + sl[c]);
                cS[h] = fmaf(u0, om, cS[h]);
                cX[h] += gg;
                const float gd = gg * d;
                ca[h] += gd;
                cb[h] = fmaf(-vc, gd, cb[h]);
                u[c] = u0;
            }
        };
        if (q.y < kThinK) channels(std::true_type{});
        else channels(std::false_type{});
        const float m = -2.0f * kLn2 * kLn2;
        float4 o = make_float4(cS[0] + cS[1], (cX[0] + cX[1]) * kLn2, (ca[0] + ca[1]) * m, (cb[0] + cb[1]) * m);
        if constexpr (SHIFT) o.w = fmaf(-vsh, o.z, o.w);
        if constexpr (G >= 2) {
            o.x += swap_pair(o.x);
            o.y += swap_pair(o.y);
            o.z += swap_pair(o.z);
            o.w += swap_pair(o.w);
        }
        if constexpr (G == 4) {
            o.x += swap_half_quad(o.x);
            o.y += swap_half_quad(o.y);
            o.z += swap_half_quad(o.z);
            o.w += swap_half_quad(o.w);
        }
        if (g == 0) cot[((size_t)blk * nsamp + k) * npix + pix] = o;
    }
}

// Pass C for one pixel-sample: the local derivatives of the shading chained
// from the sample's cotangents c = (dL/dS, dL/d ln K, dL/da, dL/db) to the
// interpolated fields and surfaces (and, with the network, to its outputs).
struct ChainTerms {
    float gn, gT, gV;     // dL/d(ln n, T, v_phi) at the sample
    float gzl, gzu;       // dL/d(z_lo, z_up) at the sample
    float fu, fv;         // bilinear weights
    int i0, j0;           // cell corner
    float4 dout;          // dL/d(network outputs)
};

__device__ __forceinline__ ChainTerms chain_terms(const Geometry &g, const Shade &s, const float4 *ztab, float4 r,
                                                  float4 c, int k, int pix) {
    ChainTerms out;
    const float ds = r.w;
    const float t = ((float)k + 0.5f - 0.5f * (float)g.nsamp) * ds;
    const float wy = (float)g.si, wz = (float)(-g.ci);
    const float py = fmaf(t, wy, r.y), pz = fmaf(t, wz, r.z);
    const Locus L = locate(s, r.x, py, pz);
    Fields F = fetch(s, L);
    float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float tfac = 1.0f;
    const float t_grid = F.T;
    if (s.mlp_o) {
        o = s.mlp_o[o_index(s, k, pix)];
        apply_mlp(s, F, L, o);
        tfac = F.T / t_grid;
    }
    PhysTape tp;
    const SampleQ q = physics<true>(s, ztab, L, F, r.x, ds, &tp);
    const float gS = c.x, gK = c.y, ga = c.z, gb = c.w;
    const float gKK = gK;  // dL/d ln K, and d ln K / d ln n = 1
    const float dlnK_dT = tp.rT * (s.el_log2e * kLn2 * tp.rT - tp.x / tp.em1 - tp.dZ / (tp.Z * kLn2) - 0.5f);
    const float dS_dT = q.S * (1.0f + tp.em1) / tp.em1 * tp.x * tp.rT;
    float gT = gS * dS_dT + gKK * dlnK_dT - 0.5f * tp.rT * (gb * q.b + ga * q.a);
    float gzu = gKK * tp.sa * tp.iw * kLn2;
    float gzl = -gKK * tp.sb * tp.iw * kLn2;
    out.dout = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (s.mlp_o) {
        // network outputs: z_up = zr rho sigma(o0), z_lo = zr rho sigma(o1),
        // T = T_grid exp(0.5 tanh(o2)); the grid surfaces are not used
        const float s0 = sigmoidf_(o.x), s0c = sigmoidf_(-o.x);
        const float s1 = sigmoidf_(o.y), s1c = sigmoidf_(-o.y);
        const float th = tanhf_(o.z);
        out.dout.x = gzu * s.zr_max * L.rho * s0 * s0c;
        out.dout.y = gzl * s.zr_max * L.rho * s1 * s1c;
        out.dout.z = gT * F.T * 0.5f * (1.0f - th * th);
        gT *= tfac;
        gzu = 0.0f;
        gzl = 0.0f;
    }
    out.gn = gKK;
    out.gT = gT;
    out.gV = ga * q.b * tp.vfac;
    out.gzl = gzl;
    out.gzu = gzu;
    out.fu = L.fu;
    out.fv = L.fv;
    out.i0 = L.i0;
    out.j0 = L.j0;
    return out;
}

} // namespace rt
