// rt_adjoint.hip -- reverse-mode derivative of the ray march.
//
// Pass A (adj_tape): one lane per pixel walks its ray and writes the
//   channel-independent sample quantities (S, K, a, b) to a sample-major
//   tape, plus the ray's set-up and its span: the run of samples with K > 0,
//   outside which a sample changes nothing and has no cotangents (with the
//   checkpoint-free march and one chunk per ray only that run is written).
// Pass B (adj_march<CB, KSEG>): one lane per pixel x channel block.  A
//   forward sweep stores the transmission of each channel at the start of
//   every KSEG-sample segment (the checkpoints); the reverse sweep visits the
//   segments back to front, recomputes the segment's transmissions in
//   registers from its checkpoint, and walks it backwards with the
//   intensity-from-behind recurrence
//       J_{k-1} = S_k (1 - a_k) + a_k J_k,
//   giving dI/dS_k = Tr_k (1 - a_k) and dI/ddtau_k = Tr_{k+1} (S_k - J_k)
//   without the cancellation of I minus a prefix sum.  Channel sums of the
//   per-sample cotangents (S, ln K, a, b) are written per channel block.
// Pass B without checkpoints (adj_march_tau<CB, G, CUBE>, the default; G
//   lanes per pixel): the
//   optical depth is additive, so the transmission in front of sample k is
//   2^-(tau_tot - tau_suf(k)) with tau_suf the depth behind it.  A first
//   back-to-front sweep adds up tau_tot (and, when the intensity is wanted,
//   runs the J recurrence to the observer); the second sweep re-accumulates
//   tau_suf in the same order, so the only state kept per (ray, channel) is
//   the total depth, in a register, and nothing is written but the
//   cotangents.  Both sweeps cover only the union of the spans of the
//   wave's rays; rays that miss the grid only clear their cube channels.
// Pass C (adj_chain_lds, or adj_chain for grids too large for LDS): each
//   pixel-sample inside its ray's span that has a cotangent has its shading
//   recomputed with its local derivatives, the cotangents chained to the
//   interpolated fields and added to the grid nodes (one field per pass
//   privatised in LDS and flushed once, the T pass from terms the first pass
//   stored when ln n and T are asked for; adj_chain scatters with global
//   atomics; the surface vectors in LDS either way).
#include <type_traits>

#include "rt_adjoint.h"
#include "rt_adjoint_dev.h"
#include "rt_host.h"

namespace rt {

// blockIdx.y selects a chunk of the samples, so short images still give the
// GPU enough lanes
__global__ __launch_bounds__(256) void adj_tape(Geometry g, Shade s, float4 *__restrict__ tape,
                                                float4 *__restrict__ rays, int2 *__restrict__ span, int span_only) {
    __shared__ float4 ztab[kZTableNodes - 1];
    stage_ztab(s, ztab);
    const int npix = g.nx * g.ny;
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= npix) return;
    const int len = (g.nsamp + gridDim.y - 1) / gridDim.y;
    const int k0 = blockIdx.y * len, k1 = min(g.nsamp, k0 + len);
    tape_pixel(g, s, ztab, pix, k0, k1, blockIdx.y == 0, tape, rays, span, gridDim.y > 1,
               span_only && gridDim.y == 1);
}

// dl_dcube: the cotangent dL/dI; or, with target != NULL, the cotangent of
// the L2 loss sum (I - D)^2 is formed from the forward sweep's own I:
// dL/dI = 2 (I - D).
template <int CB, int KSEG>
__global__ __launch_bounds__(256) void adj_march(int nsamp, int npix, int plane, Channels ch,
                                                 const float4 *__restrict__ tape, const float *__restrict__ dl_dcube,
                                                 const float *__restrict__ target, float *__restrict__ ckpt,
                                                 float4 *__restrict__ cot, float *__restrict__ cube_out) {
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= npix) return;
    const int blk = blockIdx.y, nblk = gridDim.y;
    const int c0 = blk * CB;
    const int nseg = (nsamp + KSEG - 1) / KSEG;
    float w[CB], Tr[CB], I[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        Tr[c] = 1.0f;
        I[c] = 0.0f;
    }
    // forward sweep with checkpoints
    for (int seg = 0; seg < nseg; ++seg) {
#pragma unroll
        for (int c = 0; c < CB; ++c) ckpt[((size_t)seg * nblk * CB + c0 + c) * npix + pix] = Tr[c];
#pragma unroll
        for (int kk = 0; kk < KSEG; ++kk) {
            const int k = seg * KSEG + kk;
            if (k < nsamp) {
                const float4 q = tape[(size_t)k * npix + pix];
                const float lK = flog2(q.y);    // K 2^-d^2 = 2^(log2 K - d^2)
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const float d = fmaf(-ch.v[c0 + c], q.w, q.z);
                    const float x = fexp2(fmaf(-d, d, lK));
                    const float att = fexp2(-x);
                    I[c] = fmaf(Tr[c] * om_select(x, att), q.x, I[c]);
                    Tr[c] *= att;
                }
            }
        }
    }
    if (cube_out) {
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c0 + c < ch.n) cube_out[(size_t)(c0 + c) * plane + pix] = I[c];
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const size_t i = (size_t)(c0 + c) * plane + pix;
        w[c] = c0 + c >= ch.n ? 0.0f : (target ? 2.0f * (I[c] - target[i]) : dl_dcube[i]);
    }
    // reverse sweep, one segment at a time
    float J[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) J[c] = 0.0f;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        float4 Q[KSEG];
        float TrK[KSEG][CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) Tr[c] = ckpt[((size_t)seg * nblk * CB + c0 + c) * npix + pix];
#pragma unroll
        for (int kk = 0; kk < KSEG; ++kk) {
            const int k = seg * KSEG + kk;
            Q[kk] = k < nsamp ? tape[(size_t)k * npix + pix] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const float lK = flog2(Q[kk].y);
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                TrK[kk][c] = Tr[c];
                const float d = fmaf(-ch.v[c0 + c], Q[kk].w, Q[kk].z);
                Tr[c] *= fexp2(-fexp2(fmaf(-d, d, lK)));
            }
        }
#pragma unroll
        for (int kk = KSEG - 1; kk >= 0; --kk) {
            const int k = seg * KSEG + kk;
            if (k >= nsamp) continue;
            const float S = Q[kk].x, K = Q[kk].y, a = Q[kk].z, b = Q[kk].w;
            // the ln2 of dtau = ln2 K g is applied once per sample: to cK at
            // the end, and folded into Km for the chain to d
            const float Km = K * (-2.0f * kLn2 * kLn2);
            float cS = 0.0f, cK = 0.0f, ca = 0.0f, cb = 0.0f;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const float vc = ch.v[c0 + c];
                const float d = fmaf(-vc, b, a);
                const float gk = fexp2(-(d * d));
                const float att = fexp2(-(K * gk));
                const float om = om_select(K * gk, att);
                const float t0 = TrK[kk][c];
                const float t1 = t0 * att;
                const float smj = S - J[c];
                // dI/dS = Tr_k (1 - att)  (as a difference of transmissions it
                // keeps t1 live longer: one occupancy step fewer)
                cS = fmaf(w[c] * t0, om, cS);
                // dL/d(dtau) / ln2, with dtau = ln2 K g, g = 2^-d^2
                const float gg = w[c] * t1 * smj * gk;
                // J_k-1 = S (1 - att) + att J_k = J_k + (1 - att)(S - J_k)
                J[c] = fmaf(om, smj, J[c]);
                cK += gg;
                const float gd = gg * Km * d;
                ca += gd;
                cb = fmaf(-vc, gd, cb);
            }
            // the K slot carries dL/d ln K = K dL/dK
            cot[((size_t)blk * nsamp + k) * npix + pix] = make_float4(cS, cK * (kLn2 * K), ca, cb);
        }
    }
}

// Checkpoint-free reverse march.  Per sample and channel, with x = K 2^-d^2
// the depth in log2 units (att = 2^-x) and t1 = Tr_{k+1}, t0 = Tr_k:
//   dL/dS     += w t0 (1 - att)
//   dL/dln K  += ln2 w t1 (S - J_k) x
//   dL/dd      = -2 ln2^2 w t1 (S - J_k) x d, to a as 1 and to b as -v.
// The prefix depth tau_tot - tau_suf is the small difference of two large
// sums when the back of the ray is thick (tau_tot reaches 10^4 at line
// centre), so both sums carry the rounding error of every addition in a
// second float (Fast2Sum, exact when the larger operand comes first).
// Sweep 1 sums tau_tot = th + tl, ordering the operands; sweep 2 starts its
// running sum at -th and its error at -tl and adds the same x back to front,
// where the running sum (minus the prefix depth plus x) is never the smaller
// operand, so after sample k the pair holds minus the prefix depth of k to
// within one rounding of the prefix itself.

// Work items: G adjacent lanes per pixel, each with CB channels (G = 2 or 4:
// the group's channel sums are added across its lanes, so one cotangent
// slice is written per G CB channels and the group reads each tape entry
// once); the channel blocks of one tile take workgroup ids 8 apart, so they
// run on one XCD at about the same time and share the tile's tape through
// its L2.  At G = 4 the channels are uniformly spaced in groups of CB (lane
// g's velocities are lane 0's plus g shift): the velocities stay scalars and
// each lane folds its offset into a.
template <int CB, int G, bool CUBE>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(CB * G <= 8 ? 6 : G == 4 ? 4 : CB <= 16 && G == 1 ? 4 : CB <= 24 && G == 1 ? 3 : 2)))
void adj_march_tau(int nsamp, int npix, int plane, int nblk, Channels ch, float shift,
                   const float4 *__restrict__ tape, const int2 *__restrict__ span, const float *__restrict__ dl_dcube,
                   const float *__restrict__ target, float4 *__restrict__ cot, float *__restrict__ cube_out) {
    static_assert(G == 1 || G == 2 || G == 4, "one, two or four lanes per pixel");
    const int id = blockIdx.x, r8 = id >> 3;
    const int blk = r8 % nblk;
    const int g = G == 1 ? 0 : (int)(threadIdx.x % G);
    const int pix = ((r8 / nblk) * 8 + (id & 7)) * (256 / G) + (int)threadIdx.x / G;
    if (pix >= npix) return;   // the lanes of a pixel leave together
    const int c0 = (blk * G + g) * CB;
    const int2 ks = span_of(span[pix], nsamp);
    const bool live = ks.y >= ks.x;
    if constexpr (G == 4) {
        auto vel = [&](int c) { return ch.v[blk * G * CB + c]; };
        march_tau_pixel<CB, G, CUBE, true, true>(pix, blk, g, c0, ch.n, nsamp, npix, plane, live, vel, tape, dl_dcube,
                                                 target, cot, cube_out, (float)g * shift, ks);
    } else {
        // channel velocities: scalar registers with one lane per pixel,
        // vector registers when the lanes of a pixel take different channels
        float vv[G > 1 ? CB : 1];
        if constexpr (G > 1) {
#pragma unroll
            for (int c = 0; c < CB; ++c) vv[c] = g ? ch.v[blk * G * CB + CB + c] : ch.v[blk * G * CB + c];
        }
        auto vel = [&](int c) -> float {
            if constexpr (G > 1) return vv[c];
            else return ch.v[c0 + c];
        };
        march_tau_pixel<CB, G, CUBE, false, true>(pix, blk, g, c0, ch.n, nsamp, npix, plane, live, vel, tape, dl_dcube,
                                                  target, cot, cube_out, 0.0f, ks);
    }
}


template <typename A>
__device__ __forceinline__ void scatter4(A *dst, int n00, int n10, float gv, float w00, float w01, float w10,
                                         float w11) {
    if (!dst || gv == 0.0f) return;
    atomicAdd(dst + n00, (A)(gv * w00));
    atomicAdd(dst + n00 + 1, (A)(gv * w01));
    atomicAdd(dst + n10, (A)(gv * w10));
    atomicAdd(dst + n10 + 1, (A)(gv * w11));
}

template <typename A>
__global__ __launch_bounds__(256) void adj_chain(Geometry g, Shade s, const float4 *__restrict__ rays,
                                                 const int2 *__restrict__ span, const float4 *__restrict__ cot,
                                                 int nblk, GradAcc go, int lds_surfaces, float4 *__restrict__ dO) {
    extern __shared__ float lds[];   // [2][nr] surface gradients when lds_surfaces
    __shared__ float4 ztab[kZTableNodes - 1];
    stage_ztab(s, ztab);
    const int npix = g.nx * g.ny;
    const int nr = s.nr;
    A *const gzlo = (A *)go.zlo, *const gzup = (A *)go.zup;
    if (lds_surfaces) {
        for (int i = threadIdx.x; i < 2 * nr; i += 256) lds[i] = 0.0f;
        __syncthreads();
    }
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t total = (size_t)g.nsamp * npix;
    if (idx < total) {
        const int k = (int)(idx / npix);
        const int pix = (int)(idx - (size_t)k * npix);
        // samples outside the ray's run of K > 0 have no cotangents
        const int2 ks = span_of(span[pix], g.nsamp);
        float4 c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float4 r = c;
        if (k >= ks.x && k <= ks.y) {
            r = rays[pix];
            for (int b = 0; b < nblk; ++b) {
                const float4 t = cot[((size_t)b * g.nsamp + k) * npix + pix];
                c.x += t.x; c.y += t.y; c.z += t.z; c.w += t.w;
            }
        }
        float4 dout = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (r.w > 0.0f && (c.x != 0.0f || c.y != 0.0f || c.z != 0.0f || c.w != 0.0f)) {
            const ChainTerms t = chain_terms(g, s, ztab, r, c, k, pix);
            dout = t.dout;
            const float fu = t.fu, fv = t.fv;
            const float w00 = (1.0f - fu) * (1.0f - fv), w01 = (1.0f - fu) * fv, w10 = fu * (1.0f - fv), w11 = fu * fv;
            const int n00 = t.i0 * s.nz + t.j0, n10 = n00 + s.nz;
            scatter4((A *)go.ln_n, n00, n10, t.gn, w00, w01, w10, w11);
            scatter4((A *)go.temp, n00, n10, t.gT, w00, w01, w10, w11);
            scatter4((A *)go.vphi, n00, n10, t.gV, w00, w01, w10, w11);
            if (lds_surfaces) {
                if (t.gzl != 0.0f) { atomicAdd(lds + t.i0, t.gzl * (1.0f - fu)); atomicAdd(lds + t.i0 + 1, t.gzl * fu); }
                if (t.gzu != 0.0f) { atomicAdd(lds + nr + t.i0, t.gzu * (1.0f - fu)); atomicAdd(lds + nr + t.i0 + 1, t.gzu * fu); }
            } else {
                if (gzlo && t.gzl != 0.0f) { atomicAdd(gzlo + t.i0, (A)(t.gzl * (1.0f - fu))); atomicAdd(gzlo + t.i0 + 1, (A)(t.gzl * fu)); }
                if (gzup && t.gzu != 0.0f) { atomicAdd(gzup + t.i0, (A)(t.gzu * (1.0f - fu))); atomicAdd(gzup + t.i0 + 1, (A)(t.gzu * fu)); }
            }
        }
        if (dO) dO[o_index(s, k, pix)] = dout;
    }
    if (lds_surfaces) {
        __syncthreads();
        for (int i = threadIdx.x; i < nr; i += 256) {
            const float a = lds[i], b = lds[nr + i];
            if (gzlo && a != 0.0f) atomicAdd(gzlo + i, (A)a);
            if (gzup && b != 0.0f) atomicAdd(gzup + i, (A)b);
        }
    }
}

// lanes per workgroup of the privatised chain pass: one workgroup fills a CU's
// LDS, so it brings sixteen waves to keep the CU busy
constexpr int kChainThreads = 1024;
// pixel rotation from one sample plane to the next in the chain pass (an odd
// number of workgroup spans)
constexpr int kChainTurn = 37 * kChainThreads;

// Chain pass with the gradient of one field privatised in LDS.  Persistent
// workgroups take runs of 1024 consecutive pixel-samples in grid-stride
// order, so every workgroup sees every depth along the rays (with one
// contiguous share each, the few whose samples crossed the disk did the work
// while those beyond it, where the cotangents vanish, sat idle), accumulate
// field FIELD (0 ln n, 1 T, 2 v_phi, 3 none) over the whole grid in LDS
// (float), and flush it once with atomics into the accumulators of type A;
// the FIRST pass also accumulates the two surface vectors (LDS, float) and
// writes dL/do.
// With STORE (the first pass, FIELD 0) each sample inside a ray's run also
// leaves the temperature term of its chain in slice 0 of the cotangents,
// which it has consumed: (dL/dT at the sample, the cell's first node as
// integer bits, the two bilinear weights), zero where there is none; the
// second pass (adj_chain_lds_stored) then adds those into the T gradient
// without shading the sample again.
template <int FIELD, bool FIRST, typename A, bool STORE = false>
__global__ __launch_bounds__(kChainThreads) void adj_chain_lds(Geometry g, Shade s, const float4 *__restrict__ rays,
                                                     const int2 *__restrict__ span, float4 *__restrict__ cot,
                                                     int nblk, GradAcc go, float4 *__restrict__ dO) {
    extern __shared__ float dyn[];               // [2 nr] surfaces (FIRST), then [nr nz] field
    __shared__ float4 ztab[kZTableNodes - 1];
    const int nr = s.nr, nn = s.nr * s.nz;
    float *surf = dyn;
    float *field = dyn + (FIRST ? 2 * nr : 0);
    for (int i = threadIdx.x; i < kZTableNodes - 1; i += kChainThreads) ztab[i] = s.ztab[i];
    if (FIELD < 3) for (int i = threadIdx.x; i < nn; i += kChainThreads) field[i] = 0.0f;
    if (FIRST) for (int i = threadIdx.x; i < 2 * nr; i += kChainThreads) surf[i] = 0.0f;
    __syncthreads();
    const int npix = g.nx * g.ny;
    const size_t total = (size_t)g.nsamp * npix;
    // sample plane k is visited with its pixels rotated by k kChainTurn: a
    // lane's pixel moves across the image from one plane to the next, so no
    // workgroup keeps the same rays (the disk's centre or the empty corners)
    // for every sample when the grid stride is a multiple of the image
    const int turn = (int)((size_t)kChainTurn % (size_t)npix);
    for (size_t idx = (size_t)blockIdx.x * kChainThreads + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * kChainThreads) {
        const int k = (int)(idx / npix);
        int pix = (int)(idx - (size_t)k * npix) + (int)(((long)k * turn) % npix);
        if (pix >= npix) pix -= npix;
        // samples outside the ray's run of K > 0 have no cotangents (the
        // march leaves them unwritten)
        const int2 ks = span_of(span[pix], g.nsamp);
        float4 c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float4 r = c;
        const bool in_run = k >= ks.x && k <= ks.y;
        if (in_run) {
            r = rays[pix];
            // the first pass sums the channel-block slices and keeps the sum in slice 0
            const int nb = FIRST ? nblk : 1;
            for (int b = 0; b < nb; ++b) {
                const float4 t = cot[((size_t)b * g.nsamp + k) * npix + pix];
                c.x += t.x; c.y += t.y; c.z += t.z; c.w += t.w;
            }
            if (FIRST && !STORE && nblk > 1) cot[(size_t)k * npix + pix] = c;
        }
        float4 dout = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float4 tterm = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // STORE: the sample's T term
        if (r.w > 0.0f && (c.x != 0.0f || c.y != 0.0f || c.z != 0.0f || c.w != 0.0f)) {
            const float ds = r.w;
            const float t = ((float)k + 0.5f - 0.5f * (float)g.nsamp) * ds;
            const float py = fmaf(t, (float)g.si, r.y), pz = fmaf(t, (float)(-g.ci), r.z);
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
            const float gKK = gK;
            float gv = 0.0f;
            if (FIELD == 0) gv = gKK;
            if (FIELD == 1 || FIRST) {
                const float dlnK_dT = tp.rT * (s.el_log2e * kLn2 * tp.rT - tp.x / tp.em1 -
                                               tp.dZ / (tp.Z * kLn2) - 0.5f);
                const float dS_dT = q.S * (1.0f + tp.em1) / tp.em1 * tp.x * tp.rT;
                const float gT = gS * dS_dT + gKK * dlnK_dT - 0.5f * tp.rT * (gb * q.b + ga * q.a);
                if (FIELD == 1) gv = gT * tfac;
                if (STORE) tterm = make_float4(gT * tfac, __int_as_float(L.i0 * s.nz + L.j0), L.fu, L.fv);
                if (FIRST && s.mlp_o) {
                    const float s0 = sigmoidf_(o.x), s0c = sigmoidf_(-o.x);
                    const float s1 = sigmoidf_(o.y), s1c = sigmoidf_(-o.y);
                    const float th = tanhf_(o.z);
                    dout.x = gKK * tp.sa * tp.iw * kLn2 * s.zr_max * L.rho * s0 * s0c;
                    dout.y = -gKK * tp.sb * tp.iw * kLn2 * s.zr_max * L.rho * s1 * s1c;
                    dout.z = gT * F.T * 0.5f * (1.0f - th * th);
                }
            }
            if (FIELD == 2) gv = ga * q.b * tp.vfac;
            const float fu = L.fu, fv = L.fv;
            if (FIELD < 3 && gv != 0.0f) {
                const int n00 = L.i0 * s.nz + L.j0, n10 = n00 + s.nz;
                atomicAdd(field + n00, gv * (1.0f - fu) * (1.0f - fv));
                atomicAdd(field + n00 + 1, gv * (1.0f - fu) * fv);
                atomicAdd(field + n10, gv * fu * (1.0f - fv));
                atomicAdd(field + n10 + 1, gv * fu * fv);
            }
            if (FIRST && !s.mlp_o) {
                const float gzu = gKK * tp.sa * tp.iw * kLn2;
                const float gzl = -gKK * tp.sb * tp.iw * kLn2;
                if (gzl != 0.0f) { atomicAdd(surf + L.i0, gzl * (1.0f - fu)); atomicAdd(surf + L.i0 + 1, gzl * fu); }
                if (gzu != 0.0f) { atomicAdd(surf + nr + L.i0, gzu * (1.0f - fu)); atomicAdd(surf + nr + L.i0 + 1, gzu * fu); }
            }
        }
        if (FIRST && dO) dO[o_index(s, k, pix)] = dout;
        if (STORE && in_run) cot[(size_t)k * npix + pix] = tterm;
    }
    __syncthreads();
    A *dst = (A *)(FIELD == 0 ? go.ln_n : (FIELD == 1 ? go.temp : (FIELD == 2 ? go.vphi : nullptr)));
    if (FIELD < 3 && dst)
        for (int i = threadIdx.x; i < nn; i += kChainThreads)
            if (field[i] != 0.0f) atomicAdd(dst + i, (A)field[i]);
    if (FIRST)
        for (int i = threadIdx.x; i < nr; i += kChainThreads) {
            if (go.zlo && surf[i] != 0.0f) atomicAdd((A *)go.zlo + i, (A)surf[i]);
            if (go.zup && surf[nr + i] != 0.0f) atomicAdd((A *)go.zup + i, (A)surf[nr + i]);
        }
}

// The temperature pass from the terms a STORE first pass left in slice 0
// of the cotangents: no shading, only the bilinear scatter into the grid in
// LDS and one flush, in the first pass's order of the samples.
template <typename A>
__global__ __launch_bounds__(kChainThreads) void adj_chain_lds_stored(Geometry g, Shade s, const int2 *__restrict__ span,
                                                             const float4 *__restrict__ cot, GradAcc go) {
    extern __shared__ float field[];   // [nr nz]
    const int nn = s.nr * s.nz;
    for (int i = threadIdx.x; i < nn; i += kChainThreads) field[i] = 0.0f;
    __syncthreads();
    const int npix = g.nx * g.ny;
    const size_t total = (size_t)g.nsamp * npix;
    const int turn = (int)((size_t)kChainTurn % (size_t)npix);
    for (size_t idx = (size_t)blockIdx.x * kChainThreads + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * kChainThreads) {
        const int k = (int)(idx / npix);
        int pix = (int)(idx - (size_t)k * npix) + (int)(((long)k * turn) % npix);
        if (pix >= npix) pix -= npix;
        const int2 ks = span_of(span[pix], g.nsamp);
        if (k < ks.x || k > ks.y) continue;
        const float4 t = cot[(size_t)k * npix + pix];
        const float gv = t.x;
        if (gv != 0.0f) {
            const int n00 = __float_as_int(t.y), n10 = n00 + s.nz;
            const float fu = t.z, fv = t.w;
            atomicAdd(field + n00, gv * (1.0f - fu) * (1.0f - fv));
            atomicAdd(field + n00 + 1, gv * (1.0f - fu) * fv);
            atomicAdd(field + n10, gv * fu * (1.0f - fv));
            atomicAdd(field + n10 + 1, gv * fu * fv);
        }
    }
    __syncthreads();
    A *dst = (A *)go.temp;
    for (int i = threadIdx.x; i < nn; i += kChainThreads)
        if (field[i] != 0.0f) atomicAdd(dst + i, (A)field[i]);
}

template <int FIELD, bool FIRST, typename A, bool STORE = false>
static hipError_t launch_chain_lds_t(const Geometry &g, const Shade &s, const float4 *rays, const int2 *span, float4 *cot,
                                     int nblk, const GradAcc &go, float4 *dO, int nwg, size_t shmem, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)adj_chain_lds<FIELD, FIRST, A, STORE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((adj_chain_lds<FIELD, FIRST, A, STORE>), dim3(nwg), dim3(kChainThreads), shmem, st, g, s, rays,
                       span, cot, nblk, go, dO);
    return hipGetLastError();
}

// largest dynamic LDS the privatised chain may use (the LDS of a CU, less
// the partition table)
constexpr size_t kChainLdsMax = 160 * 1024 - sizeof(float4) * (kZTableNodes - 1) - 1024;

bool chain_lds_fits(int nr, int nz) {
    return (size_t)nr * nz * sizeof(float) + 2 * (size_t)nr * sizeof(float) <= kChainLdsMax;
}

template <typename A>
static hipError_t chain_lds_passes(const Geometry &g, const Shade &s, const float4 *rays, const int2 *span,
                                   float4 *cot, int nblk, const GradAcc &go, float4 *dO, int nwg, hipStream_t st) {
    const size_t fb = (size_t)s.nr * s.nz * sizeof(float), sb = 2 * (size_t)s.nr * sizeof(float);
    const bool want[3] = {go.ln_n != nullptr, go.temp != nullptr, go.vphi != nullptr};
    if (want[0] && want[1] && !want[2]) {
        // ln n and T: the first pass leaves the T terms for the second
        hipError_t e = launch_chain_lds_t<0, true, A, true>(g, s, rays, span, cot, nblk, go, dO, nwg, fb + sb, st);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void *)adj_chain_lds_stored<A>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)fb);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(adj_chain_lds_stored<A>, dim3(nwg), dim3(kChainThreads), fb, st, g, s, span, cot, go);
        return hipGetLastError();
    }
    bool first = true;
    hipError_t e = hipSuccess;
    for (int f = 0; f < 3; ++f) {
        if (!want[f]) continue;
        const size_t shmem = fb + (first ? sb : 0);
        if (first) {
            e = f == 0 ? launch_chain_lds_t<0, true, A>(g, s, rays, span, cot, nblk, go, dO, nwg, shmem, st)
              : f == 1 ? launch_chain_lds_t<1, true, A>(g, s, rays, span, cot, nblk, go, dO, nwg, shmem, st)
                       : launch_chain_lds_t<2, true, A>(g, s, rays, span, cot, nblk, go, dO, nwg, shmem, st);
        } else {
            e = f == 1 ? launch_chain_lds_t<1, false, A>(g, s, rays, span, cot, nblk, go, dO, nwg, shmem, st)
                       : launch_chain_lds_t<2, false, A>(g, s, rays, span, cot, nblk, go, dO, nwg, shmem, st);
        }
        if (e != hipSuccess) return e;
        first = false;
    }
    if (first) e = launch_chain_lds_t<3, true, A>(g, s, rays, span, cot, nblk, go, dO, nwg, sb, st);
    return e;
}

hipError_t launch_adj_chain_lds(const Geometry &g, const Shade &s, const float4 *rays, const int2 *span, float4 *cot,
                                int nblk, const GradAcc &go, float4 *dO, hipStream_t st) {
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t total = (size_t)g.nsamp * g.nx * g.ny;
    const int nwg = (int)std::min<size_t>((size_t)ncu, (total + kChainThreads - 1) / kChainThreads);
    return grad_accum_double() ? chain_lds_passes<double>(g, s, rays, span, cot, nblk, go, dO, nwg, st)
                               : chain_lds_passes<float>(g, s, rays, span, cot, nblk, go, dO, nwg, st);
}

__global__ void fill_zero_d(double *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void to_float(const double *src, float *dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// field accumulators held as float: copy them out (same layout as double)
__global__ void copy_float(const float *src, float *dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t zero_async_d(double *p, size_t n, hipStream_t st) {
    if (!p || n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_zero_d, dim3(blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t copy_float_async(const float *src, float *dst, size_t n, hipStream_t st) {
    if (!dst || n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_float, dim3(blocks), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t to_float_async(const double *src, float *dst, size_t n, hipStream_t st) {
    if (!dst || n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(to_float, dim3(blocks), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

__global__ void fill_zero(float *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0f;
}

hipError_t zero_async(float *p, size_t n, hipStream_t st) {
    if (!p || n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_zero, dim3(blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_adj_tape(const Geometry &g, const Shade &s, float4 *tape, float4 *rays, int2 *span, bool span_only,
                           hipStream_t st) {
    const int npix = g.nx * g.ny;
    const int tiles = (npix + 255) / 256;
    // sample chunks until about 16 waves per CU (of at least 32 samples each)
    int chunks = 1;
    while (chunks < 16 && (long)tiles * 4 * chunks < 16L * 256 && g.nsamp >= 64 * chunks) chunks *= 2;
    if (chunks > 1) {   // the chunks merge their spans into a cleared record
        const hipError_t e = zero_async((float *)span, 2 * (size_t)npix, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(adj_tape, dim3(tiles, chunks), dim3(256), 0, st, g, s, tape, rays, span, span_only ? 1 : 0);
    return hipGetLastError();
}

template <int CB, int KSEG>
static hipError_t launch_march_t(int nsamp, int npix, int plane, const Channels &ch, const float4 *tape,
                                 const float *dl, const float *target, float *ckpt, float4 *cot, float *cube_out,
                                 hipStream_t st) {
    dim3 grid((npix + 255) / 256, (ch.n + CB - 1) / CB);
    hipLaunchKernelGGL((adj_march<CB, KSEG>), grid, dim3(256), 0, st, nsamp, npix, plane, ch, tape, dl, target, ckpt,
                       cot, cube_out);
    return hipGetLastError();
}

template <int CB, int G, bool CUBE>
static hipError_t launch_tau_t(int nsamp, int npix, int plane, const Channels &ch, float shift, const float4 *tape,
                               const int2 *span, const float *dl, const float *target, float4 *cot, float *cube_out,
                               hipStream_t st) {
    const int nblk = (ch.n + G * CB - 1) / (G * CB);
    const long tiles = (npix + 256 / G - 1) / (256 / G);
    const long ids = (tiles + 7) / 8 * 8 * nblk;
    hipLaunchKernelGGL((adj_march_tau<CB, G, CUBE>), dim3((unsigned)ids), dim3(256), 0, st, nsamp, npix, plane, nblk,
                       ch, shift, tape, span, dl, target, cot, cube_out);
    return hipGetLastError();
}

hipError_t launch_adj_march(int cb, int kseg, int lanes, int nsamp, int npix, int plane, const Channels &ch,
                            float shift, const float4 *tape, const int2 *span, const float *dl,
                            const float *target, float *ckpt,
                            float4 *cot, float *cube_out, hipStream_t st) {
    if (kseg == 0) {
        const bool cube = target || cube_out;
#define RT_TAU_CASE(C, G)                                                                                         \
    if (cb == C && lanes == G)                                                                                   \
        return cube ? launch_tau_t<C, G, true>(nsamp, npix, plane, ch, shift, tape, span, dl, target, cot, cube_out, st) \
                    : launch_tau_t<C, G, false>(nsamp, npix, plane, ch, shift, tape, span, dl, target, cot, cube_out, st);
        RT_TAU_CASE(8, 1) RT_TAU_CASE(16, 1) RT_TAU_CASE(24, 1) RT_TAU_CASE(32, 1)
        RT_TAU_CASE(16, 2) RT_TAU_CASE(24, 2) RT_TAU_CASE(25, 2) RT_TAU_CASE(32, 2)
        RT_TAU_CASE(12, 4) RT_TAU_CASE(16, 4)
#undef RT_TAU_CASE
        return hipErrorInvalidValue;
    }
    if (lanes != 1) return hipErrorInvalidValue;
#define RT_MARCH_CASE(C, K) \
    if (cb == C && kseg == K) return launch_march_t<C, K>(nsamp, npix, plane, ch, tape, dl, target, ckpt, cot, cube_out, st);
    RT_MARCH_CASE(8, 2) RT_MARCH_CASE(8, 4) RT_MARCH_CASE(8, 8) RT_MARCH_CASE(8, 16)
    RT_MARCH_CASE(16, 2) RT_MARCH_CASE(16, 4) RT_MARCH_CASE(16, 8)
    RT_MARCH_CASE(32, 2) RT_MARCH_CASE(32, 4)
#undef RT_MARCH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_adj_chain(const Geometry &g, const Shade &s, const float4 *rays, const int2 *span, const float4 *cot,
                            int nblk, const GradAcc &go, float4 *dO, hipStream_t st) {
    const size_t total = (size_t)g.nsamp * g.nx * g.ny;
    const int lds_surf = (s.nr <= 2048) ? 1 : 0;
    const size_t shmem = lds_surf ? sizeof(float) * 2 * s.nr : 0;
    if (grad_accum_double())
        hipLaunchKernelGGL(adj_chain<double>, dim3((unsigned)((total + 255) / 256)), dim3(256), shmem, st, g, s, rays,
                           span, cot, nblk, go, lds_surf, dO);
    else
        hipLaunchKernelGGL(adj_chain<float>, dim3((unsigned)((total + 255) / 256)), dim3(256), shmem, st, g, s, rays,
                           span, cot, nblk, go, lds_surf, dO);
    return hipGetLastError();
}

} // namespace rt
