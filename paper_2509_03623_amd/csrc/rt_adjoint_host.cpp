// rt_adjoint_host.cpp -- rt_render_cube_adjoint: scratch sizing and the
// three adjoint passes, all stream-ordered on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "rt_adjoint.h"
#include "rt_host.h"

namespace rt {

// Reverse-march shape (measured): of (channels per lane, lanes per pixel) =
// (32, 2), (24, 2), (16, 2), (32, 1), (24, 1), (25, 2) that still give 2048
// waves, the one padding the fewest channels, the earlier in that order on a
// tie (25 per lane is the pair form of a 50-channel batch);
// (32, 1) only when the march forms the intensity (without it that form
// spills registers); else (16, 1), or (8, 1) for at most 8 channels.  Pairs
// write one cotangent slice per 2 CB channels (at 512^2 x 64: 10.9 ms fused
// with (32, 2) against 11.8 ms with (32, 1)).  The checkpointed march
// (option) takes 8, 16 or 32 channels per lane and one lane per pixel.
void adjoint_shape(int nch, long npix, bool cube, int *cb, int *lanes, int *kseg) {
    *cb = nch > 8 ? 16 : 8;
    *lanes = 1;
    static const int cand[][2] = {{32, 2}, {24, 2}, {16, 2}, {32, 1}, {24, 1}, {25, 2}};
    int best = 1 << 30;
    for (const auto &cl : cand) {
        const int c = cl[0], gl = cl[1], grp = c * gl;
        const int nblk = (nch + grp - 1) / grp, padded = nblk * grp;
        if ((c == 32 && gl == 1 && !cube) || nch <= 16 || npix * nblk * gl < 2048L * 64) continue;
        if (padded < best) {
            best = padded;
            *cb = c;
            *lanes = gl;
        }
    }
    const int ocb = adjoint_block_option();
    if (ocb == 8 || ocb == 16 || ocb == 24 || ocb == 25 || ocb == 32) *cb = ocb;
    const int olanes = adjoint_lanes_option();
    if (olanes == 1 || olanes == 2) *lanes = olanes;
    if (olanes == 4) *lanes = 2;   // a pair, made four lanes at launch when the channels allow
    if (*cb == 25) *lanes = 2;   // 25 channels per lane only as a pair
    if (*lanes == 2 && *cb == 8) {
        // no 2 x 8 form: a pair asked for explicitly widens the block,
        // otherwise the 8-channel block keeps one lane per pixel
        if (olanes == 2) *cb = 16;
        else *lanes = 1;
    }
    *kseg = 0;
    const int opt = ckpt_segment_option();
    if (opt == 2 || opt == 4 || opt == 8 || opt == 16) *kseg = opt;
    if (*kseg) {
        // the checkpointed march has no 24- or 25-channel and no paired form
        *lanes = 1;
        if (*cb == 24 || *cb == 25) *cb = 16;
        if (*cb == 16 && *kseg == 16) *kseg = 8;
        if (*cb == 32 && *kseg > 4) *kseg = 4;
    }
}

size_t adjoint_bytes_per_pixel(int nch, long npix, int nsamp, bool cube) {
    int cb, lanes, kseg;
    adjoint_shape(std::min(nch, kLaunchChannels), npix, cube, &cb, &lanes, &kseg);
    const size_t ch = std::min(nch, kLaunchChannels), nblk = (ch + lanes * cb - 1) / (lanes * cb);
    const size_t nseg = kseg ? ((size_t)nsamp + kseg - 1) / kseg : 0;
    // tape, ray set-up, span, transmission checkpoints, per-block cotangents
    return 16 * (size_t)nsamp + 16 + 8 + 4 * nseg * nblk * cb + 16 * nblk * (size_t)nsamp;
}


static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// layout of a FixedScratch: partition table, accumulators, band scratch
static size_t fixed_table_bytes() { return align256(sizeof(float4) * (kZTableNodes - 1)); }
static size_t fixed_acc_bytes(const rt_problem *p) {
    const size_t nn = (size_t)p->grid.nr * p->grid.nz, nr = (size_t)p->grid.nr;
    return align256(sizeof(double) * (3 * nn + 2 * nr));
}

size_t fixed_scratch_min_bytes(const rt_problem *p) {
    const size_t row = adjoint_bytes_per_pixel(p->spec.nch, (long)p->cam.nx * p->cam.ny, p->nsamp, true) *
                       (size_t)p->cam.nx;
    return fixed_table_bytes() + fixed_acc_bytes(p) + row;
}

rt_status adjoint_core(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st,
                       const float4 *mlp_o, float4 *dO, const float *target, const FixedScratch *fx) {
    Geometry geo;
    Shade sh;
    hipError_t e;
    const float4 *ztab = nullptr;
    if (fx) {
        // the partition table goes to the head of the fixed region
        float4 tab[kZTableNodes - 1];
        partition_table_host(p->line, tab);
        e = hipMemcpyAsync(fx->base, tab, sizeof tab, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return fail_hip(e, "partition table upload");
        ztab = (const float4 *)fx->base;
    }
    rt_status rs = build_launch(p, &geo, &sh, ztab);
    if (rs != RT_OK) return rs;
    sh.mlp_o = mlp_o;
    const int npix = p->cam.nx * p->cam.ny;
    const int ns = p->nsamp;
    const size_t nn = (size_t)p->grid.nr * p->grid.nz, nr = (size_t)p->grid.nr;
    // gradients accumulate in float (double with RT_OPT_GRAD_ACCUM 1), then
    // overwrite the caller's float outputs
    const size_t acc_n = 3 * nn + 2 * nr;
    double *ab = fx ? (double *)(fx->base + fixed_table_bytes())
                    : (double *)stream_workspace(st, kWsGradAcc, sizeof(double) * acc_n, &e);
    if (!ab) return fail_hip(e, "gradient accumulators");
    if ((e = zero_async_d(ab, acc_n, st)) != hipSuccess) return fail_hip(e, "zero");
    GradAcc go{g->d_ln_nh2 ? ab : nullptr, g->d_temp_k ? ab + nn : nullptr, g->d_vphi_kms ? ab + 2 * nn : nullptr,
               g->d_z_lo_au ? ab + 3 * nn : nullptr, g->d_z_up_au ? ab + 3 * nn + nr : nullptr};
    int cb, lanes, kseg;
    const bool cube = target || cube_opt;
    adjoint_shape(std::min(p->spec.nch, kLaunchChannels), (long)p->cam.nx * p->cam.ny, cube, &cb, &lanes, &kseg);
    const int nseg = kseg ? (ns + kseg - 1) / kseg : 0;
    const size_t plane = (size_t)npix;
    const int nx = p->cam.nx, ny = p->cam.ny;
    // bands of image rows whose scratch fits the cap (at least one row)
    const size_t row_bytes = adjoint_bytes_per_pixel(p->spec.nch, (long)nx * ny, ns, cube) * (size_t)nx;
    // (as few bands as the cap allows, of equal height: a thin last band
    // would march its full rays on too few lanes)
    const size_t fx_band = fx ? fx->bytes - fixed_table_bytes() - fixed_acc_bytes(p) : 0;
    if (fx && fx->bytes < fixed_scratch_min_bytes(p))
        return fail(RT_ETOOBIG, "one row of adjoint scratch does not fit the fixed region");
    const size_t cap = fx ? fx_band : adjoint_scratch_cap();
    const int band_max = (int)std::max<size_t>(1, std::min<size_t>((size_t)ny, cap / row_bytes));
    const int nband = (ny + band_max - 1) / band_max;
    const int band = (ny + nband - 1) / nband;
    const bool lds = chain_lds_fits(p->grid.nr, p->grid.nz);
    for (int c0 = 0; c0 < p->spec.nch; c0 += kLaunchChannels) {
        Channels ch;
        std::memset(&ch, 0, sizeof ch);
        ch.n = std::min(kLaunchChannels, p->spec.nch - c0);
        for (int c = 0; c < ch.n; ++c) ch.v[c] = (float)p->spec.v_kms[c0 + c];
        const int nblk = (ch.n + lanes * cb - 1) / (lanes * cb);   // cotangent slices
        // a pair of 32- or 24-channel lanes becomes four lanes of 16 or 12
        // (same slices) when the channels are uniformly spaced in those groups
        int cb_l = cb, lanes_l = lanes;
        double shift = 0.0;
        if (kseg == 0 && lanes == 2 && (cb == 32 || cb == 24) && adjoint_lanes_option() != 2 &&
            group_shift(p->spec.v_kms + c0, ch.n, 4, cb / 2, &shift)) {
            cb_l = cb / 2;
            lanes_l = 4;
        }
        for (int q0 = 0; q0 < ny; q0 += band) {
            const int rows = std::min(band, ny - q0);
            const int bpix = rows * nx;
            const size_t pix0 = (size_t)q0 * nx;
            Geometry gb = geo;
            gb.ny = rows;
            gb.yc = 0.5 * ny - q0;
            Shade sb = sh;
            sb.o_pix0 = (int64_t)pix0;
            const size_t tape_b = sizeof(float4) * (size_t)ns * bpix;
            const size_t rays_b = sizeof(float4) * (size_t)bpix;
            const size_t span_b = sizeof(int2) * (size_t)bpix;
            const size_t ckpt_b = sizeof(float) * (size_t)nseg * nblk * cb * bpix;
            const size_t cot_b = sizeof(float4) * (size_t)nblk * ns * bpix;
            char *base = fx ? fx->base + fixed_table_bytes() + fixed_acc_bytes(p)
                            : (char *)stream_workspace(st, kWsAdjoint, tape_b + rays_b + ckpt_b + cot_b + span_b, &e);
            if (!base) return fail_hip(e, "adjoint scratch");
            float4 *tape = (float4 *)base;
            float4 *rays = (float4 *)(base + tape_b);
            float *ckpt = (float *)(base + tape_b + rays_b);
            float4 *cot = (float4 *)(base + tape_b + rays_b + ckpt_b);
            int2 *span = (int2 *)(base + tape_b + rays_b + ckpt_b + cot_b);   // last: 8-byte records
            // the checkpointed march reads every tape entry
            if ((e = launch_adj_tape(gb, sb, tape, rays, span, kseg == 0, st)) != hipSuccess)
                return fail_hip(e, "adjoint tape");
            const size_t off = (size_t)c0 * plane + pix0;
            if ((e = launch_adj_march(cb_l, kseg, lanes_l, ns, bpix, (int)plane, ch, (float)shift, tape, span,
                                      dl ? dl + off : nullptr, target ? target + off : nullptr, ckpt, cot,
                                      cube_opt ? cube_opt + off : nullptr, st)) != hipSuccess)
                return fail_hip(e, "adjoint march");
            float4 *dOc = c0 == 0 ? dO : nullptr;
            e = lds ? launch_adj_chain_lds(gb, sb, rays, span, cot, nblk, go, dOc, st)
                    : launch_adj_chain(gb, sb, rays, span, cot, nblk, go, dOc, st);
            if (e != hipSuccess) return fail_hip(e, "adjoint chain");
        }
    }
    // accumulators are double or float (option), at the offsets of the double layout
    auto acc_out = [&](size_t off, float *dst, size_t n) {
        return grad_accum_double() ? to_float_async(ab + off, dst, n, st)
                                   : copy_float_async((const float *)(ab + off), dst, n, st);
    };
    if ((e = acc_out(0, g->d_ln_nh2, nn)) != hipSuccess ||
        (e = acc_out(nn, g->d_temp_k, nn)) != hipSuccess ||
        (e = acc_out(2 * nn, g->d_vphi_kms, nn)) != hipSuccess ||
        (e = acc_out(3 * nn, g->d_z_lo_au, nr)) != hipSuccess ||
        (e = acc_out(3 * nn + nr, g->d_z_up_au, nr)) != hipSuccess)
        return fail_hip(e, "gradient output");
    return RT_OK;
}

rt_status adjoint_grid(const rt_problem *p, const float *dl, const rt_grads *g, float *cube_opt, hipStream_t st,
                       const float *target) {
    return adjoint_core(p, dl, g, cube_opt, st, nullptr, nullptr, target);
}

} // namespace rt

using namespace rt;

extern "C" rt_status rt_render_cube_l2_adjoint(const rt_problem *p, const float *target, const rt_grads *g,
                                               float *cube, double *loss, void *stream) {
    rt_status st = validate(p);
    if (st != RT_OK) return st;
    if (!target || !cube) return fail(RT_EINVAL, "target and cube must not be NULL");
    if (!g) return fail(RT_EINVAL, "grads is NULL");
    if (p->spec.nch > kLaunchChannels)
        return fail(RT_EINVAL, "the fused L2 adjoint takes at most %d channels per call", kLaunchChannels);
    hipStream_t s = (hipStream_t)stream;
    if (p->mlp) st = adjoint_mlp(p, nullptr, g, cube, s, target);
    else if (g->d_mlp) return fail(RT_EINVAL, "d_mlp requested but the problem has no network");
    else st = adjoint_grid(p, nullptr, g, cube, s, target);
    if (st != RT_OK || !loss) return st;
    const size_t n = (size_t)p->spec.nch * p->cam.nx * p->cam.ny;
    const hipError_t e = launch_l2_value(cube, target, n, loss, s);
    return e == hipSuccess ? RT_OK : fail_hip(e, "loss");
}

extern "C" rt_status rt_render_cube_adjoint(const rt_problem *p, const float *dl_dcube, const rt_grads *g,
                                            float *cube_opt, void *stream) {
    rt_status st = validate(p);
    if (st != RT_OK) return st;
    if (!dl_dcube) return fail(RT_EINVAL, "dl_dcube is NULL");
    if (!g) return fail(RT_EINVAL, "grads is NULL");
    if (p->mlp) return adjoint_mlp(p, dl_dcube, g, cube_opt, (hipStream_t)stream);
    if (g->d_mlp) return fail(RT_EINVAL, "d_mlp requested but the problem has no network");
    return adjoint_grid(p, dl_dcube, g, cube_opt, (hipStream_t)stream);
}
