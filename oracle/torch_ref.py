"""Float64 torch (CPU) mirror of the oracle, for gradients.

TEST INFRASTRUCTURE (see the package docstring).  The forward quantity is
the same discrete march as ``rt_oracle.c`` (Methods, "Line Radiative
Transfer": Eqs. rt-int and optical_depth, LTE j and beta, Gaussian Doppler
profile), written with tensor operations vectorised over pixels and channels
and a Python loop over samples.  The positions of the samples do not depend
on any differentiable input, so they are computed once in numpy float64; the
fields, surfaces and network weights are torch leaves whose autograd
gradients are the exact derivatives of the discrete forward (at the clamp
kinks, the branch that was taken).
"""
from __future__ import annotations

import math

import numpy as np
import torch

H = 6.62607015e-27
KB = 1.380649e-16
CL = 2.99792458e10
AMU = 1.66053906660e-24
AU = 1.495978707e13

NF = 16
WIDTH = 128


def as_leaves(prob, requires_grad=True):
    """Field tensors (float64 promotions of the float32 inputs)."""
    t = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=torch.float64, requires_grad=requires_grad)
    d = dict(ln_nh2=t(prob.ln_nh2), temp_k=t(prob.temp_k), vphi_kms=t(prob.vphi_kms),
             z_lo_au=t(prob.z_lo_au), z_up_au=t(prob.z_up_au))
    if getattr(prob, "mlp_w", None) is not None:
        d["mlp_w"] = t(prob.mlp_w)
    return d


def mlp_eval(w, rh, zh):
    """Neural CO-layer network on normalised coordinates (tensors [n]) -> [n, 3]."""
    f = torch.tensor([2.0 ** (3.0 * k / 15.0) for k in range(NF)], dtype=torch.float64)
    ar = math.pi * rh[:, None] * f[None, :]
    az = math.pi * zh[:, None] * f[None, :]
    x = torch.cat([torch.sin(ar), torch.cos(ar), torch.sin(az), torch.cos(az)], dim=1)
    off = 0
    dims = [4 * NF, WIDTH, WIDTH, WIDTH, WIDTH, 3]
    for li in range(5):
        i, o = dims[li], dims[li + 1]
        W = w[off:off + o * i].view(o, i)
        off += o * i
        b = w[off:off + o]
        off += o
        x = x @ W.T + b
        if li < 4:
            x = x * torch.sigmoid(x)
    return x


def pixel_chords(prob, px, py):
    """Per-pixel (x', y', s_a, s_b, valid) in float64 numpy."""
    g, cam = prob.grid, prob.camera
    d = cam.fov_au / cam.nx
    X = (px + 0.5 - 0.5 * cam.nx) * d
    Y = (py + 0.5 - 0.5 * cam.ny) * d
    pa = math.radians(cam.pa_deg)
    xp = math.cos(pa) * X - math.sin(pa) * Y
    yp = math.sin(pa) * X + math.cos(pa) * Y
    dln = math.log(g.r_max_au / g.r_min_au) / (g.nr - 1)
    dzr = g.zr_max / (g.nz - 1)
    Rc = g.r_max_au * math.exp(dln)
    Zc = (g.zr_max + dzr) * Rc
    ang = math.radians(cam.incl_deg)
    si, ci = math.sin(ang), math.cos(ang)
    lo = np.full(xp.shape, -np.inf)
    hi = np.full(xp.shape, np.inf)
    ok = xp * xp < Rc * Rc
    qq = np.sqrt(np.maximum(Rc * Rc - xp * xp, 0.0))
    if si > 0:
        lo = np.maximum(lo, (-yp * ci - qq) / si)
        hi = np.minimum(hi, (-yp * ci + qq) / si)
    else:
        ok &= np.abs(yp * ci) <= qq
    if ci > 0:
        lo = np.maximum(lo, (yp * si - Zc) / ci)
        hi = np.minimum(hi, (yp * si + Zc) / ci)
    else:
        ok &= np.abs(yp * si) <= Zc
    ok &= hi > lo
    lo = np.where(ok, lo, 0.0)
    hi = np.where(ok, hi, 0.0)
    return xp, yp, lo, hi, ok


def render(prob, leaves=None, px=None, py=None):
    """Intensities [npix, nch] (float64 tensor) of the given pixels (default:
    every pixel, row-major q, p)."""
    g, cam, line = prob.grid, prob.camera, prob.line
    if leaves is None:
        leaves = as_leaves(prob, requires_grad=False)
    if px is None:
        qq, pp = np.meshgrid(np.arange(cam.ny), np.arange(cam.nx), indexing="ij")
        px, py = pp.ravel(), qq.ravel()
    px = np.asarray(px, np.float64)
    py = np.asarray(py, np.float64)
    xp, yp, sa, sb, ok = pixel_chords(prob, px, py)
    ns = prob.nsamp
    ds = (sb - sa) / ns
    ang = math.radians(cam.incl_deg)
    si, ci = math.sin(ang), math.cos(ang)
    dln = math.log(g.r_max_au / g.r_min_au) / (g.nr - 1)
    dzr = g.zr_max / (g.nz - 1)
    vch = torch.tensor(np.asarray(prob.v_kms, np.float64))
    lev_e = torch.tensor(np.asarray(line.lev_e_k, np.float64))
    lev_g = torch.tensor(np.asarray(line.lev_g, np.float64))
    nu0 = line.nu0_hz
    bul = line.a_ul * CL * CL / (2 * H * nu0 ** 3)
    blu = line.g_u / line.g_l * bul
    pre = H * nu0 / (4 * math.pi)
    lnf = leaves["ln_nh2"].reshape(-1)
    tf = leaves["temp_k"].reshape(-1)
    vf = leaves["vphi_kms"].reshape(-1)
    zlo_f, zup_f = leaves["z_lo_au"], leaves["z_up_au"]
    w_mlp = leaves.get("mlp_w") if getattr(prob, "mlp_w", None) is not None else None
    npix, nch = len(px), len(prob.v_kms)
    I = torch.zeros(npix, nch, dtype=torch.float64)
    tr = torch.ones(npix, nch, dtype=torch.float64)
    okt = torch.tensor(ok)
    dscm = torch.tensor(ds * AU)
    for k in range(ns):
        s = sa + (k + 0.5) * ds
        pxk = xp
        pyk = yp * ci + s * si
        pzk = yp * si - s * ci
        rho = np.sqrt(pxk * pxk + pyk * pyk)
        a = np.abs(pzk)
        live = ok & (rho > 0)
        rs = np.where(live, rho, 1.0)
        u = np.log(rs / g.r_min_au) / dln
        v = (a / rs) / dzr
        uc = np.clip(u, 0, g.nr - 1)
        vc = np.clip(v, 0, g.nz - 1)
        i0 = np.minimum(np.floor(uc), g.nr - 2).astype(np.int64)
        j0 = np.minimum(np.floor(vc), g.nz - 2).astype(np.int64)
        fu = torch.tensor(uc - i0)
        fv = torch.tensor(vc - j0)
        n00 = torch.tensor(i0 * g.nz + j0)
        idx = [n00, n00 + 1, n00 + g.nz, n00 + g.nz + 1]
        wts = [(1 - fu) * (1 - fv), (1 - fu) * fv, fu * (1 - fv), fu * fv]

        def bil(F):
            return sum(w_ * F[i_] for w_, i_ in zip(wts, idx))

        ln_n = bil(lnf)
        t = bil(tf)
        vphi = bil(vf)
        i0t = torch.tensor(i0)
        zlo = (1 - fu) * zlo_f[i0t] + fu * zlo_f[i0t + 1]
        zup = (1 - fu) * zup_f[i0t] + fu * zup_f[i0t + 1]
        rho_t = torch.tensor(rs)
        a_t = torch.tensor(a)
        if w_mlp is not None:
            rh = torch.tensor(np.clip(u, -1.0, g.nr) / (g.nr - 1))
            zh = torch.tensor(np.clip(v, 0.0, g.nz) / (g.nz - 1))
            o = mlp_eval(w_mlp, rh, zh)
            zup = g.zr_max * rho_t * torch.sigmoid(o[:, 0])
            zlo = g.zr_max * rho_t * torch.sigmoid(o[:, 1])
            t = t * torch.exp(0.5 * torch.tanh(o[:, 2]))
        taper = np.clip(u + 1, 0, 1) * np.clip(g.nr - u, 0, 1) * np.clip(g.nz - v, 0, 1)
        taper = torch.tensor(np.where(live, taper, 0.0))
        nh2 = torch.exp(ln_n) * taper
        w = prob.mask_width * rho_t * dzr
        mask = torch.sigmoid((zup - a_t) / w) * torch.sigmoid((a_t - zlo) / w)
        nco = prob.x_co * mask * nh2
        zpart = torch.sum(lev_g[None, :] * torch.exp(-lev_e[None, :] / t[:, None]), dim=1)
        n_u = nco * line.g_u * torch.exp(-line.e_u_k / t) / zpart
        n_l = nco * line.g_l * torch.exp(-line.e_l_k / t) / zpart
        jbar = pre * n_u * line.a_ul
        kbar = pre * (n_l * blu - n_u * bul)
        pos = kbar > 0
        S = torch.where(pos, jbar / torch.where(pos, kbar, torch.ones_like(kbar)), torch.zeros_like(kbar))
        th = 2 * KB * t / (line.m_co_amu * AMU)
        cs2 = 2 * KB * t / (line.m_mol_amu * AMU)
        alpha = torch.sqrt(th + prob.v_turb ** 2 * cs2) / 1e5
        vlos = prob.v_sys_kms + vphi * si * torch.tensor(pxk / rs)
        d = (vlos[:, None] - vch[None, :]) / alpha[:, None]
        phi = (CL / nu0) / (alpha[:, None] * 1e5 * math.sqrt(math.pi)) * torch.exp(-d * d)
        dtau = kbar[:, None] * phi * dscm[:, None]
        dtau = torch.where(okt[:, None], dtau, torch.zeros_like(dtau))
        I = I + tr * S[:, None] * (-torch.expm1(-dtau))
        tr = tr * torch.exp(-dtau)
    return I * prob.intensity_scale


def cube(prob, leaves=None):
    """Whole-image cube [nch][ny][nx] (float64 tensor)."""
    I = render(prob, leaves)
    return I.T.reshape(len(prob.v_kms), prob.camera.ny, prob.camera.nx)


def loss_and_grad(prob, target, chunk=4096):
    """L = sum (I - D)^2 over the cube and dL/d{ln n, T, v_phi, z_lo, z_up
    [, mlp_w]} as float64 numpy arrays.  Pixels are processed in chunks (the
    loss is a sum over pixels) to bound autograd memory."""
    cam = prob.camera
    leaves = as_leaves(prob)
    qq, pp = np.meshgrid(np.arange(cam.ny), np.arange(cam.nx), indexing="ij")
    px, py = pp.ravel(), qq.ravel()
    D = torch.tensor(np.asarray(target, np.float64).reshape(len(prob.v_kms), -1).T)
    total = 0.0
    for s in range(0, len(px), chunk):
        I = render(prob, leaves, px[s:s + chunk], py[s:s + chunk])
        r = I - D[s:s + chunk]
        L = torch.sum(r * r)
        L.backward()
        total += float(L.detach())
    grads = {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape)) for k, v in leaves.items()}
    return total, grads
