"""FP64 oracle of the fields derived from a temperature grid.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU leg use this module.  It is plain float64 torch on
the CPU, written step by step from Methods, "Parametric Disk Modeling" and
"Neural Temperature Recovery" (physics-informed constraints), so that its
autograd gradients are the exact derivatives of the discrete chain (with the
crossing nodes of the two surfaces held at the ones the forward picked).

Discrete definitions (the readings are listed with the design notes):
  * grid: r_i = r_min (r_max/r_min)^(i/(nr-1)) au, zeta_j = zr_max j/(nz-1),
    heights z_ij = zeta_j r_i; the temperature T_ij is the input;
  * hydrostatic equilibrium, Eq. gas_density_temp, integrated upward from the
    midplane of each column: with the gravity integrand
    g_j = G M* m_mol z_j / (k_B T_j (r^2 + z_j^2)^(3/2)), the trapezoid sum
    I_j over the nodes below j, and the log-T term taken exactly,
    l_j = ln rho_j - ln rho_0 = -I_j - ln T_j + ln T_0;
  * normalisation: 2 * (trapezoid integral of rho over 0 <= z <= z_top) equals
    the tapered power-law surface density Sigma(r) = Sigma0 (r/rc)^-gamma
    exp(-(r/rc)^(2-gamma)), Sigma0 = M_gas (2 - gamma) / (2 pi rc^2);
    n_H2 = rho / m_mol with m_mol = mu m_H;
  * column density, Eq. column_density: trapezoid rule from each node up to
    the top node (zero there);
  * CO surfaces, Eq. co_layer: z_up where 0.706 N = N_dissoc, log-linear
    between the last node above the threshold and the next (linear if the next
    is the top node, where N = 0); -zr_max r when even the midplane is below
    it, the top node's height when the top node is still above it.  z_lo
    where T first exceeds T_freeze going up, linear in T between the two
    nodes; -zr_max r for a warm midplane, 2 zr_max r for a column that is
    never warm;
  * azimuthal velocity, Eq. gas_velocity_pressure: v^2 = G M* r^2 /
    (r^2 + z^2)^(3/2) + (k_B T / m_mol) (d ln P/d u - zeta d ln P/d zeta) with
    u = ln r, P = n k_B T, central differences on the node grid (one-sided at
    its edges); v = sqrt(max(v^2, 0)).
"""
from __future__ import annotations

import math

import numpy as np
import torch

# cgs constants (CODATA 2018, IAU 2015 nominal), typed for this module
G = 6.67430e-8
MSUN = 1.98847e33
AU = 1.495978707e13
KB = 1.380649e-16
MH = 1.6735575e-24
PHOTO_FACTOR = 0.706   # vertical H2 column -> total gas column, Eq. co_layer


def nodes(nr, nz, r_min_au, r_max_au, zr_max):
    """Radial nodes [au] and z/r nodes, float64 numpy."""
    r = r_min_au * (r_max_au / r_min_au) ** (np.arange(nr) / (nr - 1))
    zr = zr_max * np.arange(nz) / (nz - 1)
    return r, zr


def surface_density(r_au, mgas_msun, rc_au, gamma):
    """Sigma(r) [g cm^-2] of the tapered power law holding the mass M_gas."""
    rc = rc_au * AU
    sig0 = mgas_msun * MSUN * (2.0 - gamma) / (2.0 * math.pi * rc * rc)
    x = np.asarray(r_au, np.float64) / rc_au
    return sig0 * x ** (-gamma) * np.exp(-x ** (2.0 - gamma))


def _trap_segments(f, dz):
    """Trapezoid areas of the segments between consecutive nodes (last axis)."""
    return 0.5 * (f[..., :-1] + f[..., 1:]) * dz


def hydrostatic_ln_n(T, r_au, zr, mstar_msun, mu, sigma):
    """ln n_H2 [cm^-3] per node from Eq. gas_density_temp and Sigma(r)."""
    r = torch.as_tensor(r_au, dtype=torch.float64)[:, None]
    z = r * torch.as_tensor(zr, dtype=torch.float64)[None, :]            # au
    m_mol = mu * MH
    # gravity integrand per cm of height, with z and r in cm
    g = G * mstar_msun * MSUN * m_mol * (z * AU) / (KB * T * ((r * AU) ** 2 + (z * AU) ** 2) ** 1.5)
    dz = (z[:, 1:] - z[:, :-1]) * AU
    I = torch.cat([torch.zeros_like(g[:, :1]), torch.cumsum(_trap_segments(g, dz), dim=1)], dim=1)
    ell = -I - torch.log(T) + torch.log(T[:, :1])
    col = 2.0 * _trap_segments(torch.exp(ell), dz).sum(dim=1)             # g/cm^2 per unit rho_0
    ln_rho0 = torch.log(torch.as_tensor(sigma, dtype=torch.float64)) - torch.log(col)
    return ln_rho0[:, None] + ell - math.log(m_mol)


def column(n, r_au, zr):
    """Vertical H2 column [cm^-2] from each node to the top node."""
    r = torch.as_tensor(r_au, dtype=torch.float64)[:, None]
    dz = r * torch.as_tensor(np.diff(zr), dtype=torch.float64)[None, :] * AU
    seg = _trap_segments(n, dz)
    tail = torch.flip(torch.cumsum(torch.flip(seg, dims=[1]), dim=1), dims=[1])
    return torch.cat([tail, torch.zeros_like(n[:, :1])], dim=1)


def co_surfaces(N, T, r_au, zr, zr_max, t_freeze_k, n_dissoc):
    """(z_lo, z_up) [au] per radial node, Eq. co_layer."""
    thr = n_dissoc / PHOTO_FACTOR
    Nd, Td = N.detach().numpy(), T.detach().numpy()
    nr, nz = Nd.shape
    zlo, zup = [], []
    for i in range(nr):
        z = zr * r_au[i]
        if Nd[i, 0] <= thr:
            zup.append(torch.tensor(-zr_max * r_au[i], dtype=torch.float64))
        else:
            a = int(np.nonzero(Nd[i] > thr)[0].max())
            b = a + 1
            if b == nz:
                zup.append(torch.tensor(z[-1], dtype=torch.float64))   # shielded up to the top node
            elif Nd[i, b] > 0:
                f = (math.log(thr) - torch.log(N[i, a])) / (torch.log(N[i, b]) - torch.log(N[i, a]))
            else:
                f = (thr - N[i, a]) / (N[i, b] - N[i, a])
            if b < nz:
                zup.append(z[a] + f * (z[b] - z[a]))
        if Td[i, 0] > t_freeze_k:
            zlo.append(torch.tensor(-zr_max * r_au[i], dtype=torch.float64))
        else:
            warm = np.nonzero(Td[i] > t_freeze_k)[0]
            if len(warm) == 0:
                zlo.append(torch.tensor(2.0 * zr_max * r_au[i], dtype=torch.float64))
            else:
                b = int(warm[0])
                a = b - 1
                f = (t_freeze_k - T[i, a]) / (T[i, b] - T[i, a])
                zlo.append(z[a] + f * (z[b] - z[a]))
    return torch.stack(zlo), torch.stack(zup)


def _diff_central(x, coord, dim):
    """d x / d coord along dim: central inside, one-sided at both ends."""
    n = x.shape[dim]
    lo = np.maximum(np.arange(n) - 1, 0)
    hi = np.minimum(np.arange(n) + 1, n - 1)
    c = torch.as_tensor(coord[hi] - coord[lo], dtype=torch.float64)
    xl, xh = torch.index_select(x, dim, torch.as_tensor(lo)), torch.index_select(x, dim, torch.as_tensor(hi))
    shape = [1, 1]
    shape[dim] = n
    return (xh - xl) / c.view(shape)


def vphi_kms(ln_n, T, r_au, zr, mstar_msun, mu):
    """Azimuthal velocity [km/s] with the radial pressure term."""
    r = np.asarray(r_au, np.float64)
    rr = torch.as_tensor(r, dtype=torch.float64)[:, None] * AU
    zz = rr * torch.as_tensor(zr, dtype=torch.float64)[None, :]
    lnP = ln_n + torch.log(T)
    d_u = _diff_central(lnP, np.log(r), 0)
    d_zeta = _diff_central(lnP, np.asarray(zr, np.float64), 1)
    grav = G * mstar_msun * MSUN * rr ** 2 / (rr ** 2 + zz ** 2) ** 1.5
    press = KB * T / (mu * MH) * (d_u - torch.as_tensor(zr, dtype=torch.float64)[None, :] * d_zeta)
    v2 = grav + press
    pos = v2 > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, v2, torch.ones_like(v2))), torch.zeros_like(v2)) / 1e5


def derive_fields(T, grid, mstar_msun, mgas_msun, rc_au, gamma, mu, t_freeze_k, n_dissoc):
    """The whole chain: T [nr][nz] (float64 tensor) -> dict of ln_nh2,
    vphi_kms [nr][nz] and z_lo_au, z_up_au [nr].  grid: (nr, nz, r_min_au,
    r_max_au, zr_max)."""
    nr, nz, r_min, r_max, zr_max = grid
    r, zr = nodes(nr, nz, r_min, r_max, zr_max)
    ln_n = hydrostatic_ln_n(T, r, zr, mstar_msun, mu, surface_density(r, mgas_msun, rc_au, gamma))
    N = column(torch.exp(ln_n), r, zr)
    z_lo, z_up = co_surfaces(N, T, r, zr, zr_max, t_freeze_k, n_dissoc)
    return dict(ln_nh2=ln_n, vphi_kms=vphi_kms(ln_n, T, r, zr, mstar_msun, mu), z_lo_au=z_lo, z_up_au=z_up)


def parametric_temperature(nr, nz, r_min_au, r_max_au, zr_max, t_mid0_k, t_atm0_k, q, r_scale_au, zq0_au, delta):
    """Two-layer temperature of Methods, "Parametric Disk Modeling": midplane
    and atmosphere radial power laws T_mid = t_mid0 (r/r_scale)^q, T_atm =
    t_atm0 (r/r_scale)^q, blended as T_atm + (T_mid - T_atm) cos^(2 delta)(pi
    z / (2 z_q)) below z_q(r) = zq0 (r/r_scale)^1.3 and T_atm above, at the
    grid nodes (float64 numpy [nr][nz])."""
    r, zr = nodes(nr, nz, r_min_au, r_max_au, zr_max)
    R, ZR = np.meshgrid(r, zr, indexing="ij")
    z = ZR * R
    x = R / r_scale_au
    t_mid = t_mid0_k * x ** q
    t_atm = t_atm0_k * x ** q
    zq = zq0_au * x ** 1.3
    blend = np.where(z < zq, np.cos(np.pi * z / (2.0 * zq)) ** (2.0 * delta), 0.0)
    return t_atm + (t_mid - t_atm) * blend
