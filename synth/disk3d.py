"""Seeded 3-D spherical-grid disks (non-axisymmetric) for the 3-D renderer.

The fields of the parametric disk (two-layer temperature, Gaussian density of
the tapered surface density, height-dependent Keplerian v_phi) are laid on a
spherical node grid (r log-spaced, polar angle theta in a wedge about the
midplane, phi periodic), then made non-axisymmetric: a two-armed logarithmic
spiral in the density and a small radial velocity following it.  The CO
abundance field is x_co between the freeze-out and photodissociation surfaces
of the axisymmetric disk, 0 elsewhere.  The 512 x 96 x 256 shape is the one of
the hydrodynamic simulation the paper benchmarks on.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import disk as D


@dataclass
class Grid3Spec:
    nr: int
    nt: int
    nphi: int
    r_min_au: float = 5.0
    r_max_au: float = 400.0
    th_min: float = 0.5 * np.pi - 0.5
    th_max: float = 0.5 * np.pi + 0.5


@dataclass
class Problem3:
    grid: Grid3Spec
    ln_nh2: np.ndarray       # float32 [nr, nt, nphi]
    temp_k: np.ndarray
    v_r_kms: np.ndarray
    v_theta_kms: np.ndarray
    v_phi_kms: np.ndarray
    x_co: np.ndarray
    camera: D.Camera
    v_kms: np.ndarray
    line: D.LineData
    nsamp: int
    v_sys_kms: float = 0.0
    v_turb: float = 0.05
    intensity_scale: float = 1.0

    def replace(self, **kw):
        return replace(self, **kw)


def make_problem3(grid: Grid3Spec, seed: int = 50, *, nx: int, ny: int, nch: int, dv: float, nsamp: int,
                  incl: float = 40.0, pa: float = 0.0, x_co: float = 1e-4, spiral: float = 0.3,
                  inflow: float = 0.05, noise: float = 0.05, fov_au: float | None = None) -> Problem3:
    p = D.DiskParams()
    rng = np.random.Generator(np.random.PCG64(seed))
    r = grid.r_min_au * (grid.r_max_au / grid.r_min_au) ** (np.arange(grid.nr) / (grid.nr - 1))
    th = grid.th_min + (grid.th_max - grid.th_min) * np.arange(grid.nt) / (grid.nt - 1)
    ph = 2.0 * np.pi * np.arange(grid.nphi) / grid.nphi
    R3 = r[:, None] * np.sin(th)[None, :]                    # cylindrical radius [nr, nt]
    Z3 = np.abs(r[:, None] * np.cos(th)[None, :])
    T, t_mid = D._temperature(R3, Z3, p)
    cs2 = D._KB * t_mid / (D.MU_GAS * D._MH)
    om2 = D._G * p.mstar_msun * D._MSUN / (R3 * D._AU) ** 3
    h = np.sqrt(cs2 / om2) / D._AU
    sig = D._surface_density(R3, p)
    rho = sig / (np.sqrt(2 * np.pi) * h * D._AU) * np.exp(-Z3 ** 2 / (2 * h ** 2))
    n = np.maximum(rho / (D.MU_GAS * D._MH), 1e-30)
    # CO surfaces of the axisymmetric disk on a fine (r, z/r) grid, then looked up
    g2 = D.GridSpec(nr=256, nz=128, r_min_au=1.0, r_max_au=800.0, zr_max=1.0)
    with np.errstate(divide="ignore"):
        _, _, _, z_lo, z_up = D.make_disk(g2, replace(p, noise_sigma=0.0), seed)
    r2 = g2.r_nodes()
    zl = np.interp(R3, r2, z_lo)
    zu = np.interp(R3, r2, z_up)
    xco = np.where((Z3 >= zl) & (Z3 <= zu), x_co, 0.0)
    # two-armed logarithmic spiral in the density, radial inflow along the arms
    arm = np.cos(2.0 * (ph[None, None, :] - 3.0 * np.log(R3[:, :, None] / 100.0)))
    ln_n = np.log(n)[:, :, None] + np.log1p(spiral * arm) + noise * rng.standard_normal((grid.nr, grid.nt, grid.nphi))
    vk = np.sqrt(D._G * p.mstar_msun * D._MSUN / (R3 * D._AU)) * (1 + (Z3 / R3) ** 2) ** -0.75 / 1e5
    vphi = np.broadcast_to(vk[:, :, None], ln_n.shape)
    vr = -inflow * vk[:, :, None] * arm
    f32 = lambda a: np.ascontiguousarray(np.broadcast_to(a, ln_n.shape), dtype=np.float32)
    cam = D.Camera(nx=nx, ny=ny, fov_au=2.2 * grid.r_max_au if fov_au is None else fov_au, incl_deg=incl,
                   pa_deg=pa, dist_pc=100.0)
    return Problem3(grid=grid, ln_nh2=f32(ln_n), temp_k=f32(T[:, :, None]), v_r_kms=f32(vr),
                    v_theta_kms=f32(np.zeros(1)), v_phi_kms=f32(vphi), x_co=f32(xco[:, :, None]), camera=cam,
                    v_kms=D.channels(nch, dv, 0.0), line=D.co21_line(), nsamp=nsamp,
                    intensity_scale=D.rj_kelvin_scale(D.co21_line()))


def uniform_problem3(grid: Grid3Spec, *, temp: float = 40.0, ln_n: float = np.log(1e6), x_co: float = 1e-4,
                     v=(0.0, 0.0, 0.0), nx: int = 9, ny: int = 9, nch: int = 5, dv: float = 0.1, nsamp: int = 256,
                     incl: float = 90.0, pa: float = 0.0, fov_au: float | None = None) -> Problem3:
    """Constant fields (T, n_H2, x_CO, velocity components) on a spherical grid."""
    shape = (grid.nr, grid.nt, grid.nphi)
    full = lambda x: np.full(shape, x, np.float32)
    cam = D.Camera(nx=nx, ny=ny, fov_au=2.2 * grid.r_max_au if fov_au is None else fov_au, incl_deg=incl,
                   pa_deg=pa, dist_pc=100.0)
    return Problem3(grid=grid, ln_nh2=full(ln_n), temp_k=full(temp), v_r_kms=full(v[0]), v_theta_kms=full(v[1]),
                    v_phi_kms=full(v[2]), x_co=full(x_co), camera=cam, v_kms=D.channels(nch, dv, 0.0),
                    line=D.co21_line(), nsamp=nsamp, intensity_scale=1.0)
