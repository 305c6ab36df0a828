"""Pins of the 2-D oracle's grid fetch (O5) and CO mask (S6).

The oracle samples the fields bilinearly in (ln r, z/r) index space with
clamp-to-edge, fades the density linearly to zero over one cell beyond the
grid, interpolates the two surface heights linearly in the log-radius index,
and multiplies the CO abundance by a logistic mask of width
w = mask_width * rho * (z/r spacing).  These tests fix each of those choices
from outside the oracle's formulas:

* a field that is linear in the node indices (i, j) must come back exactly
  at any point, because bilinear interpolation reproduces linear functions;
  the point is placed here from the grid's own definition (r_i log-spaced,
  z/r linear), so a different index map or a swapped weight fails;
* each field is read back through a quantity that depends on it alone
  (ln n through the upper-level density, T through the line width, v_phi
  through the projected velocity, the surfaces through the mask);
* the mask's logit is linear in height with slope 1/w, which fixes w, and
  its zero crossing is the surface height;
* half a cell beyond each edge the density is exactly halved, a full cell
  beyond it is zero.

Methods, Line RT (log-spaced grids) and Eq. co_layer; the readings S4-S6.
The same checks run against planted mistakes in ``test_oracle_mutants.py``.
"""
import math

import numpy as np
import pytest

import oracle
import synth

# CODATA 2018 cgs, typed here on their own
KB = 1.380649e-16
AMU = 1.66053906660e-24

NR, NZ = 12, 9
GRID = dict(r_min_au=5.0, r_max_au=200.0, zr_max=0.5)
T0 = 40.0
LN_N0 = math.log(1e6)
FAR = 1.0e6          # a surface this far away leaves its mask factor at exactly 1
INCL, PHI, VSYS = 30.0, 0.4, 0.3

# (u, v) index-space points: interior (with f_u != f_v), and the clamped
# border regions on every side
INTERIOR = [(3.25, 2.5), (0.125, 7.75), (10.6, 0.3), (5.5, 4.0), (7.9, 6.15)]
CLAMPED = [(11.5, 3.3), (-0.5, 2.2), (4.3, 8.6), (11.7, 8.9), (-0.25, 0.4)]


def _base(**fields):
    g = synth.GridSpec(nr=NR, nz=NZ, **GRID)
    prob = synth.slab_problem(nr=NR, nz=NZ)
    prob = prob.replace(grid=g, camera=synth.Camera(nx=4, ny=4, fov_au=400.0, incl_deg=INCL), v_sys_kms=VSYS,
                        ln_nh2=np.full((NR, NZ), LN_N0, np.float32), temp_k=np.full((NR, NZ), T0, np.float32),
                        vphi_kms=np.zeros((NR, NZ), np.float32), z_lo_au=np.full(NR, -FAR, np.float32),
                        z_up_au=np.full(NR, FAR, np.float32), mask_width=1.0)
    return prob.replace(**fields)


def _dln():
    return math.log(GRID["r_max_au"] / GRID["r_min_au"]) / (NR - 1)


def _dzr():
    return GRID["zr_max"] / (NZ - 1)


def _point(u, v, phi=PHI, sign=1.0):
    """Position of index-space point (u, v) at azimuth phi: r = r_min e^(u dln),
    |z| = v dzr r."""
    rho = GRID["r_min_au"] * math.exp(u * _dln())
    return rho * math.cos(phi), rho * math.sin(phi), sign * v * _dzr() * rho


def _linear(a, b, c):
    i, j = np.meshgrid(np.arange(NR), np.arange(NZ), indexing="ij")
    return (a + b * i + c * j).astype(np.float32)


def _clamp(x, lo, hi):
    return min(max(x, lo), hi)


def _taper(u, v):
    return _clamp(u + 1.0, 0.0, 1.0) * _clamp(NR - u, 0.0, 1.0) * _clamp(NZ - v, 0.0, 1.0)


def _nfac(prob, t=T0):
    """n_u / (n_H2 mask): LTE fraction of CO in the upper level, typed here."""
    line = prob.line
    z = float(np.sum(line.lev_g * np.exp(-line.lev_e_k / t)))
    return prob.x_co * line.g_u * math.exp(-line.e_u_k / t) / z


def _temperature_from_width(prob, alpha_kms):
    line = prob.line
    per_k = 2 * KB / (line.m_co_amu * AMU) + prob.v_turb ** 2 * 2 * KB / (line.m_mol_amu * AMU)
    return (alpha_kms * 1e5) ** 2 / per_k


def test_linear_log_density_is_exact():
    a, b, c = 10.0, 0.25, -0.375
    prob = _base(ln_nh2=_linear(a, b, c))
    nfac = _nfac(prob)
    for u, v in INTERIOR + CLAMPED:
        uc, vc = _clamp(u, 0.0, NR - 1), _clamp(v, 0.0, NZ - 1)
        for sign in (1.0, -1.0):
            got = oracle.sample_point(prob, *_point(u, v, sign=sign))["n_u"] / nfac
            expect = math.exp(a + b * uc + c * vc) * _taper(u, v)
            assert got == pytest.approx(expect, rel=1e-12), (u, v, sign)


def test_linear_temperature_is_exact():
    a, b, c = 30.0, 2.0, 1.5
    prob = _base(temp_k=_linear(a, b, c))
    for u, v in INTERIOR + CLAMPED:
        uc, vc = _clamp(u, 0.0, NR - 1), _clamp(v, 0.0, NZ - 1)
        got = _temperature_from_width(prob, oracle.sample_point(prob, *_point(u, v))["alpha"])
        assert got == pytest.approx(a + b * uc + c * vc, rel=1e-12), (u, v)


def test_linear_rotation_velocity_is_exact():
    a, b, c = 1.0, 0.5, 0.25
    prob = _base(vphi_kms=_linear(a, b, c))
    proj = math.sin(math.radians(INCL)) * math.cos(PHI)
    for u, v in INTERIOR + CLAMPED:
        uc, vc = _clamp(u, 0.0, NR - 1), _clamp(v, 0.0, NZ - 1)
        got = (oracle.sample_point(prob, *_point(u, v))["vlos"] - VSYS) / proj
        assert got == pytest.approx(a + b * uc + c * vc, rel=1e-12), (u, v)


def test_taper_halves_density_half_a_cell_out():
    prob = _base()
    nfac = _nfac(prob)
    n0 = math.exp(float(np.float32(LN_N0)))
    n_at = lambda u, v: oracle.sample_point(prob, *_point(u, v))["n_u"] / nfac
    for u, v in [(NR - 0.5, 3.0), (-0.5, 3.0), (5.0, NZ - 0.5)]:
        assert n_at(u, v) == pytest.approx(0.5 * n0, rel=1e-12), (u, v)
    for u, v in [(NR - 1.0, 3.0), (0.0, 3.0), (5.0, NZ - 1.0)]:
        assert n_at(u, v) == pytest.approx(n0, rel=1e-12), (u, v)
    for u, v in [(NR, 3.0), (-1.0, 3.0), (5.0, NZ), (NR + 0.3, 3.0), (-1.6, 3.0), (5.0, NZ + 0.5)]:
        assert n_at(u, v) == 0.0, (u, v)


def _mask_at(prob, u, a_au):
    """The CO mask at index u and height |z| = a_au, from the upper-level density."""
    nfac = _nfac(prob)
    rho = GRID["r_min_au"] * math.exp(u * _dln())
    v = a_au / (rho * _dzr())
    n = math.exp(float(np.float32(LN_N0))) * _taper(u, v)
    x, y, _ = _point(u, 0.0)
    return oracle.sample_point(prob, x, y, a_au)["n_u"] / (nfac * n)


def _logit(m):
    return math.log(m / (1.0 - m))


@pytest.mark.parametrize("width", [1.0, 2.5])
def test_mask_width_and_lower_surface(width):
    """With the upper surface far away, logit(mask) = (|z| - z_lo(u)) / w:
    slope 1/w with w = width rho dzr, zero at z_lo, z_lo linear in u."""
    zl = (0.5 + 0.75 * np.arange(NR)).astype(np.float32)
    prob = _base(z_lo_au=zl, mask_width=width)
    for u in [3.25, 0.4, 6.7, 10.45, 11.3]:
        uc = _clamp(u, 0.0, NR - 1)
        rho = GRID["r_min_au"] * math.exp(u * _dln())
        w = width * rho * _dzr()
        z_lo = 0.5 + 0.75 * uc
        a1, a2 = z_lo + 0.1 * w, z_lo + 0.9 * w
        l1, l2 = _logit(_mask_at(prob, u, a1)), _logit(_mask_at(prob, u, a2))
        assert (a2 - a1) / (l2 - l1) == pytest.approx(w, rel=1e-9), u
        assert a1 - l1 * w == pytest.approx(z_lo, rel=1e-9), u


def test_mask_upper_surface_logistic():
    """With the lower surface far below: the mask is exactly the logistic
    1/(1 + e^((|z| - z_up)/w)); at z_up + w it is 1/(1+e), at z_up - w
    e/(1+e), and z_up is linear in u."""
    zu = (1.0 + 0.625 * np.arange(NR)).astype(np.float32)
    prob = _base(z_up_au=zu)
    for u in [2.75, 5.1, 6.2]:
        rho = GRID["r_min_au"] * math.exp(u * _dln())
        w = rho * _dzr()
        z_up = 1.0 + 0.625 * u
        assert _mask_at(prob, u, z_up + w) == pytest.approx(1.0 / (1.0 + math.e), rel=1e-9), u
        assert _mask_at(prob, u, z_up - w) == pytest.approx(math.e / (1.0 + math.e), rel=1e-9), u
        assert _mask_at(prob, u, z_up) == pytest.approx(0.5, rel=1e-9), u
        for frac in (-1.7, -0.3, 0.6, 2.2):
            expect = 1.0 / (1.0 + math.exp(frac))
            assert _mask_at(prob, u, z_up + frac * w) == pytest.approx(expect, rel=1e-9), (u, frac)


def test_mask_is_product_of_both_surfaces():
    """Both surfaces near: the mask is the product of the two logistics."""
    zl = np.full(NR, 2.0, np.float32)
    zu = np.full(NR, 3.5, np.float32)
    prob = _base(z_lo_au=zl, z_up_au=zu)
    u = 4.0
    rho = GRID["r_min_au"] * math.exp(u * _dln())
    w = rho * _dzr()
    for a in (1.6, 2.0, 2.8, 3.5, 4.1):
        expect = 1.0 / (1.0 + math.exp((a - 3.5) / w)) / (1.0 + math.exp((2.0 - a) / w))
        assert _mask_at(prob, u, a) == pytest.approx(expect, rel=1e-12), a
