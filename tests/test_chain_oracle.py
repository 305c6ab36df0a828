"""Pins of the derived-field oracle (oracle/chain.py) to closed forms.

Each test fixes one step of the chain to a result the mathematics gives
independently of the oracle's code: an exact solution of the hydrostatic
equation, exact column integrals, exact crossings, exact velocities, and
central finite differences of the oracle's own forward for its gradient.
"""
import math

import numpy as np
import pytest
import torch

from oracle import chain as C

MU = 2.37


def _ell(T, r, zr, mstar):
    """ln n - ln n(midplane) per node."""
    sig = np.ones(len(r))
    ln_n = C.hydrostatic_ln_n(torch.as_tensor(T, dtype=torch.float64), r, zr, mstar, MU, sig)
    return (ln_n - ln_n[:, :1]).numpy()


def test_isothermal_column_converges_to_the_spherical_potential_solution():
    """Constant T: ln rho(z) - ln rho(0) = -(G M m_mol / k_B T)(1/r - 1/sqrt(r^2 + z^2)),
    reached at second order in the node spacing."""
    r = np.array([40.0, 120.0])
    T0, M = 25.0, 2.0
    errs = []
    for nz in (129, 257, 513):
        zr = 0.5 * np.arange(nz) / (nz - 1)
        ell = _ell(np.full((2, nz), T0), r, zr, M)
        rr = r[:, None] * C.AU
        zz = rr * zr[None, :]
        exact = -(C.G * M * C.MSUN * MU * C.MH / (C.KB * T0)) * (1.0 / rr - 1.0 / np.sqrt(rr ** 2 + zz ** 2))
        errs.append(np.abs(ell - exact).max() / np.abs(exact).max())
    assert errs[-1] < 2e-6
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_without_gravity_pressure_is_constant_up_each_column():
    """M* = 0 leaves only the log-T term: rho T is the same at every height."""
    rng = np.random.default_rng(3)
    T = rng.uniform(10.0, 200.0, size=(3, 17))
    r = np.array([10.0, 50.0, 300.0])
    zr = np.linspace(0.0, 0.4, 17)
    ell = _ell(T, r, zr, 0.0)
    np.testing.assert_allclose(ell + np.log(T) - np.log(T[:, :1]), 0.0, atol=1e-12)


def test_surface_density_normalisation_holds_the_disk_mass():
    """2 pi int r Sigma(r) dr = M_gas for the tapered power law."""
    for gamma in (0.5, 1.0, 1.5):
        r = np.exp(np.linspace(np.log(1e-14), np.log(2e4), 400001))
        sig = C.surface_density(r, 0.09, 150.0, gamma)
        f = 2.0 * np.pi * r * C.AU * sig
        mass = np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(r) * C.AU)
        assert mass == pytest.approx(0.09 * C.MSUN, rel=1e-5), gamma


def test_normalised_density_integrates_to_sigma():
    """2 x the trapezoid integral of rho = n m_mol over each column is Sigma(r)."""
    nr, nz = 4, 33
    r, zr = C.nodes(nr, nz, 5.0, 400.0, 0.45)
    rng = np.random.default_rng(5)
    T = torch.as_tensor(rng.uniform(15.0, 90.0, size=(nr, nz)))
    sig = C.surface_density(r, 0.05, 120.0, 1.0)
    ln_n = C.hydrostatic_ln_n(T, r, zr, 1.5, MU, sig).numpy()
    rho = np.exp(ln_n) * MU * C.MH
    z = r[:, None] * zr[None, :] * C.AU
    integral = 2.0 * np.sum(0.5 * (rho[:, 1:] + rho[:, :-1]) * np.diff(z, axis=1), axis=1)
    np.testing.assert_allclose(integral, sig, rtol=1e-12)


def test_column_of_constant_and_exponential_density():
    r = np.array([30.0, 90.0])
    zr = np.linspace(0.0, 0.5, 41)
    z = r[:, None] * zr[None, :] * C.AU
    n = torch.full((2, 41), 1e6, dtype=torch.float64)
    np.testing.assert_allclose(C.column(n, r, zr).numpy(), 1e6 * (z[:, -1:] - z), rtol=1e-12, atol=1e-3)
    # exponential atmosphere: second-order convergence to n0 h (e^-z/h - e^-ztop/h)
    errs = []
    for m in (65, 129, 257):
        zr = np.linspace(0.0, 0.5, m)
        z = r[:, None] * zr[None, :] * C.AU
        h = 0.05 * r[:, None] * C.AU
        n = torch.as_tensor(1e8 * np.exp(-z / h))
        exact = 1e8 * h * (np.exp(-z / h) - np.exp(-z[:, -1:] / h))
        got = C.column(n, r, zr).numpy()
        errs.append(np.abs(got - exact)[:, :-1].max() / exact.max())
    assert errs[-1] < 3e-4
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_photodissociation_surface_of_an_exponential_column():
    """N = N0 e^-z/h is log-linear, so the crossing of 0.706 N = N_d is exact."""
    r = np.array([50.0, 200.0])
    zr = np.linspace(0.0, 0.5, 21)
    z_au = r[:, None] * zr[None, :]
    h_au = np.array([[2.0], [15.0]])
    N0 = np.array([[1e25], [3e23]])
    N = torch.as_tensor(N0 * np.exp(-z_au / h_au))
    nd = 1e21
    T = torch.full((2, 21), 50.0, dtype=torch.float64)
    _, z_up = C.co_surfaces(N, T, r, zr, 0.5, 20.0, nd)
    exact = h_au[:, 0] * np.log(N0[:, 0] * C.PHOTO_FACTOR / nd)
    np.testing.assert_allclose(z_up.numpy(), exact, rtol=1e-12)
    # still above the threshold at the top node: the layer reaches the top
    _, z_top = C.co_surfaces(N * 1e6, T, r, zr, 0.5, 20.0, nd)
    np.testing.assert_allclose(z_top.numpy(), z_au[:, -1], rtol=1e-12)


def test_freezeout_surface_and_the_no_layer_cases():
    r = np.array([20.0, 60.0, 100.0, 150.0])
    zr = np.linspace(0.0, 0.5, 11)
    z_au = r[:, None] * zr[None, :]
    T = np.empty((4, 11))
    T[0] = 10.0 + 1.6 * z_au[0]          # linear: crosses 20 K at z = 6.25 au (top 10 au)
    T[1] = 25.0                          # warm midplane
    T[2] = 12.0                          # never warm
    T[3] = 15.0 + 0.2 * z_au[3]          # crosses at z = 25 au
    N = torch.full((4, 11), 1e30, dtype=torch.float64)
    N[:, -1] = 0.0
    z_lo, z_up = C.co_surfaces(N, torch.as_tensor(T), r, zr, 0.5, 20.0, 1e21)
    np.testing.assert_allclose(z_lo.numpy(), [6.25, -0.5 * 60.0, 2 * 0.5 * 100.0, 25.0], rtol=1e-12)
    # a column shielded up to the node below the top crosses on the linear top segment
    thr = 1e21 / C.PHOTO_FACTOR
    np.testing.assert_allclose(z_up.numpy(), z_au[:, -2] + (thr - 1e30) / (0.0 - 1e30) * (z_au[:, -1] - z_au[:, -2]),
                               rtol=1e-12)
    # a column below the threshold even at the midplane has no layer
    _, z_up2 = C.co_surfaces(torch.full((4, 11), 1e20, dtype=torch.float64), torch.as_tensor(T), r, zr, 0.5, 20.0, 1e21)
    np.testing.assert_allclose(z_up2.numpy(), -0.5 * r, rtol=1e-12)


def test_vphi_keplerian_and_power_law_pressure():
    """Uniform pressure: the height-dependent Keplerian speed.  P ~ r^-p at
    fixed z/r: v^2 = v_K^2 - p k_B T / m_mol (central differences of a linear
    function of ln r are exact, one-sided ones too)."""
    nr, nz = 9, 7
    r, zr = C.nodes(nr, nz, 10.0, 300.0, 0.4)
    rr = r[:, None] * C.AU
    zz = rr * zr[None, :]
    vk2 = C.G * 1.7 * C.MSUN * rr ** 2 / (rr ** 2 + zz ** 2) ** 1.5
    T = torch.full((nr, nz), 40.0, dtype=torch.float64)
    flat = C.vphi_kms(torch.full((nr, nz), 20.0, dtype=torch.float64), T, r, zr, 1.7, MU).numpy()
    np.testing.assert_allclose(flat, np.sqrt(vk2) / 1e5, rtol=1e-12)
    p = 2.25
    ln_n = torch.as_tensor(20.0 - p * np.log(r)[:, None] * np.ones((1, nz)))
    got = C.vphi_kms(ln_n, T, r, zr, 1.7, MU).numpy()
    exact = np.sqrt(vk2 - p * C.KB * 40.0 / (MU * C.MH)) / 1e5
    np.testing.assert_allclose(got, exact, rtol=1e-12)


def test_chain_gradient_matches_central_differences():
    """Autograd through the whole chain against central differences of the
    FP64 forward (steps small enough to keep every crossing node)."""
    import synth
    nr, nz = 7, 16
    grid = (nr, nz, 8.0, 400.0, 0.5)
    r, zr = C.nodes(*grid)
    R, ZR = np.meshgrid(r, zr, indexing="ij")
    T0, _ = synth.disk._temperature(R, ZR * R, synth.disk.DiskParams())
    args = dict(mstar_msun=2.0, mgas_msun=0.09, rc_au=150.0, gamma=1.0, mu=MU, t_freeze_k=20.0, n_dissoc=1e21)
    rng = np.random.default_rng(11)
    cot = {k: torch.as_tensor(rng.standard_normal(s)) for k, s in
           (("ln_nh2", (nr, nz)), ("vphi_kms", (nr, nz)), ("z_lo_au", (nr,)), ("z_up_au", (nr,)))}

    def loss(Tv):
        out = C.derive_fields(Tv, grid, **args)
        return sum((out[k] * cot[k]).sum() for k in cot)

    T = torch.as_tensor(T0).clone().requires_grad_(True)
    loss(T).backward()
    g = T.grad.numpy()
    for (i, j) in [(0, 0), (1, 5), (3, 3), (4, 10), (6, 15), (2, 8), (5, 1)]:
        h = 1e-5 * T0[i, j]
        tp, tm = T0.copy(), T0.copy()
        tp[i, j] += h
        tm[i, j] -= h
        with torch.no_grad():
            fd = (loss(torch.as_tensor(tp)) - loss(torch.as_tensor(tm))).item() / (2 * h)
        assert g[i, j] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g).max()), (i, j)


def test_parametric_temperature_special_heights():
    """Midplane: T_mid; at and above z_q: T_atm; delta = 1 at z_q / 2:
    cos^2(pi/4) = 1/2, the mean of the two layers."""
    nr, nz = 5, 401
    args = dict(t_mid0_k=30.0, t_atm0_k=70.0, q=-0.5, r_scale_au=100.0, zq0_au=12.0, delta=1.0)
    T = C.parametric_temperature(nr, nz, 10.0, 400.0, 0.5, **args)
    r, zr = C.nodes(nr, nz, 10.0, 400.0, 0.5)
    x = r / 100.0
    np.testing.assert_allclose(T[:, 0], 30.0 * x ** -0.5, rtol=1e-14)
    zq = 12.0 * x ** 1.3
    z = r[:, None] * zr[None, :]
    above = z >= zq[:, None]
    np.testing.assert_allclose(T[above], (70.0 * x[:, None] ** -0.5 * np.ones((1, nz)))[above], rtol=1e-14)
    # r = 100 au: x = 1, z_q = 12 au; the node at z = 6 au is z/r = 0.06 -> j = 0.06 / 0.5 * 400 = 48
    T1 = C.parametric_temperature(2, 401, 100.0, 400.0, 0.5, **args)
    assert T1[0, 48] == pytest.approx(50.0, rel=1e-12)
