"""Pins of the FP64 oracle against what the physics and mathematics fix.

Each test compares the oracle with something that does not come from the
oracle's own formulas: textbook closed forms typed here independently, exact
symmetries, brute-force re-evaluation, or convergence to the continuous
transfer integral.
"""
import math

import numpy as np
import pytest

import oracle
import synth

# CODATA 2018 cgs, typed here on their own
H = 6.62607015e-27
KB = 1.380649e-16
CL = 2.99792458e10
AMU = 1.66053906660e-24
AU = 1.495978707e13


def planck(nu, t):
    return 2 * H * nu ** 3 / CL ** 2 / math.expm1(H * nu / (KB * t))


def boltzmann_z(line, t):
    return float(np.sum(line.lev_g * np.exp(-line.lev_e_k / t)))


def doppler_width_kms(line, t, vturb):
    return math.sqrt(2 * KB * t / (line.m_co_amu * AMU) + vturb ** 2 * 2 * KB * t / (line.m_mol_amu * AMU)) / 1e5


def line_opacity(prob, t, n_h2, v_kms, vlos=0.0):
    """Textbook LTE line absorption coefficient [cm^-1] at channel velocity:
    (c^2 / 8 pi nu^2) (g_u/g_l) A_ul n_l (1 - exp(-h nu/kT)) phi_nu."""
    line = prob.line
    nco = prob.x_co * n_h2
    n_l = nco * line.g_l * math.exp(-line.e_l_k / t) / boltzmann_z(line, t)
    alpha = doppler_width_kms(line, t, prob.v_turb)
    phi = (CL / line.nu0_hz) / (alpha * 1e5 * math.sqrt(math.pi)) * np.exp(-((np.asarray(v_kms) - vlos) / alpha) ** 2)
    stim = -math.expm1(-H * line.nu0_hz / (KB * t))
    return CL ** 2 / (8 * math.pi * line.nu0_hz ** 2) * line.g_u / line.g_l * line.a_ul * n_l * stim * phi


def pixel_radius(prob, p, q):
    cam = prob.camera
    d = cam.fov_au / cam.nx
    return math.hypot((p + 0.5 - cam.nx / 2) * d, (q + 0.5 - cam.ny / 2) * d)


def slab_pixels(prob, h):
    g = prob.grid
    out = []
    for q in range(prob.camera.ny):
        for p in range(prob.camera.nx):
            r = pixel_radius(prob, p, q)
            if h / g.zr_max * 1.001 <= r <= g.r_max_au * 0.999:
                out.append((p, q))
    assert out
    return out


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("temp,ln_n", [(40.0, math.log(1e6)), (15.0, math.log(3e4)), (250.0, math.log(2e7))])
def test_isothermal_slab(temp, ln_n):
    """Face-on uniform isothermal slab of thickness 2H: I = B_nu(T) (1 - e^-tau),
    tau = kappa(v) 2H, for every channel and every pixel inside the grid."""
    prob = synth.slab_problem(temp=temp, ln_n=ln_n)
    g = prob.grid
    rc = g.outer_radius()
    zc = g.outer_zr() * rc
    h = zc * (1 - 2 * 24 / prob.nsamp)
    cube = oracle.render(prob)
    n = math.exp(float(np.float32(ln_n)))
    kap = line_opacity(prob, float(np.float32(temp)), n, prob.v_kms)
    expect = planck(prob.line.nu0_hz, float(np.float32(temp))) * -np.expm1(-kap * 2 * h * AU)
    assert expect.max() > 0 and (kap * 2 * h * AU).max() > 0.1
    for p, q in slab_pixels(prob, h):
        np.testing.assert_allclose(cube[:, q, p], expect, rtol=1e-12, atol=0)


def test_optically_thin_limit():
    """X_CO -> 0: the velocity-integrated intensity equals
    (h nu0 / 4 pi) A_ul n_u L (no absorption), and it scales with column."""
    prob = synth.slab_problem(temp=40.0, nch=121, dv=0.015, x_co=1e-15)
    g = prob.grid
    rc = g.outer_radius()
    zc = g.outer_zr() * rc
    h = zc * (1 - 2 * 24 / prob.nsamp)
    t = 40.0
    line = prob.line
    alpha = doppler_width_kms(line, t, prob.v_turb)
    assert prob.v_kms.max() > 5.5 * alpha and prob.v_kms[1] - prob.v_kms[0] < alpha / 4
    n = math.exp(float(np.float32(prob.ln_nh2[0, 0])))
    n_u = prob.x_co * n * line.g_u * math.exp(-line.e_u_k / t) / boltzmann_z(line, t)
    expect = H * line.nu0_hz / (4 * math.pi) * line.a_ul * n_u * 2 * h * AU
    dnu = line.nu0_hz * (prob.v_kms[1] - prob.v_kms[0]) / 1e5 * 1e5 / CL
    cube = oracle.render(prob)
    prob2 = prob.replace(ln_nh2=(prob.ln_nh2 + np.float32(math.log(2.0))).astype(np.float32))
    cube2 = oracle.render(prob2)
    for p, q in slab_pixels(prob, h):
        tot = float(np.sum(cube[:, q, p]) * dnu)
        assert tot == pytest.approx(expect, rel=1e-9)
        ratio = float(np.sum(cube2[:, q, p]) / np.sum(cube[:, q, p]))
        n2 = math.exp(float(prob2.ln_nh2[0, 0]))
        assert ratio == pytest.approx(n2 / n, rel=1e-9)


def test_thin_ring_doppler_sign():
    """Optically thin narrow ring rotating counter-clockwise about +z: the
    intensity-weighted mean velocity of a pixel is v_phi sin(i) x' / r0
    (positive = receding for x' > 0)."""
    prob = synth.ring_problem(width=1.0, nr=512)
    cube = oracle.render(prob)
    cam = prob.camera
    r0 = prob.meta["r0"]
    si = math.sin(math.radians(cam.incl_deg))
    d = cam.fov_au / cam.nx
    tot = cube.sum(axis=0)
    mom1 = np.tensordot(prob.v_kms, cube, axes=(0, 0))
    checked = 0
    for q in range(cam.ny):
        for p in range(cam.nx):
            x = (p + 0.5 - cam.nx / 2) * d
            # the ray must cross the ring (closest approach |x'| well inside r0)
            if tot[q, p] < 1e-3 * tot.max() or abs(x) < 0.1 * r0 or abs(x) > r0 - 5.0:
                continue
            vbar = mom1[q, p] / tot[q, p]
            expect = 5.0 * si * x / r0
            assert vbar == pytest.approx(expect, rel=2e-3), (p, q)
            checked += 1
    assert checked >= 12


def test_partition_function_high_temperature():
    """Rigid rotor: Z(T) -> T/theta + 1/3 + theta/(15T) + 4 theta^2/(315 T^2)."""
    prob = synth.config1(nx=4, ny=4)
    theta = prob.line.e_l_k / 2.0
    for t in (150.0, 400.0, 1000.0):
        z = oracle.partition(prob, t)
        x = theta / t
        assert z == pytest.approx(1 / x + 1 / 3 + x / 15 + 4 * x * x / 315, rel=1e-7)


def test_source_function_is_planck():
    """LTE: j / beta equals the Planck function at nu0 at every sample."""
    for t in (12.0, 40.0, 300.0):
        prob = synth.slab_problem(temp=t)
        s = oracle.sample_point(prob, 300.0, 0.0, 10.0)
        assert s["kbar"] > 0
        assert s["S"] == pytest.approx(planck(prob.line.nu0_hz, float(np.float32(t))), rel=1e-13)


# ------------------------------------------------------------------ invariants
def test_velocity_mirror_symmetry_bitwise():
    """PA = 0, v_sys = 0, symmetric pixel and channel grids:
    I(x', y', v) = I(-x', y', -v) exactly, at any inclination and noise."""
    for incl in (30.0, 45.0, 70.0):
        prob = synth.config1(nx=24, ny=20, nch=9, nsamp=64, nr=48, nz=24, incl=incl)
        cube = oracle.render(prob)
        assert np.array_equal(cube, cube[::-1, :, ::-1])
        assert cube.max() > 0


def test_face_on_symmetries():
    """Face-on: v_los = v_sys, so I(v) = I(-v); with smooth (noise-free)
    fields the image also has the symmetries of the square pixel grid."""
    grid = synth.GridSpec(nr=48, nz=24)
    prob = synth.make_problem(grid, synth.DiskParams(noise_sigma=0.0), 3, nx=16, ny=16, nch=7, dv=0.2,
                              nsamp=64, incl=0.0)
    cube = oracle.render(prob)
    np.testing.assert_array_equal(cube, cube[::-1])
    pk = cube.max()
    np.testing.assert_allclose(cube, cube[:, ::-1, :], atol=1e-12 * pk)
    np.testing.assert_allclose(cube, cube[:, :, ::-1], atol=1e-12 * pk)
    np.testing.assert_allclose(cube, np.transpose(cube, (0, 2, 1)), atol=1e-12 * pk)


def test_bounds_and_zero_density():
    prob = synth.small_problem(nx=10, ny=10, nch=6, nsamp=40)
    for q in range(0, 10, 3):
        for p in range(0, 10, 3):
            I, S, dt, _ = oracle.ray_dump(prob, p, q)
            tau = dt.sum(axis=0)
            assert np.all(I >= 0)
            assert np.all(I <= -np.expm1(-tau) * S.max() * (1 + 1e-14) + 1e-300)
    empty = prob.replace(ln_nh2=np.full_like(prob.ln_nh2, -1000.0))
    assert np.all(oracle.render(empty) == 0.0)


def test_recurrence_equals_nested_sum():
    """The O(N) front-to-back recurrence equals the O(N^2) explicit sum
    sum_k S_k (1 - e^-dtau_k) exp(-sum_{j<k} dtau_j)."""
    prob = synth.small_problem(nx=8, ny=8, nch=5, nsamp=60)
    checked = 0
    for (p, q) in [(3, 4), (4, 4), (2, 6), (5, 2)]:
        I, S, dt, _ = oracle.ray_dump(prob, p, q)
        ref = np.zeros_like(I)
        for k in range(len(S)):
            front = np.zeros(dt.shape[1])
            for j in range(k):
                front = front + dt[j]
            ref += np.exp(-front) * S[k] * -np.expm1(-dt[k])
        np.testing.assert_allclose(I, ref * prob.intensity_scale, rtol=1e-12, atol=1e-14 * max(I.max(), 1e-300))
        checked += I.max() > 0
    assert checked >= 2


@pytest.mark.slow
def test_converges_to_continuous_integral():
    """Tiny grid: the discrete march converges to an adaptive ODE solution of
    dtau/ds = beta, dI/ds = j e^-tau along the same continuous fields, at
    second order in the segment length."""
    from scipy.integrate import solve_ivp

    grid = synth.GridSpec(nr=8, nz=4)
    prob = synth.make_problem(grid, synth.DiskParams(), 11, nx=4, ny=4, nch=3, dv=1.2, nsamp=128,
                              incl=50.0)
    prob = prob.replace(x_co=1e-5, intensity_scale=synth.disk.rj_kelvin_scale(synth.co21_line()))
    pts = oracle.PointSampler(prob)
    cam = prob.camera
    ang = math.radians(cam.incl_deg)
    si, ci = math.sin(ang), math.cos(ang)
    d = cam.fov_au / cam.nx
    line = prob.line
    refs = {}
    for (p, q) in [(0, 1), (0, 2), (3, 1)]:
        _, _, _, ch = oracle.ray_dump(prob, p, q)
        sa, sb = ch[0], ch[1]
        x = (p + 0.5 - cam.nx / 2) * d
        y = (q + 0.5 - cam.ny / 2) * d

        def rhs(s, st):
            smp = pts(x, y * ci + s * si, y * si - s * ci)
            if smp["alpha"] <= 0:
                return np.zeros(6)
            phi = (CL / line.nu0_hz) / (smp["alpha"] * 1e5 * math.sqrt(math.pi)) * \
                np.exp(-((smp["vlos"] - prob.v_kms) / smp["alpha"]) ** 2)
            beta = smp["kbar"] * phi * AU
            return np.concatenate([beta, smp["S"] * beta * np.exp(-st[:3]) * prob.intensity_scale])

        sol = solve_ivp(rhs, (sa, sb), np.zeros(6), method="DOP853", rtol=1e-12, atol=1e-14,
                        max_step=(sb - sa) / 1000)
        refs[(p, q)] = sol.y[3:, -1]
    errs = []
    ns_list = [2 ** k for k in range(7, 14)]
    for ns in ns_list:
        cube = oracle.render(prob.replace(nsamp=ns))
        errs.append(max(np.abs(cube[:, q, p] - refs[(p, q)]).max() for (p, q) in refs))
    peak = max(np.abs(r).max() for r in refs.values())
    assert peak > 1.0
    assert errs[-1] < 1e-6 * peak
    # bilinear fields have kinks, so the error constant jumps about with where
    # the kinks fall; the least-squares slope over the sweep is the order
    slope = -np.polyfit(np.log2(ns_list), np.log2(errs), 1)[0]
    assert 1.6 < slope < 2.6, (slope, errs)
