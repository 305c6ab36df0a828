"""Pins of the oracle's 3-D spherical-grid path (rt_oracle.c, orc_render3).

Checked against what does not come from its own formulas: a field linear in
the cell coordinates, which trilinear interpolation must return exactly; the
line-of-sight velocity against v . w with the spherical unit vectors built
here; the central ray's total optical depth against the closed-form length of
the tapered radial profile; an optically thick sphere against the Planck
function; and two exact symmetries of the rendered cube (a roll of the fields
in phi against a sky rotation, face-on; the mirror of an axisymmetric rotating
disk in x and velocity)."""
import math

import numpy as np
import pytest

import oracle
from synth import disk3d as S3
from test_oracle_pins import AU, boltzmann_z, line_opacity, planck


class _Scalar:
    """The attributes line_opacity reads, with a scalar x_CO."""

    def __init__(self, prob, x_co):
        self.line, self.v_turb, self.x_co = prob.line, prob.v_turb, x_co


def _point(g, u, w, s):
    dln = math.log(g.r_max_au / g.r_min_au) / (g.nr - 1)
    r = g.r_min_au * math.exp(u * dln)
    th = g.th_min + w * (g.th_max - g.th_min) / (g.nt - 1)
    ph = s * 2 * math.pi / g.nphi
    x = r * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    e_r = x / r
    e_t = np.array([math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)])
    e_p = np.array([-math.sin(ph), math.cos(ph), 0.0])
    return x, e_r, e_t, e_p


def _linear(g, a, b, c, d):
    i, j, k = np.meshgrid(np.arange(g.nr), np.arange(g.nt), np.arange(g.nphi), indexing="ij")
    return (a + b * i + c * j + d * k).astype(np.float32)


@pytest.mark.parametrize("incl", [90.0, 35.0])
def test_interpolation_and_velocity_projection(incl):
    g = S3.Grid3Spec(12, 9, 16, r_min_au=5.0, r_max_au=200.0)
    base = S3.uniform_problem3(g, incl=incl)
    w_dir = np.array([0.0, math.sin(math.radians(incl)), -math.cos(math.radians(incl))])
    lin = _linear(g, 0.5, 0.25, -0.375, 0.125)
    line = base.line
    t = float(base.temp_k[0, 0, 0])
    nfac = float(base.x_co[0, 0, 0]) * line.g_u * math.exp(-line.e_u_k / t) / boltzmann_z(line, t)
    for (u, w, s) in [(3.25, 2.5, 4.75), (0.125, 7.5, 13.0), (10.5, 0.75, 9.25)]:
        x, e_r, e_t, e_p = _point(g, u, w, s)
        expect = 0.5 + 0.25 * u - 0.375 * w + 0.125 * s
        for field, unit in (("v_r_kms", e_r), ("v_theta_kms", e_t), ("v_phi_kms", e_p)):
            got = oracle.sample_point3(base.replace(**{field: lin}), *x)
            assert got["vlos"] == pytest.approx(expect * float(unit @ w_dir), rel=1e-12, abs=1e-13), field
        got = oracle.sample_point3(base.replace(ln_nh2=lin), *x)
        assert math.log(got["n_u"] / nfac) == pytest.approx(expect, rel=1e-12)


def test_taper_and_periodic_phi():
    g = S3.Grid3Spec(12, 9, 16, r_min_au=5.0, r_max_au=200.0)
    base = S3.uniform_problem3(g)
    lin = _linear(g, 0.0, 0.0, 0.0, 0.5)          # ln n = k / 2
    line = base.line
    t = float(base.temp_k[0, 0, 0])
    nfac = float(base.x_co[0, 0, 0]) * line.g_u * math.exp(-line.e_u_k / t) / boltzmann_z(line, t)
    n_u = lambda u, w, s: oracle.sample_point3(base.replace(ln_nh2=lin), *_point(g, u, w, s)[0])["n_u"] / nfac
    # across the phi seam, halfway between k = nphi - 1 and k = 0 (ln n is interpolated)
    assert n_u(5.0, 4.0, 15.5) == pytest.approx(math.exp(0.5 * (7.5 + 0.0)), rel=1e-12)
    # half a cell beyond each edge: the edge value times 1/2; a full cell beyond: zero
    for u, w in [(11.5, 4.0), (-0.5, 4.0), (5.0, 8.5), (5.0, -0.5)]:
        assert n_u(u, w, 3.0) == pytest.approx(0.5 * math.exp(1.5), rel=1e-12), (u, w)
    for u, w in [(12.0, 4.0), (-1.0, 4.0), (5.0, 9.0), (5.0, -1.25)]:
        assert n_u(u, w, 3.0) == 0.0, (u, w)


def test_central_ray_optical_depth_closed_form():
    """Edge-on central ray through uniform fields at rest: the opacity is the
    textbook LTE value times the radial taper (linear in ln r over one cell at
    each end), so tau = kappa * 2 * [r_max (1 + (e^D - 1 - D)/D) - r_min (1 - e^-D)/D]."""
    g = S3.Grid3Spec(16, 9, 8, r_min_au=5.0, r_max_au=400.0)
    prob = S3.uniform_problem3(g, nx=9, ny=9, nch=5, dv=0.1, nsamp=40000)
    _, _, dtau, ch = oracle.ray_dump3(prob, 4, 4)
    D = math.log(g.r_max_au / g.r_min_au) / (g.nr - 1)
    assert ch[1] == pytest.approx(g.r_max_au * math.exp(D), rel=1e-14)
    length = g.r_max_au * (1 + (math.expm1(D) - D) / D) - g.r_min_au * (-math.expm1(-D)) / D
    t, n = float(np.float32(40.0)), math.exp(float(np.float32(math.log(1e6))))
    kap = line_opacity(_Scalar(prob, float(np.float32(1e-4))), t, n, prob.v_kms)
    np.testing.assert_allclose(dtau.sum(axis=0), kap * 2 * length * AU, rtol=2e-7)
    # inside the grid every sample carries kappa ds
    s = ch[0] + (np.arange(prob.nsamp) + 0.5) * ch[2]
    inside = (np.abs(s) > g.r_min_au * 1.01) & (np.abs(s) < g.r_max_au * 0.99)
    np.testing.assert_allclose(dtau[inside], np.broadcast_to(kap * ch[2] * AU, dtau[inside].shape), rtol=1e-12)


def test_optically_thick_sphere_is_planck():
    g = S3.Grid3Spec(10, 24, 8, r_min_au=2.0, r_max_au=100.0, th_min=0.2, th_max=math.pi - 0.2)
    prob = S3.uniform_problem3(g, temp=55.0, ln_n=math.log(1e9), nx=11, ny=11, nch=3, dv=0.05, nsamp=512)
    cube = oracle.render3(prob)
    B = planck(prob.line.nu0_hz, float(np.float32(55.0)))
    d = prob.camera.fov_au / prob.camera.nx
    for q in range(11):
        for p in range(11):
            if math.hypot((p - 5) * d, (q - 5) * d) < 0.6 * g.r_max_au:
                np.testing.assert_allclose(cube[:, q, p], B, rtol=1e-12)


def test_phi_roll_equals_sky_rotation_face_on():
    g = S3.Grid3Spec(20, 10, 16)
    prob = S3.make_problem3(g, seed=51, nx=14, ny=12, nch=5, dv=0.4, nsamp=96, incl=0.0, pa=10.0)
    rng = np.random.Generator(np.random.PCG64(52))
    prob = prob.replace(v_theta_kms=(0.3 * rng.standard_normal(prob.ln_nh2.shape)).astype(np.float32))
    m = 4
    roll = {k: np.roll(getattr(prob, k), m, axis=2)
            for k in ("ln_nh2", "temp_k", "v_r_kms", "v_theta_kms", "v_phi_kms", "x_co")}
    rolled = prob.replace(**roll)
    rolled.camera = S3.D.Camera(**{**prob.camera.__dict__, "pa_deg": 10.0 + 360.0 * m / g.nphi})
    a, b = oracle.render3(prob), oracle.render3(rolled)
    assert a.max() > 0
    np.testing.assert_allclose(b, a, rtol=1e-9, atol=1e-12 * a.max())


def test_axisymmetric_rotation_mirror():
    g = S3.Grid3Spec(20, 10, 12)
    prob = S3.make_problem3(g, seed=53, nx=14, ny=10, nch=7, dv=0.5, nsamp=96, incl=50.0, spiral=0.0,
                            inflow=0.0, noise=0.0)
    cube = oracle.render3(prob)
    assert cube.max() > 0
    np.testing.assert_allclose(cube[::-1, :, ::-1], cube, rtol=1e-11, atol=1e-13 * cube.max())
