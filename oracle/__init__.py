"""FP64 CPU oracle of the line radiative-transfer ray march.

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.

Two implementations of the same discrete quantity live here:

* ``librt_oracle.so`` (``rt_oracle.c``): plain scalar FP64 loops, OpenMP over
  pixel rows -- the forward reference and the CPU baseline;
* ``torch_ref``: the same definition written with float64 torch tensor ops,
  vectorised over pixels and channels, whose autograd gives the exact
  gradient of the discrete forward (the gradient reference).

Both take a problem object with the attributes of ``synth.Problem`` (duck
typed; nothing from ``synth`` is imported).  ``render3`` and its siblings are
the C oracle's 3-D path: fields on a spherical (ln r, theta, phi) grid with all
three velocity components and an abundance field, attributes as in
``synth.disk3d.Problem3``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librt_oracle.so")

_f = C.POINTER(C.c_float)
_d = C.POINTER(C.c_double)


class OrcProblem(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32),
        ("r_min_au", C.c_double), ("r_max_au", C.c_double), ("zr_max", C.c_double),
        ("ln_nh2", _f), ("temp_k", _f), ("vphi_kms", _f), ("z_lo_au", _f), ("z_up_au", _f),
        ("x_co", C.c_double), ("mask_width", C.c_double), ("v_turb", C.c_double),
        ("nu0_hz", C.c_double), ("a_ul", C.c_double), ("g_u", C.c_double), ("g_l", C.c_double),
        ("e_u_k", C.c_double), ("e_l_k", C.c_double), ("m_co_amu", C.c_double), ("m_mol_amu", C.c_double),
        ("nlev", C.c_int32), ("lev_e_k", _d), ("lev_g", _d),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("fov_au", C.c_double), ("incl_deg", C.c_double), ("pa_deg", C.c_double),
        ("nch", C.c_int32), ("v_kms", _d), ("v_sys_kms", C.c_double),
        ("nsamp", C.c_int32), ("intensity_scale", C.c_double),
        ("mlp_w", _f),
    ]


_lib = None


def load(path: str):
    """Open a build of rt_oracle.c and declare the argument types of its 2-D
    entry points."""
    L = C.CDLL(path)
    P = C.POINTER(OrcProblem)
    L.orc_render.argtypes = [P, _d, C.c_int]
    L.orc_render_pixels.argtypes = [P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _d, C.c_int]
    L.orc_ray_dump.argtypes = [P, C.c_int, C.c_int, _d, _d, _d, _d]
    L.orc_sample_point.argtypes = [P, C.c_double, C.c_double, C.c_double, _d]
    L.orc_partition.argtypes = [P, C.c_double]
    L.orc_partition.restype = C.c_double
    L.orc_constants.argtypes = [_d, C.c_int]
    L.orc_mlp.argtypes = [_f, C.c_double, C.c_double, _d]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = load(LIB_PATH)
    return _lib


class _Packed:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, prob, **over):
        g = prob.grid
        line = prob.line
        self.arrs = {}

        def fp(name, a):
            a = np.ascontiguousarray(a, dtype=np.float32)
            self.arrs[name] = a
            return a.ctypes.data_as(_f)

        def dp(name, a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self.arrs[name] = a
            return a.ctypes.data_as(_d)

        cam = prob.camera
        vals = dict(
            nr=g.nr, nz=g.nz, r_min_au=g.r_min_au, r_max_au=g.r_max_au, zr_max=g.zr_max,
            x_co=prob.x_co, mask_width=prob.mask_width, v_turb=prob.v_turb,
            nu0_hz=line.nu0_hz, a_ul=line.a_ul, g_u=line.g_u, g_l=line.g_l, e_u_k=line.e_u_k,
            e_l_k=line.e_l_k, m_co_amu=line.m_co_amu, m_mol_amu=line.m_mol_amu,
            nlev=len(line.lev_e_k), nx=cam.nx, ny=cam.ny, fov_au=cam.fov_au,
            incl_deg=cam.incl_deg, pa_deg=cam.pa_deg, nch=len(prob.v_kms),
            v_sys_kms=prob.v_sys_kms, nsamp=prob.nsamp, intensity_scale=prob.intensity_scale)
        vals.update(over)
        s = OrcProblem()
        for k, v in vals.items():
            setattr(s, k, v)
        s.ln_nh2 = fp("ln", prob.ln_nh2)
        s.temp_k = fp("t", prob.temp_k)
        s.vphi_kms = fp("v", prob.vphi_kms)
        s.z_lo_au = fp("zlo", prob.z_lo_au)
        s.z_up_au = fp("zup", prob.z_up_au)
        s.lev_e_k = dp("le", line.lev_e_k)
        s.lev_g = dp("lg", line.lev_g)
        s.v_kms = dp("vk", prob.v_kms)
        s.mlp_w = fp("mlp", prob.mlp_w) if getattr(prob, "mlp_w", None) is not None else _f()
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def render(prob, nthreads: int = 0) -> np.ndarray:
    """FP64 cube [nch][ny][nx] of the whole image."""
    pk = _Packed(prob)
    out = np.zeros((len(prob.v_kms), prob.camera.ny, prob.camera.nx), np.float64)
    rc = lib().orc_render(pk.ref, out.ctypes.data_as(_d), nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return out


def render_pixels(prob, px, py, nthreads: int = 0) -> np.ndarray:
    """FP64 spectra [n][nch] of pixels (px[n], py[n])."""
    pk = _Packed(prob)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    out = np.zeros((len(px), len(prob.v_kms)), np.float64)
    lib().orc_render_pixels(pk.ref, len(px), px.ctypes.data_as(C.POINTER(C.c_int32)),
                            py.ctypes.data_as(C.POINTER(C.c_int32)), out.ctypes.data_as(_d), nthreads)
    return out


def ray_dump(prob, p: int, q: int):
    """(I[c], S[k], dtau[k][c], (s_a, s_b, ds)) of one ray."""
    pk = _Packed(prob)
    nch, ns = len(prob.v_kms), prob.nsamp
    I = np.zeros(nch)
    S = np.zeros(ns)
    dt = np.zeros((ns, nch))
    ch = np.zeros(3)
    lib().orc_ray_dump(pk.ref, p, q, I.ctypes.data_as(_d), S.ctypes.data_as(_d), dt.ctypes.data_as(_d),
                       ch.ctypes.data_as(_d))
    return I, S, dt, ch


def sample_point(prob, px, py, pz):
    """{S, kbar, alpha [km/s], vlos [km/s], n_u} at one point."""
    pk = _Packed(prob)
    out = np.zeros(5)
    lib().orc_sample_point(pk.ref, px, py, pz, out.ctypes.data_as(_d))
    return dict(S=out[0], kbar=out[1], alpha=out[2], vlos=out[3], n_u=out[4])


def partition(prob, t: float) -> float:
    pk = _Packed(prob)
    return lib().orc_partition(pk.ref, t)


def constants() -> dict:
    out = np.zeros(6)
    lib().orc_constants(out.ctypes.data_as(_d), 6)
    return dict(zip(["h", "k_B", "c", "amu", "au", "pi"], out.tolist()))


def mlp(w, rh: float, zh: float) -> np.ndarray:
    w = np.ascontiguousarray(w, np.float32)
    out = np.zeros(3)
    lib().orc_mlp(w.ctypes.data_as(_f), rh, zh, out.ctypes.data_as(_d))
    return out


def loss(cube, target) -> float:
    """L = sum over voxels of (I - D)^2 (the L2 loss; chi^2 up to 1/sigma^2)."""
    d = np.asarray(cube, np.float64) - np.asarray(target, np.float64)
    return float(np.sum(d * d))


class PointSampler:
    """Repeated point evaluations of the shading of one problem (packs once)."""

    def __init__(self, prob):
        self.pk = _Packed(prob)
        self.out = np.zeros(5)
        self.L = lib()

    def __call__(self, px, py, pz):
        self.L.orc_sample_point(self.pk.ref, px, py, pz, self.out.ctypes.data_as(_d))
        o = self.out
        return dict(S=o[0], kbar=o[1], alpha=o[2], vlos=o[3], n_u=o[4])


# ------------------------------------------------------------ 3-D spherical grid

class OrcProblem3(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nt", C.c_int32), ("np", C.c_int32),
        ("r_min_au", C.c_double), ("r_max_au", C.c_double), ("th_min", C.c_double), ("th_max", C.c_double),
        ("ln_nh2", _f), ("temp_k", _f), ("v_r", _f), ("v_t", _f), ("v_p", _f), ("x_co", _f),
        ("v_turb", C.c_double),
        ("nu0_hz", C.c_double), ("a_ul", C.c_double), ("g_u", C.c_double), ("g_l", C.c_double),
        ("e_u_k", C.c_double), ("e_l_k", C.c_double), ("m_co_amu", C.c_double), ("m_mol_amu", C.c_double),
        ("nlev", C.c_int32), ("lev_e_k", _d), ("lev_g", _d),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("fov_au", C.c_double), ("incl_deg", C.c_double), ("pa_deg", C.c_double),
        ("nch", C.c_int32), ("v_kms", _d), ("v_sys_kms", C.c_double),
        ("nsamp", C.c_int32), ("intensity_scale", C.c_double),
    ]


class _Packed3:
    def __init__(self, prob):
        g, line, cam = prob.grid, prob.line, prob.camera
        self.arrs = {}

        def fp(name, a):
            a = np.ascontiguousarray(a, dtype=np.float32)
            self.arrs[name] = a
            return a.ctypes.data_as(_f)

        def dp(name, a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self.arrs[name] = a
            return a.ctypes.data_as(_d)

        s = OrcProblem3()
        for k, v in dict(nr=g.nr, nt=g.nt, np=g.nphi, r_min_au=g.r_min_au, r_max_au=g.r_max_au, th_min=g.th_min,
                         th_max=g.th_max, v_turb=prob.v_turb, nu0_hz=line.nu0_hz, a_ul=line.a_ul, g_u=line.g_u,
                         g_l=line.g_l, e_u_k=line.e_u_k, e_l_k=line.e_l_k, m_co_amu=line.m_co_amu,
                         m_mol_amu=line.m_mol_amu, nlev=len(line.lev_e_k), nx=cam.nx, ny=cam.ny,
                         fov_au=cam.fov_au, incl_deg=cam.incl_deg, pa_deg=cam.pa_deg, nch=len(prob.v_kms),
                         v_sys_kms=prob.v_sys_kms, nsamp=prob.nsamp, intensity_scale=prob.intensity_scale).items():
            setattr(s, k, v)
        s.ln_nh2 = fp("ln", prob.ln_nh2)
        s.temp_k = fp("t", prob.temp_k)
        s.v_r = fp("vr", prob.v_r_kms)
        s.v_t = fp("vt", prob.v_theta_kms)
        s.v_p = fp("vp", prob.v_phi_kms)
        s.x_co = fp("x", prob.x_co)
        s.lev_e_k = dp("le", line.lev_e_k)
        s.lev_g = dp("lg", line.lev_g)
        s.v_kms = dp("vk", prob.v_kms)
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def _lib3():
    L = lib()
    if not getattr(L, "_has3", False):
        P = C.POINTER(OrcProblem3)
        L.orc_render3.argtypes = [P, _d, C.c_int]
        L.orc_render3_pixels.argtypes = [P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _d, C.c_int]
        L.orc_ray_dump3.argtypes = [P, C.c_int, C.c_int, _d, _d, _d, _d]
        L.orc_sample_point3.argtypes = [P, C.c_double, C.c_double, C.c_double, _d]
        L._has3 = True
    return L


def render3(prob, nthreads: int = 0) -> np.ndarray:
    """FP64 cube [nch][ny][nx] of a 3-D spherical-grid problem."""
    pk = _Packed3(prob)
    out = np.zeros((len(prob.v_kms), prob.camera.ny, prob.camera.nx), np.float64)
    if _lib3().orc_render3(pk.ref, out.ctypes.data_as(_d), nthreads) != 0:
        raise ValueError("oracle rejected the problem")
    return out


def render3_pixels(prob, px, py, nthreads: int = 0) -> np.ndarray:
    pk = _Packed3(prob)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    out = np.zeros((len(px), len(prob.v_kms)), np.float64)
    _lib3().orc_render3_pixels(pk.ref, len(px), px.ctypes.data_as(C.POINTER(C.c_int32)),
                               py.ctypes.data_as(C.POINTER(C.c_int32)), out.ctypes.data_as(_d), nthreads)
    return out


def ray_dump3(prob, p: int, q: int):
    """(I[c], S[k], dtau[k][c], (s_a, s_b, ds)) of one ray of a 3-D problem."""
    pk = _Packed3(prob)
    nch, ns = len(prob.v_kms), prob.nsamp
    I, S, dt, ch = np.zeros(nch), np.zeros(ns), np.zeros((ns, nch)), np.zeros(3)
    _lib3().orc_ray_dump3(pk.ref, p, q, I.ctypes.data_as(_d), S.ctypes.data_as(_d), dt.ctypes.data_as(_d),
                          ch.ctypes.data_as(_d))
    return I, S, dt, ch


def sample_point3(prob, x, y, z) -> dict:
    """Line quantities at a disk-frame point (au) of a 3-D problem."""
    pk = _Packed3(prob)
    out = np.zeros(5)
    _lib3().orc_sample_point3(pk.ref, float(x), float(y), float(z), out.ctypes.data_as(_d))
    return dict(S=out[0], kbar=out[1], alpha=out[2], vlos=out[3], n_u=out[4])
