"""Torch-facing calls of the renderer (device memory and streams only).

``Scene`` holds a problem with its fields resident on the GPU; ``render``
and ``render_adjoint`` marshal it into the C structs of include/rtcube.h and
call the library on torch's current stream.  ``Render`` is the
torch.autograd.Function whose backward is the library's adjoint.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
import torch

from . import _lib as L

@dataclass
class Scene:
    nr: int
    nz: int
    r_min_au: float
    r_max_au: float
    zr_max: float
    ln_nh2: torch.Tensor      # [nr, nz] float32, device
    temp_k: torch.Tensor
    vphi_kms: torch.Tensor
    z_lo_au: torch.Tensor     # [nr]
    z_up_au: torch.Tensor
    x_co: float
    mask_width: float
    v_turb: float
    nu0_hz: float
    a_ul: float
    g_u: float
    g_l: float
    e_u_k: float
    e_l_k: float
    m_co_amu: float
    m_mol_amu: float
    lev_e_k: np.ndarray
    lev_g: np.ndarray
    nx: int
    ny: int
    fov_au: float
    incl_deg: float
    pa_deg: float
    dist_pc: float
    v_kms: np.ndarray
    v_sys_kms: float
    nsamp: int
    intensity_scale: float = 1.0
    mlp_w: Optional[torch.Tensor] = None
    mlp_precision: int = L.RT_MLP_BF16
    keep: list = field(default_factory=list, repr=False)
    _struct: tuple = field(default=None, repr=False, compare=False)
    _live: Optional[dict] = field(default=None, repr=False, compare=False)

    @property
    def nch(self) -> int:
        return int(len(self.v_kms))

    def census(self, stream=None) -> dict:
        """The library's work accounting of this render (rt_render_census):
        the [ny, nx] bool mask of rays that cross the grid's bounding
        cylinder (the others have no samples: zero intensity, no work), their
        number, their pixel-samples, how many of those the march takes as
        optically thin, how many have any opacity and how many lie inside the
        grid's edge taper (the last three -1 with the network)."""
        if self._live is None:
            mask = torch.empty(self.ny, self.nx, dtype=torch.uint8, device=self.ln_nh2.device)
            counts = (C.c_int64 * 5)()
            p, keep = problem_struct(self)
            L.check(L.lib().rt_render_census(C.byref(p), mask.data_ptr(), counts, C.c_void_p(_stream(stream))))
            object.__setattr__(self, "_live", dict(mask=mask.cpu().numpy().astype(bool), rays=int(counts[0]),
                                                   pixel_samples=int(counts[1]), thin_pixel_samples=int(counts[2]),
                                                   emitting_pixel_samples=int(counts[3]),
                                                   shaded_pixel_samples=int(counts[4])))
        return self._live

    def live_mask(self) -> np.ndarray:
        """[ny, nx] bool: pixels whose ray crosses the grid's bounding volume."""
        return self.census()["mask"]

    @property
    def ray_samples(self) -> int:
        """(pixel, channel, sample) triples of the rays that cross the grid."""
        return self.census()["pixel_samples"] * self.nch

    def replace(self, **kw) -> "Scene":
        return replace(self, _struct=None, _live=None, **kw)


def scene_from_problem(prob, device="cuda", mlp_precision=L.RT_MLP_BF16) -> Scene:
    """Copy a problem description (attributes as in synth.Problem) to the GPU."""
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
    g, cam, line = prob.grid, prob.camera, prob.line
    mlp = getattr(prob, "mlp_w", None)
    return Scene(nr=g.nr, nz=g.nz, r_min_au=g.r_min_au, r_max_au=g.r_max_au, zr_max=g.zr_max,
                 ln_nh2=t(prob.ln_nh2), temp_k=t(prob.temp_k), vphi_kms=t(prob.vphi_kms),
                 z_lo_au=t(prob.z_lo_au), z_up_au=t(prob.z_up_au), x_co=prob.x_co,
                 mask_width=prob.mask_width, v_turb=prob.v_turb, nu0_hz=line.nu0_hz, a_ul=line.a_ul,
                 g_u=line.g_u, g_l=line.g_l, e_u_k=line.e_u_k, e_l_k=line.e_l_k,
                 m_co_amu=line.m_co_amu, m_mol_amu=line.m_mol_amu,
                 lev_e_k=np.ascontiguousarray(line.lev_e_k, np.float64),
                 lev_g=np.ascontiguousarray(line.lev_g, np.float64), nx=cam.nx, ny=cam.ny,
                 fov_au=cam.fov_au, incl_deg=cam.incl_deg, pa_deg=cam.pa_deg, dist_pc=cam.dist_pc,
                 v_kms=np.ascontiguousarray(prob.v_kms, np.float64), v_sys_kms=prob.v_sys_kms,
                 nsamp=prob.nsamp, intensity_scale=prob.intensity_scale,
                 mlp_w=None if mlp is None else t(mlp), mlp_precision=mlp_precision)


def _fptr(t: Optional[torch.Tensor]):
    """Device address of a contiguous float32 CUDA tensor (None for NULL)."""
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return t.data_ptr()


def problem_struct(sc: Scene, fields: Optional[dict] = None):
    """rt_problem for the scene (fields may override the scene's tensors).
    Returns (struct, keepalive); without overrides the struct is built once
    per scene and reused."""
    if fields is None and sc._struct is not None:
        return sc._struct
    built = _build_struct(sc, fields)
    if fields is None:
        sc._struct = built
    return built


def _build_struct(sc: Scene, fields: Optional[dict]):
    fl = dict(ln_nh2=sc.ln_nh2, temp_k=sc.temp_k, vphi_kms=sc.vphi_kms, z_lo_au=sc.z_lo_au,
              z_up_au=sc.z_up_au, mlp_w=sc.mlp_w)
    if fields:
        fl.update(fields)
    for k, n in (("ln_nh2", sc.nr * sc.nz), ("temp_k", sc.nr * sc.nz), ("vphi_kms", sc.nr * sc.nz),
                 ("z_lo_au", sc.nr), ("z_up_au", sc.nr)):
        if fl[k].numel() != n:
            raise ValueError(f"{k} has {fl[k].numel()} elements, expected {n}")
    lev_e = np.ascontiguousarray(sc.lev_e_k, np.float64)
    lev_g = np.ascontiguousarray(sc.lev_g, np.float64)
    vk = np.ascontiguousarray(sc.v_kms, np.float64)
    p = L.rt_problem()
    p.grid = L.rt_grid(sc.nr, sc.nz, sc.r_min_au, sc.r_max_au, sc.zr_max)
    p.f = L.rt_fields(_fptr(fl["ln_nh2"]), _fptr(fl["temp_k"]), _fptr(fl["vphi_kms"]), _fptr(fl["z_lo_au"]),
                      _fptr(fl["z_up_au"]), sc.x_co, sc.mask_width, sc.v_turb)
    p.line = L.rt_line(sc.nu0_hz, sc.a_ul, sc.g_u, sc.g_l, sc.e_u_k, sc.e_l_k, sc.m_co_amu, sc.m_mol_amu,
                       len(lev_e), lev_e.ctypes.data_as(C.POINTER(C.c_double)),
                       lev_g.ctypes.data_as(C.POINTER(C.c_double)))
    p.cam = L.rt_camera(sc.nx, sc.ny, sc.fov_au, sc.incl_deg, sc.pa_deg, sc.dist_pc)
    p.spec = L.rt_spectral(len(vk), vk.ctypes.data_as(C.POINTER(C.c_double)), sc.v_sys_kms)
    p.nsamp = sc.nsamp
    p.intensity_scale = sc.intensity_scale
    keep = [lev_e, lev_g, vk, fl]
    if fl["mlp_w"] is not None:
        if fl["mlp_w"].numel() != L.RT_MLP_PARAMS:
            raise ValueError("mlp_w has the wrong number of parameters")
        m = L.rt_mlp(_fptr(fl["mlp_w"]), sc.mlp_precision)
        keep.append(m)
        p.mlp = C.pointer(m)
    return p, keep


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def render(sc: Scene, out: Optional[torch.Tensor] = None, stream=None, fields=None) -> torch.Tensor:
    """Cube [nch, ny, nx] (float32, on the scene's device)."""
    dev = sc.ln_nh2.device
    if out is None:
        out = torch.empty(sc.nch, sc.ny, sc.nx, dtype=torch.float32, device=dev)
    if out.shape != (sc.nch, sc.ny, sc.nx):
        raise ValueError("output has the wrong shape")
    p, keep = problem_struct(sc, fields)
    L.check(L.lib().rt_render_cube(C.byref(p), _fptr(out), C.c_void_p(_stream(stream))))
    del keep
    return out


GRAD_KEYS = ("ln_nh2", "temp_k", "vphi_kms", "z_lo_au", "z_up_au", "mlp_w")


def render_adjoint(sc: Scene, dl_dcube: torch.Tensor, want=GRAD_KEYS, cube_out: Optional[torch.Tensor] = None,
                   stream=None, fields=None) -> dict:
    """Gradients of L w.r.t. the requested inputs given dL/dcube."""
    dev = sc.ln_nh2.device
    dl = dl_dcube.contiguous().to(torch.float32)
    if dl.shape != (sc.nch, sc.ny, sc.nx):
        raise ValueError("dL/dcube has the wrong shape")
    shapes = dict(ln_nh2=(sc.nr, sc.nz), temp_k=(sc.nr, sc.nz), vphi_kms=(sc.nr, sc.nz), z_lo_au=(sc.nr,),
                  z_up_au=(sc.nr,), mlp_w=(L.RT_MLP_PARAMS,))
    out = {}
    for k in want:
        if k == "mlp_w" and sc.mlp_w is None:
            continue
        out[k] = torch.empty(shapes[k], dtype=torch.float32, device=dev)
    g = L.rt_grads(_fptr(out.get("ln_nh2")), _fptr(out.get("temp_k")), _fptr(out.get("vphi_kms")),
                   _fptr(out.get("z_lo_au")), _fptr(out.get("z_up_au")), _fptr(out.get("mlp_w")))
    p, keep = problem_struct(sc, fields)
    L.check(L.lib().rt_render_cube_adjoint(C.byref(p), _fptr(dl), C.byref(g), _fptr(cube_out),
                                           C.c_void_p(_stream(stream))))
    del keep
    return out


def render_l2_adjoint(sc: Scene, target: torch.Tensor, want=GRAD_KEYS, cube_out: Optional[torch.Tensor] = None,
                      stream=None, fields=None, loss_out: Optional[torch.Tensor] = None, grads_out=None,
                      noalloc: bool = False):
    """Forward + L2 loss + adjoint in one pass: (cube, loss, gradients) of
    L = sum (cube - target)^2; loss is a one-element float64 device tensor.
    With noalloc the library call allocates nothing (rt_render_cube_l2_
    adjoint_noalloc: grid fields only); pass cube_out, loss_out and grads_out
    (name -> tensor) to keep this function from allocating the outputs."""
    dev = sc.ln_nh2.device
    tgt = target.contiguous().to(torch.float32)
    if tgt.shape != (sc.nch, sc.ny, sc.nx):
        raise ValueError("target has the wrong shape")
    cube = torch.empty(sc.nch, sc.ny, sc.nx, dtype=torch.float32, device=dev) if cube_out is None else cube_out
    loss = torch.empty(1, dtype=torch.float64, device=dev) if loss_out is None else loss_out
    shapes = dict(ln_nh2=(sc.nr, sc.nz), temp_k=(sc.nr, sc.nz), vphi_kms=(sc.nr, sc.nz), z_lo_au=(sc.nr,),
                  z_up_au=(sc.nr,), mlp_w=(L.RT_MLP_PARAMS,))
    out = {}
    if grads_out is not None:
        out = dict(grads_out)
    else:
        for k in want:
            if k == "mlp_w" and sc.mlp_w is None:
                continue
            out[k] = torch.empty(shapes[k], dtype=torch.float32, device=dev)
    for k, v in out.items():
        if tuple(v.shape) != shapes[k] or v.dtype != torch.float32 or not v.is_contiguous():
            raise ValueError(f"gradient output {k} must be a contiguous float32 tensor of shape {shapes[k]}")
    g = L.rt_grads(_fptr(out.get("ln_nh2")), _fptr(out.get("temp_k")), _fptr(out.get("vphi_kms")),
                   _fptr(out.get("z_lo_au")), _fptr(out.get("z_up_au")), _fptr(out.get("mlp_w")))
    p, keep = problem_struct(sc, fields)
    fn = L.lib().rt_render_cube_l2_adjoint_noalloc if noalloc else L.lib().rt_render_cube_l2_adjoint
    L.check(fn(C.byref(p), _fptr(tgt), C.byref(g), _fptr(cube), loss.data_ptr(), C.c_void_p(_stream(stream))))
    del keep
    return cube, loss, out


class Render(torch.autograd.Function):
    """cube = Render.apply(scene, ln_nh2, temp_k, vphi_kms, z_lo_au, z_up_au, mlp_w)."""

    @staticmethod
    def forward(ctx, sc, ln_nh2, temp_k, vphi_kms, z_lo_au, z_up_au, mlp_w=None):
        fields = dict(ln_nh2=ln_nh2.detach().contiguous(), temp_k=temp_k.detach().contiguous(),
                      vphi_kms=vphi_kms.detach().contiguous(), z_lo_au=z_lo_au.detach().contiguous(),
                      z_up_au=z_up_au.detach().contiguous(),
                      mlp_w=None if mlp_w is None else mlp_w.detach().contiguous())
        ctx.sc = sc
        ctx.fields = fields
        return render(sc, fields=fields)

    @staticmethod
    def backward(ctx, grad_out):
        want = [k for k, need in zip(GRAD_KEYS, ctx.needs_input_grad[1:]) if need]
        g = render_adjoint(ctx.sc, grad_out, want=want, fields=ctx.fields)
        return (None,) + tuple(g.get(k) for k in GRAD_KEYS)


def render_differentiable(sc: Scene, ln_nh2=None, temp_k=None, vphi_kms=None, z_lo_au=None, z_up_au=None,
                          mlp_w=None) -> torch.Tensor:
    a = lambda x, d: d if x is None else x
    return Render.apply(sc, a(ln_nh2, sc.ln_nh2), a(temp_k, sc.temp_k), a(vphi_kms, sc.vphi_kms),
                        a(z_lo_au, sc.z_lo_au), a(z_up_au, sc.z_up_au), a(mlp_w, sc.mlp_w))


def set_option(key: int, value: int) -> None:
    L.check(L.lib().rt_set_option(key, value))


def get_option(key: int) -> int:
    return int(L.lib().rt_get_option(key))


def constants() -> dict:
    out = (C.c_double * 6)()
    L.lib().rt_constants(out, 6)
    return dict(zip(["h", "k_B", "c", "amu", "au", "pi"], list(out)))


@dataclass
class DiskPhysics:
    """Parameters of the fields derived from a temperature grid (rt_derive
    without the grid and the temperature)."""
    mstar_msun: float
    mgas_msun: float
    rc_au: float
    gamma: float
    mu: float = 2.37
    t_freeze_k: float = 20.0
    n_dissoc_cm2: float = 1e21


def _derive_struct(grid, temp_k: torch.Tensor, phys: DiskPhysics):
    nr, nz, r_min, r_max, zr_max = grid
    if temp_k.shape != (nr, nz):
        raise ValueError("temperature grid has the wrong shape")
    g = L.rt_grid(int(nr), int(nz), float(r_min), float(r_max), float(zr_max))
    return L.rt_derive(g, _fptr(temp_k), phys.mstar_msun, phys.mgas_msun, phys.rc_au, phys.gamma, phys.mu,
                       phys.t_freeze_k, phys.n_dissoc_cm2)


def derive_fields(grid, temp_k: torch.Tensor, phys: DiskPhysics, stream=None) -> dict:
    """ln_nh2, vphi_kms [nr, nz] and z_lo_au, z_up_au [nr] derived from the
    temperature grid; grid = (nr, nz, r_min_au, r_max_au, zr_max)."""
    nr, nz = int(grid[0]), int(grid[1])
    T = temp_k.contiguous()
    dev = T.device
    out = dict(ln_nh2=torch.empty(nr, nz, dtype=torch.float32, device=dev),
               vphi_kms=torch.empty(nr, nz, dtype=torch.float32, device=dev),
               z_lo_au=torch.empty(nr, dtype=torch.float32, device=dev),
               z_up_au=torch.empty(nr, dtype=torch.float32, device=dev))
    d = _derive_struct(grid, T, phys)
    o = L.rt_derived(_fptr(out["ln_nh2"]), _fptr(out["vphi_kms"]), _fptr(out["z_lo_au"]), _fptr(out["z_up_au"]))
    L.check(L.lib().rt_derive_fields(C.byref(d), C.byref(o), C.c_void_p(_stream(stream))))
    return out


def derive_fields_adjoint(grid, temp_k: torch.Tensor, phys: DiskPhysics, cot: dict, stream=None,
                          add_to: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dL/dT through the derived fields, given dL/d(each output) (missing
    keys count as zero).  With add_to (a float32 [nr, nz] tensor, e.g. the
    render's direct dL/dT) the product is added to it in place by the
    library (rt_derive_fields_adjoint_add) and add_to is returned."""
    T = temp_k.contiguous()
    c = {k: (None if cot.get(k) is None else cot[k].contiguous().to(torch.float32))
         for k in ("ln_nh2", "vphi_kms", "z_lo_au", "z_up_au")}
    d = _derive_struct(grid, T, phys)
    o = L.rt_derived(_fptr(c["ln_nh2"]), _fptr(c["vphi_kms"]), _fptr(c["z_lo_au"]), _fptr(c["z_up_au"]))
    if add_to is not None:
        if add_to.shape != T.shape or add_to.dtype != torch.float32 or not add_to.is_contiguous():
            raise ValueError("add_to must be a contiguous float32 tensor shaped like temp_k")
        L.check(L.lib().rt_derive_fields_adjoint_add(C.byref(d), C.byref(o), _fptr(add_to),
                                                      C.c_void_p(_stream(stream))))
        return add_to
    dT = torch.empty_like(T)
    L.check(L.lib().rt_derive_fields_adjoint(C.byref(d), C.byref(o), _fptr(dT), C.c_void_p(_stream(stream))))
    return dT


class DeriveFields(torch.autograd.Function):
    """(ln_nh2, vphi_kms, z_lo_au, z_up_au) = DeriveFields.apply(grid, phys, temp_k)."""

    @staticmethod
    def forward(ctx, grid, phys, temp_k):
        T = temp_k.detach().contiguous()
        ctx.grid, ctx.phys = grid, phys
        ctx.save_for_backward(T)
        out = derive_fields(grid, T, phys)
        return out["ln_nh2"], out["vphi_kms"], out["z_lo_au"], out["z_up_au"]

    @staticmethod
    def backward(ctx, g_n, g_v, g_lo, g_up):
        (T,) = ctx.saved_tensors
        cot = dict(ln_nh2=g_n, vphi_kms=g_v, z_lo_au=g_lo, z_up_au=g_up)
        return None, None, derive_fields_adjoint(ctx.grid, T, ctx.phys, cot)


def parametric_temperature(grid, t_mid0_k, t_atm0_k, q, r_scale_au, zq0_au, delta, device="cuda",
                           stream=None) -> torch.Tensor:
    """Two-layer parametric temperature [nr, nz] at the grid nodes."""
    nr, nz, r_min, r_max, zr_max = grid
    T = torch.empty(int(nr), int(nz), dtype=torch.float32, device=device)
    g = L.rt_grid(int(nr), int(nz), float(r_min), float(r_max), float(zr_max))
    pt = L.rt_param_temp(t_mid0_k, t_atm0_k, q, r_scale_au, zq0_au, delta)
    L.check(L.lib().rt_parametric_temperature(C.byref(g), C.byref(pt), _fptr(T), C.c_void_p(_stream(stream))))
    return T


# ---------------------------------------------------------------- 3-D spherical grid

@dataclass
class Scene3d:
    """A 3-D problem with its packed node records resident on the GPU.
    grid = (nr, nt, np, r_min_au, r_max_au, th_min, th_max); nodes: [nr, nt,
    np, 8] float32 from pack_fields3d."""
    grid: tuple
    nodes: torch.Tensor
    v_turb: float
    nu0_hz: float
    a_ul: float
    g_u: float
    g_l: float
    e_u_k: float
    e_l_k: float
    m_co_amu: float
    m_mol_amu: float
    lev_e_k: np.ndarray
    lev_g: np.ndarray
    nx: int
    ny: int
    fov_au: float
    incl_deg: float
    pa_deg: float
    dist_pc: float
    v_kms: np.ndarray
    v_sys_kms: float
    nsamp: int
    intensity_scale: float = 1.0

    @property
    def nch(self) -> int:
        return int(len(self.v_kms))

    def census(self, stream=None) -> dict:
        """The library's work accounting of this 3-D render
        (rt_render_census_3d): the [ny, nx] bool mask of rays that cross the
        bounding sphere r <= r_max e^dln, their number and pixel-samples, and
        how many of those the march takes as optically thin, have any
        opacity, and lie inside the grid's fade."""
        mask = torch.empty(self.ny, self.nx, dtype=torch.uint8, device=self.nodes.device)
        counts = (C.c_int64 * 5)()
        p, keep = _problem3d(self)
        L.check(L.lib().rt_render_census_3d(C.byref(p), mask.data_ptr(), counts, C.c_void_p(_stream(stream))))
        return dict(mask=mask.cpu().numpy().astype(bool), rays=int(counts[0]), pixel_samples=int(counts[1]),
                    thin_pixel_samples=int(counts[2]), emitting_pixel_samples=int(counts[3]),
                    shaded_pixel_samples=int(counts[4]))

    def live_mask(self) -> np.ndarray:
        """[ny, nx] bool: pixels whose ray crosses the bounding sphere."""
        return self.census()["mask"]

    @property
    def ray_samples(self) -> int:
        """(pixel, channel, sample) triples of the rays that cross the grid."""
        return self.census()["pixel_samples"] * self.nch

    def replace(self, **kw) -> "Scene3d":
        return replace(self, **kw)


def _grid3d(grid) -> "L.rt_grid3d":
    nr, nt, nph, r_min, r_max, th_min, th_max = grid
    return L.rt_grid3d(int(nr), int(nt), int(nph), float(r_min), float(r_max), float(th_min), float(th_max))


def pack_fields3d(grid, ln_nh2, temp_k, x_co, v_r=None, v_theta=None, v_phi=None, out=None,
                  stream=None) -> torch.Tensor:
    """Interleave the six [nr, nt, np] planes into the node records [nr, nt, np, 8]."""
    nr, nt, nph = (int(v) for v in grid[:3])
    n = nr * nt * nph
    for name, t in (("ln_nh2", ln_nh2), ("temp_k", temp_k), ("x_co", x_co), ("v_r", v_r), ("v_theta", v_theta),
                    ("v_phi", v_phi)):
        if t is not None and t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if out is None:
        out = torch.empty(nr, nt, nph, 8, dtype=torch.float32, device=ln_nh2.device)
    if out.numel() != 8 * n:
        raise ValueError("node buffer has the wrong size")
    g = _grid3d(grid)
    L.check(L.lib().rt_pack_fields3d(C.byref(g), _fptr(ln_nh2), _fptr(temp_k), _fptr(x_co), _fptr(v_r),
                                     _fptr(v_theta), _fptr(v_phi), _fptr(out), C.c_void_p(_stream(stream))))
    return out


def scene3d_from_problem(prob, device="cuda") -> Scene3d:
    """Copy a 3-D problem (attributes as in synth.disk3d.Problem3) to the GPU and pack its fields."""
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
    g, cam, line = prob.grid, prob.camera, prob.line
    grid = (g.nr, g.nt, g.nphi, g.r_min_au, g.r_max_au, g.th_min, g.th_max)
    nodes = pack_fields3d(grid, t(prob.ln_nh2), t(prob.temp_k), t(prob.x_co), t(prob.v_r_kms),
                          t(prob.v_theta_kms), t(prob.v_phi_kms))
    return Scene3d(grid=grid, nodes=nodes, v_turb=prob.v_turb, nu0_hz=line.nu0_hz, a_ul=line.a_ul, g_u=line.g_u,
                   g_l=line.g_l, e_u_k=line.e_u_k, e_l_k=line.e_l_k, m_co_amu=line.m_co_amu,
                   m_mol_amu=line.m_mol_amu, lev_e_k=np.ascontiguousarray(line.lev_e_k, np.float64),
                   lev_g=np.ascontiguousarray(line.lev_g, np.float64), nx=cam.nx, ny=cam.ny, fov_au=cam.fov_au,
                   incl_deg=cam.incl_deg, pa_deg=cam.pa_deg, dist_pc=cam.dist_pc,
                   v_kms=np.ascontiguousarray(prob.v_kms, np.float64), v_sys_kms=prob.v_sys_kms,
                   nsamp=prob.nsamp, intensity_scale=prob.intensity_scale)


def render3d(sc: Scene3d, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Cube [nch, ny, nx] (float32) of a 3-D scene."""
    nr, nt, nph = (int(v) for v in sc.grid[:3])
    if sc.nodes.numel() != 8 * nr * nt * nph:
        raise ValueError("node records do not match the grid")
    if out is None:
        out = torch.empty(sc.nch, sc.ny, sc.nx, dtype=torch.float32, device=sc.nodes.device)
    if out.shape != (sc.nch, sc.ny, sc.nx):
        raise ValueError("output has the wrong shape")
    p, keep = _problem3d(sc)
    L.check(L.lib().rt_render_cube_3d(C.byref(p), _fptr(out), C.c_void_p(_stream(stream))))
    return out


def _problem3d(sc: Scene3d):
    """(rt_problem3d, keepalive) of a 3-D scene."""
    lev_e = np.ascontiguousarray(sc.lev_e_k, np.float64)
    lev_g = np.ascontiguousarray(sc.lev_g, np.float64)
    vk = np.ascontiguousarray(sc.v_kms, np.float64)
    p = L.rt_problem3d()
    p.grid = _grid3d(sc.grid)
    p.nodes = _fptr(sc.nodes)
    p.v_turb = sc.v_turb
    p.line = L.rt_line(sc.nu0_hz, sc.a_ul, sc.g_u, sc.g_l, sc.e_u_k, sc.e_l_k, sc.m_co_amu, sc.m_mol_amu,
                       len(lev_e), lev_e.ctypes.data_as(C.POINTER(C.c_double)),
                       lev_g.ctypes.data_as(C.POINTER(C.c_double)))
    p.cam = L.rt_camera(sc.nx, sc.ny, sc.fov_au, sc.incl_deg, sc.pa_deg, sc.dist_pc)
    p.spec = L.rt_spectral(len(vk), vk.ctypes.data_as(C.POINTER(C.c_double)), sc.v_sys_kms)
    p.nsamp = sc.nsamp
    p.intensity_scale = sc.intensity_scale
    return p, (lev_e, lev_g, vk)


# ---------------------------------------------------------------- beam convolution

def beam_convolve(cube: torch.Tensor, bmaj_px: float, bmin_px: float, bpa_deg: float,
                  out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """cube [nch, ny, nx] convolved with the normalised elliptical Gaussian beam."""
    if cube.dim() != 3:
        raise ValueError("expected a cube [nch, ny, nx]")
    if out is None:
        out = torch.empty_like(cube)
    if out.shape != cube.shape:
        raise ValueError("output has the wrong shape")
    b = L.rt_beam(float(bmaj_px), float(bmin_px), float(bpa_deg))
    nch, ny, nx = cube.shape
    L.check(L.lib().rt_beam_convolve(_fptr(cube), _fptr(out), nch, ny, nx, C.byref(b), C.c_void_p(_stream(stream))))
    return out


class BeamConvolve(torch.autograd.Function):
    """BeamConvolve.apply(cube, bmaj_px, bmin_px, bpa_deg); the operator is its own adjoint."""

    @staticmethod
    def forward(ctx, cube, bmaj_px, bmin_px, bpa_deg):
        ctx.beam = (bmaj_px, bmin_px, bpa_deg)
        return beam_convolve(cube.detach().contiguous(), bmaj_px, bmin_px, bpa_deg)

    @staticmethod
    def backward(ctx, g):
        return beam_convolve(g.contiguous(), *ctx.beam), None, None, None
