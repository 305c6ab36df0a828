"""ctypes view of include/rtcube.h and the loader of librtcube.so.

Argument marshalling only: every step of the render runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtcube.so")

_f = C.POINTER(C.c_float)
_d = C.POINTER(C.c_double)
_dev = C.c_void_p          # device pointer: an address, never dereferenced on the host

RT_OK, RT_PENDING, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_EAGAIN, RT_ECANCELED, RT_ETOOBIG, RT_ENOTFOUND = \
    0, 1, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "RT_OK", 1: "RT_PENDING", -1: "RT_EINVAL", -2: "RT_ENOMEM", -3: "RT_EDEVICE",
                -4: "RT_EAGAIN", -5: "RT_ECANCELED", -6: "RT_ETOOBIG", -7: "RT_ENOTFOUND"}
RT_MLP_FP32, RT_MLP_BF16 = 0, 1
RT_MLP_PARAMS = 58243
RT_REQ_FWD, RT_REQ_FWD_ADJ, RT_REQ_FWD_LOSS = 0, 1, 2
RT_TICKET_QUEUED, RT_TICKET_RUNNING, RT_TICKET_DONE, RT_TICKET_CANCELED, RT_TICKET_FAILED = 0, 1, 2, 3, 4
RT_OPT_CHANNEL_BLOCK, RT_OPT_THIN_EXPM1, RT_OPT_CKPT_SEGMENT, RT_OPT_RAY_SPLIT, RT_OPT_GRAD_ACCUM = 1, 2, 3, 4, 5
RT_OPT_ADJ_SCRATCH_CAP, RT_OPT_ADJ_CHANNEL_BLOCK, RT_OPT_ADJ_PIXEL_LANES, RT_OPT_FWD_GROUP = 6, 7, 8, 9


class rt_grid(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("r_min_au", C.c_double), ("r_max_au", C.c_double),
                ("zr_max", C.c_double)]


class rt_fields(C.Structure):
    _fields_ = [("ln_nh2", _dev), ("temp_k", _dev), ("vphi_kms", _dev), ("z_lo_au", _dev), ("z_up_au", _dev),
                ("x_co", C.c_double), ("mask_width", C.c_double), ("v_turb", C.c_double)]


class rt_line(C.Structure):
    _fields_ = [("nu0_hz", C.c_double), ("a_ul", C.c_double), ("g_u", C.c_double), ("g_l", C.c_double),
                ("e_u_k", C.c_double), ("e_l_k", C.c_double), ("m_co_amu", C.c_double),
                ("m_mol_amu", C.c_double), ("nlev", C.c_int32), ("lev_e_k", _d), ("lev_g", _d)]


class rt_camera(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("fov_au", C.c_double), ("incl_deg", C.c_double),
                ("pa_deg", C.c_double), ("dist_pc", C.c_double)]


class rt_spectral(C.Structure):
    _fields_ = [("nch", C.c_int32), ("v_kms", _d), ("v_sys_kms", C.c_double)]


class rt_mlp(C.Structure):
    _fields_ = [("weights", _dev), ("precision", C.c_int32)]


class rt_problem(C.Structure):
    _fields_ = [("grid", rt_grid), ("f", rt_fields), ("line", rt_line), ("cam", rt_camera),
                ("spec", rt_spectral), ("nsamp", C.c_int32), ("intensity_scale", C.c_double),
                ("mlp", C.POINTER(rt_mlp))]


class rt_grads(C.Structure):
    _fields_ = [("d_ln_nh2", _dev), ("d_temp_k", _dev), ("d_vphi_kms", _dev), ("d_z_lo_au", _dev),
                ("d_z_up_au", _dev), ("d_mlp", _dev)]


class rt_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_slots", C.c_int32), ("max_pending", C.c_int32),
                ("device", C.c_int32), ("streams", C.c_int32)]


class rt_beam(C.Structure):
    _fields_ = [("bmaj_px", C.c_double), ("bmin_px", C.c_double), ("bpa_deg", C.c_double)]


RT_BEAM_MAX_RADIUS = 24


class rt_request(C.Structure):
    _fields_ = [("problem", rt_problem), ("kind", C.c_int32), ("cube", _dev), ("target", _dev),
                ("grads", rt_grads), ("beam", rt_beam)]


class rt_ticket_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("t_submit_ns", C.c_uint64),
                ("t_admit_ns", C.c_uint64), ("t_done_ns", C.c_uint64), ("loss", C.c_double),
                ("ray_samples", C.c_uint64)]


class rt_derive(C.Structure):
    _fields_ = [("grid", rt_grid), ("temp_k", _dev), ("mstar_msun", C.c_double), ("mgas_msun", C.c_double),
                ("rc_au", C.c_double), ("gamma", C.c_double), ("mu", C.c_double), ("t_freeze_k", C.c_double),
                ("n_dissoc_cm2", C.c_double)]


class rt_derived(C.Structure):
    _fields_ = [("ln_nh2", _dev), ("vphi_kms", _dev), ("z_lo_au", _dev), ("z_up_au", _dev)]


class rt_param_temp(C.Structure):
    _fields_ = [("t_mid0_k", C.c_double), ("t_atm0_k", C.c_double), ("q", C.c_double), ("r_scale_au", C.c_double),
                ("zq0_au", C.c_double), ("delta", C.c_double)]


class rt_adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("grad_scale", C.c_double)]


RT_NT_PARAMS = 13633


class rt_grid3d(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nt", C.c_int32), ("np", C.c_int32), ("r_min_au", C.c_double),
                ("r_max_au", C.c_double), ("th_min", C.c_double), ("th_max", C.c_double)]


class rt_problem3d(C.Structure):
    _fields_ = [("grid", rt_grid3d), ("nodes", _dev), ("v_turb", C.c_double), ("line", rt_line),
                ("cam", rt_camera), ("spec", rt_spectral), ("nsamp", C.c_int32), ("intensity_scale", C.c_double)]

# every symbol declared in include/rtcube.h
EXPORTS = ["rt_render_cube", "rt_render_cube_adjoint", "rt_render_cube_l2_adjoint",
           "rt_render_cube_l2_adjoint_noalloc", "rt_noalloc_scratch_bytes", "rt_render_census",
           "rt_render_census_3d", "rt_derive_fields", "rt_derive_fields_adjoint_add",
           "rt_derive_fields_adjoint", "rt_parametric_temperature", "rt_neural_temperature", "rt_neural_temperature_adjoint", "rt_adam_step",
           "rt_pack_fields3d", "rt_render_cube_3d", "rt_beam_convolve",
           "rt_server_create", "rt_submit", "rt_poll", "rt_wait",
           "rt_cancel", "rt_release", "rt_server_destroy", "rt_last_error", "rt_abi_version", "rt_constants",
           "rt_set_option", "rt_get_option"]

_lib = None


class RtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded librtcube.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2509_03623_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(rt_problem)
        L.rt_render_cube.argtypes = [P, _dev, C.c_void_p]
        L.rt_render_cube.restype = C.c_int
        L.rt_render_cube_adjoint.argtypes = [P, _dev, C.POINTER(rt_grads), _dev, C.c_void_p]
        L.rt_render_cube_adjoint.restype = C.c_int
        L.rt_render_cube_l2_adjoint.argtypes = [P, _dev, C.POINTER(rt_grads), _dev, _dev, C.c_void_p]
        L.rt_render_cube_l2_adjoint.restype = C.c_int
        L.rt_render_cube_l2_adjoint_noalloc.argtypes = [P, _dev, C.POINTER(rt_grads), _dev, _dev, C.c_void_p]
        L.rt_render_cube_l2_adjoint_noalloc.restype = C.c_int
        L.rt_noalloc_scratch_bytes.restype = C.c_uint64
        L.rt_render_census.argtypes = [P, _dev, C.POINTER(C.c_int64), C.c_void_p]
        L.rt_render_census.restype = C.c_int
        L.rt_render_census_3d.argtypes = [C.POINTER(rt_problem3d), _dev, C.POINTER(C.c_int64), C.c_void_p]
        L.rt_render_census_3d.restype = C.c_int
        L.rt_derive_fields.argtypes = [C.POINTER(rt_derive), C.POINTER(rt_derived), C.c_void_p]
        L.rt_derive_fields.restype = C.c_int
        L.rt_derive_fields_adjoint.argtypes = [C.POINTER(rt_derive), C.POINTER(rt_derived), _dev, C.c_void_p]
        L.rt_derive_fields_adjoint.restype = C.c_int
        L.rt_derive_fields_adjoint_add.argtypes = [C.POINTER(rt_derive), C.POINTER(rt_derived), _dev, C.c_void_p]
        L.rt_derive_fields_adjoint_add.restype = C.c_int
        L.rt_parametric_temperature.argtypes = [C.POINTER(rt_grid), C.POINTER(rt_param_temp), _dev, C.c_void_p]
        L.rt_parametric_temperature.restype = C.c_int
        L.rt_neural_temperature.argtypes = [C.POINTER(rt_grid), _dev, _dev, C.c_void_p]
        L.rt_neural_temperature.restype = C.c_int
        L.rt_neural_temperature_adjoint.argtypes = [C.POINTER(rt_grid), _dev, _dev, _dev, C.c_void_p]
        L.rt_neural_temperature_adjoint.restype = C.c_int
        L.rt_adam_step.argtypes = [_dev, _dev, _dev, _dev, C.c_int64, C.POINTER(rt_adam), C.c_int64, C.c_void_p]
        L.rt_adam_step.restype = C.c_int
        L.rt_pack_fields3d.argtypes = [C.POINTER(rt_grid3d), _dev, _dev, _dev, _dev, _dev, _dev, _dev, C.c_void_p]
        L.rt_pack_fields3d.restype = C.c_int
        L.rt_render_cube_3d.argtypes = [C.POINTER(rt_problem3d), _dev, C.c_void_p]
        L.rt_render_cube_3d.restype = C.c_int
        L.rt_beam_convolve.argtypes = [_dev, _dev, C.c_int32, C.c_int32, C.c_int32, C.POINTER(rt_beam), C.c_void_p]
        L.rt_beam_convolve.restype = C.c_int
        L.rt_server_create.argtypes = [C.POINTER(rt_server_cfg), C.POINTER(C.c_void_p)]
        L.rt_server_create.restype = C.c_int
        L.rt_submit.argtypes = [C.c_void_p, C.POINTER(rt_request), C.POINTER(C.c_uint64)]
        L.rt_submit.restype = C.c_int
        L.rt_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(rt_ticket_info)]
        L.rt_poll.restype = C.c_int
        L.rt_wait.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(rt_ticket_info), C.c_uint64]
        L.rt_wait.restype = C.c_int
        L.rt_cancel.argtypes = [C.c_void_p, C.c_uint64]
        L.rt_cancel.restype = C.c_int
        L.rt_release.argtypes = [C.c_void_p, C.c_uint64]
        L.rt_release.restype = C.c_int
        L.rt_server_destroy.argtypes = [C.c_void_p]
        L.rt_server_destroy.restype = C.c_int
        L.rt_last_error.restype = C.c_char_p
        L.rt_abi_version.restype = C.c_int32
        L.rt_constants.argtypes = [_d, C.c_int32]
        L.rt_constants.restype = C.c_int32
        L.rt_set_option.argtypes = [C.c_int32, C.c_int64]
        L.rt_set_option.restype = C.c_int
        L.rt_get_option.argtypes = [C.c_int32]
        L.rt_get_option.restype = C.c_int64
        _lib = L
    return _lib


def check(status: int) -> int:
    if status < 0:
        raise RtError(status, lib().rt_last_error().decode(errors="replace"))
    return status
