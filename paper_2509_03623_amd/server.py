"""Python handle of the C-ABI render server (rt_server_* / rt_submit /
rt_poll / rt_wait / rt_cancel / rt_release).  Keeps each request's device tensors alive
until the request has finished."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _lib as L
from .render import Scene, _fptr, problem_struct

STATE_NAMES = {L.RT_TICKET_QUEUED: "queued", L.RT_TICKET_RUNNING: "running", L.RT_TICKET_DONE: "done",
               L.RT_TICKET_CANCELED: "canceled", L.RT_TICKET_FAILED: "failed"}


class Server:
    def __init__(self, hbm_budget_bytes: int = 64 << 30, max_slots: int = 64, max_pending: int = 100000,
                 streams: int = 4, device: int = 0):
        cfg = L.rt_server_cfg(hbm_budget_bytes, max_slots, max_pending, device, streams)
        h = C.c_void_p()
        L.check(L.lib().rt_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, sc: Scene, cube: torch.Tensor, target: Optional[torch.Tensor] = None,
               grads: Optional[dict] = None, loss_only: bool = False, beam=None) -> int:
        """Queue a render into cube [nch, ny, nx]; with target, also the
        gradients of L = sum (cube - target)^2 into the tensors of grads, or
        with loss_only just L (reported by poll / wait).  beam = (bmaj_px,
        bmin_px, bpa_deg) convolves a loss_only request's cube with that beam
        before the loss."""
        p, keep = problem_struct(sc)
        rq = L.rt_request()
        rq.problem = p
        if target is None:
            rq.kind = L.RT_REQ_FWD
        else:
            rq.kind = L.RT_REQ_FWD_LOSS if loss_only else L.RT_REQ_FWD_ADJ
        rq.cube = _fptr(cube)
        rq.target = _fptr(target)
        g = grads or {}
        rq.grads = L.rt_grads(_fptr(g.get("ln_nh2")), _fptr(g.get("temp_k")), _fptr(g.get("vphi_kms")),
                              _fptr(g.get("z_lo_au")), _fptr(g.get("z_up_au")), _fptr(g.get("mlp_w")))
        if beam is not None:
            rq.beam = L.rt_beam(*(float(v) for v in beam))
        t = C.c_uint64()
        L.check(L.lib().rt_submit(self._h, C.byref(rq), C.byref(t)))
        self._keep[t.value] = (sc, cube, target, g, keep)
        return t.value

    def _info(self, ticket, info):
        d = dict(state=STATE_NAMES.get(info.state, info.state), status=info.status, t_submit_ns=info.t_submit_ns,
                 t_admit_ns=info.t_admit_ns, t_done_ns=info.t_done_ns, loss=info.loss,
                 ray_samples=info.ray_samples)
        if d["state"] in ("done", "canceled", "failed"):
            self._keep.pop(ticket, None)
        return d

    def poll(self, ticket: int) -> dict:
        info = L.rt_ticket_info()
        L.check(L.lib().rt_poll(self._h, ticket, C.byref(info)))
        return self._info(ticket, info)

    def wait(self, ticket: int, timeout_s: float = 60.0) -> dict:
        info = L.rt_ticket_info()
        L.check(L.lib().rt_wait(self._h, ticket, C.byref(info), int(timeout_s * 1e9)))
        return self._info(ticket, info)

    def cancel(self, ticket: int) -> None:
        L.check(L.lib().rt_cancel(self._h, ticket))

    def release(self, ticket: int) -> None:
        """Forget a finished ticket (the server frees its copy of the request)."""
        L.check(L.lib().rt_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def close(self) -> None:
        if self._h:
            L.check(L.lib().rt_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
