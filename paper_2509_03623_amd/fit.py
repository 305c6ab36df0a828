"""Fitting the paper's neural temperature field to a cube (Methods, "Neural
Temperature Recovery", optimisation and training): the network gives T on the
grid nodes, the derived fields follow from T, the render and its fused L2
adjoint give the chi^2 gradient, and Adam updates the weights.  Every step
runs in the library's kernels; this module only chains the calls.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .render import DiskPhysics, _fptr, _stream, derive_fields, derive_fields_adjoint, render_l2_adjoint


def _grid_struct(grid):
    nr, nz, r_min, r_max, zr_max = grid
    return L.rt_grid(int(nr), int(nz), float(r_min), float(r_max), float(zr_max))


def neural_temperature(grid, weights: torch.Tensor, stream=None) -> torch.Tensor:
    """T [nr, nz] on the grid nodes for the flat float32 weights."""
    T = torch.empty(int(grid[0]), int(grid[1]), dtype=torch.float32, device=weights.device)
    g = _grid_struct(grid)
    L.check(L.lib().rt_neural_temperature(C.byref(g), _fptr(weights.contiguous()), _fptr(T),
                                          C.c_void_p(_stream(stream))))
    return T


def neural_temperature_adjoint(grid, weights: torch.Tensor, d_temp_k: torch.Tensor, stream=None) -> torch.Tensor:
    dW = torch.empty(L.RT_NT_PARAMS, dtype=torch.float32, device=weights.device)
    g = _grid_struct(grid)
    L.check(L.lib().rt_neural_temperature_adjoint(C.byref(g), _fptr(weights.contiguous()),
                                                  _fptr(d_temp_k.contiguous().to(torch.float32)), _fptr(dW),
                                                  C.c_void_p(_stream(stream))))
    return dW


class NeuralTemperature(torch.autograd.Function):
    """T = NeuralTemperature.apply(grid, weights)."""

    @staticmethod
    def forward(ctx, grid, weights):
        w = weights.detach().contiguous()
        ctx.grid = grid
        ctx.save_for_backward(w)
        return neural_temperature(grid, w)

    @staticmethod
    def backward(ctx, g):
        (w,) = ctx.saved_tensors
        return None, neural_temperature_adjoint(ctx.grid, w, g)


class Adam:
    """Adam state (first and second moments, step count) for one float32
    parameter tensor, updated in place by rt_adam_step."""

    def __init__(self, params: torch.Tensor, beta1=0.9, beta2=0.999, eps=1e-8):
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0
        self.beta1, self.beta2, self.eps = beta1, beta2, eps

    def step(self, grad: torch.Tensor, lr: float, grad_scale: float = 1.0, stream=None) -> None:
        self.t += 1
        opt = L.rt_adam(lr, self.beta1, self.beta2, self.eps, grad_scale)
        L.check(L.lib().rt_adam_step(_fptr(self.params), _fptr(self.m), _fptr(self.v), _fptr(grad.contiguous()),
                                     self.params.numel(), C.byref(opt), self.t, C.c_void_p(_stream(stream))))


def poly_lr(t: int, total: int, lr0: float = 1e-4, lr1: float = 1e-6) -> float:
    """Learning rate decaying polynomially (power 1) from lr0 to lr1 over total steps."""
    return lr1 + (lr0 - lr1) * (1.0 - min(t, total) / total)


def fit_step(sc, grid, phys: DiskPhysics, opt: Adam, target: torch.Tensor, channels: np.ndarray, sigma: float,
             lr: float):
    """One optimisation step on the given channel slices of the loss chi^2 =
    sum((cube - target)/sigma)^2 = L2 / sigma^2 over those slices.  Every
    step runs in the library: network, derived fields, fused render + L2 +
    adjoint, the derived fields' adjoint added onto the render's dL/dT, the
    network's adjoint, and Adam with the gradient scaled by 1/sigma^2.
    Returns (L2 as a one-element float64 device tensor, dL2/dweights); the
    step's chi^2 is L2 / sigma^2."""
    w = opt.params
    T = neural_temperature(grid, w)
    fields = derive_fields(grid, T, phys)
    idx = torch.as_tensor(channels, device=target.device, dtype=torch.long)
    scb = sc.replace(v_kms=np.asarray(sc.v_kms)[channels], temp_k=T, **fields)
    tgt = target.index_select(0, idx).contiguous()
    _, l2, g = render_l2_adjoint(scb, tgt, want=("ln_nh2", "temp_k", "vphi_kms", "z_lo_au", "z_up_au"))
    dT = derive_fields_adjoint(grid, T, phys, g, add_to=g["temp_k"])
    dW = neural_temperature_adjoint(grid, w, dT)
    opt.step(dW, lr, grad_scale=1.0 / (sigma * sigma))
    return l2, dW
