"""FP64 oracle of the paper's neural temperature field and of the Adam step.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU leg use this module.  Plain float64 torch / numpy on
the CPU, from Methods, "Neural Temperature Recovery":

  * T(r, |z|) = MLP(gamma(r, |z|)): the sinusoidal encoding of degree L = 4 of
    the two normalised node coordinates x_r = i/(nr-1), x_z = j/(nz-1) of the
    (r, z/r) grid -- [sin(2^k pi x_r)]_k, [cos(2^k pi x_r)]_k,
    [sin(2^k pi x_z)]_k, [cos(2^k pi x_z)]_k for k = 0..3, 16 features --
    then four fully connected layers of 64 units with ReLU and one output o;
    the output sigmoid maps to the range [5, 400] K: T = 5 + 395 sigma(o).
    Flat float32 layout per layer: W [out][in] then b [out];
  * Adam (Kingma & Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) at step t >= 1;
  * the learning rate decays polynomially (power 1) from lr0 to lr1 over the
    schedule: lr(t) = lr1 + (lr0 - lr1) (1 - t / T).
"""
from __future__ import annotations

import math

import numpy as np
import torch

L_ENC = 4
WIDTH = 64
DEPTH = 4
T_MIN, T_MAX = 5.0, 400.0


def features(nr, nz):
    """[nr * nz, 16] float64 encoding of the node coordinates (node n = i nz + j)."""
    i, j = np.meshgrid(np.arange(nr), np.arange(nz), indexing="ij")
    xr = (i / (nr - 1)).ravel()
    xz = (j / (nz - 1)).ravel()
    cols = []
    for x in (xr, xz):
        cols += [np.sin(2.0 ** k * math.pi * x) for k in range(L_ENC)]
        cols += [np.cos(2.0 ** k * math.pi * x) for k in range(L_ENC)]
    return torch.tensor(np.stack(cols, axis=1), dtype=torch.float64)


def layer_shapes():
    dims = [4 * L_ENC] + [WIDTH] * DEPTH + [1]
    return [(dims[k + 1], dims[k]) for k in range(len(dims) - 1)]


def temperature(w, nr, nz):
    """T [nr][nz] (float64 tensor) for the flat weights w (float64 tensor)."""
    h = features(nr, nz)
    off = 0
    shapes = layer_shapes()
    for li, (o, i) in enumerate(shapes):
        W = w[off:off + o * i].view(o, i)
        off += o * i
        b = w[off:off + o]
        off += o
        h = h @ W.T + b
        if li < len(shapes) - 1:
            h = torch.relu(h)
    return (T_MIN + (T_MAX - T_MIN) * torch.sigmoid(h[:, 0])).view(nr, nz)


def adam(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in float64 numpy; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def poly_lr(t, total, lr0=1e-4, lr1=1e-6):
    return lr1 + (lr0 - lr1) * (1.0 - min(t, total) / total)
