"""Seeded weights for the neural CO-layer field.

Network shape: 16 Fourier frequencies on 2 coordinates (64 features) ->
4 hidden layers of width 128 -> 3 outputs.  Flat float32 layout, layer by
layer: W_l as [out][in] row-major, then b_l [out].
"""
from __future__ import annotations

import numpy as np

MLP_NFREQ = 16
MLP_IN = 4 * MLP_NFREQ
MLP_WIDTH = 128
MLP_DEPTH = 4
MLP_OUT = 3


def layer_shapes():
    dims = [MLP_IN] + [MLP_WIDTH] * MLP_DEPTH + [MLP_OUT]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def mlp_param_count() -> int:
    return sum(o * i + o for o, i in layer_shapes())


def make_mlp_weights(seed: int = 4, out_bias=(0.6, 0.1, None)) -> np.ndarray:
    """Xavier-normal weights, zero hidden biases; output biases are the
    logits of the given fractions (None = 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    shapes = layer_shapes()
    for li, (o, i) in enumerate(shapes):
        std = np.sqrt(2.0 / (i + o))
        parts.append(rng.standard_normal((o, i)) * std)
        b = np.zeros(o)
        if li == len(shapes) - 1:
            for k, f in enumerate(out_bias):
                if f is not None:
                    b[k] = np.log(f / (1 - f))
        parts.append(b)
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
