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


# Neural temperature field of the paper (Methods, "Neural Temperature
# Recovery"): sinusoidal encoding of degree 4 on the two normalised grid
# coordinates (16 features) -> 4 ReLU layers of width 64 -> 1 output.
NT_L = 4
NT_IN = 4 * NT_L
NT_WIDTH = 64
NT_DEPTH = 4


def nt_layer_shapes():
    dims = [NT_IN] + [NT_WIDTH] * NT_DEPTH + [1]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def nt_param_count() -> int:
    return sum(o * i + o for o, i in nt_layer_shapes())


def make_neural_t_weights(seed: int = 6, t_init_k: float = 30.0) -> np.ndarray:
    """He-normal hidden weights (ReLU), Xavier-normal output layer, zero
    hidden biases, output bias putting the initial temperature near t_init_k
    on the 5..400 K sigmoid range."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    shapes = nt_layer_shapes()
    for li, (o, i) in enumerate(shapes):
        last = li == len(shapes) - 1
        std = np.sqrt(2.0 / (i + o)) if last else np.sqrt(2.0 / i)
        parts.append(rng.standard_normal((o, i)) * std)
        f = (t_init_k - 5.0) / 395.0
        parts.append(np.full(o, np.log(f / (1 - f))) if last else np.zeros(o))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
