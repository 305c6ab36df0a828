"""FP64 oracle of the beam convolution of a model cube (TEST INFRASTRUCTURE:
only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it; it shares no code with the GPU library).

A synthetic cube is compared with a CLEANed interferometric image only after
it has been convolved with the image's restoring beam (Methods, MCMC
inference: the model cubes are compared with the observed channel maps; the
paper does not spell out the convolution).  Reading used here: every channel
map is convolved with the same elliptical Gaussian of full widths at half
maximum ``bmaj`` >= ``bmin`` (pixels) whose major axis lies at position angle
``bpa`` (degrees) from +y towards -x (east of north with east to the left);
the kernel is sampled at integer pixel offsets within |dx|, |dy| <= R =
ceil(3 sigma_maj), normalised to unit sum (flux per pixel is conserved), and
pixels outside the image count as zero.
"""
from __future__ import annotations

import math

import numpy as np


def kernel(bmaj: float, bmin: float, bpa_deg: float) -> np.ndarray:
    """Normalised (2R+1) x (2R+1) kernel, indexed [dy + R, dx + R]."""
    s_maj = bmaj / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    s_min = bmin / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    R = int(math.ceil(3.0 * s_maj))
    pa = math.radians(bpa_deg)
    d = np.arange(-R, R + 1, dtype=np.float64)
    dy, dx = np.meshgrid(d, d, indexing="ij")
    u = -dx * math.sin(pa) + dy * math.cos(pa)     # along the major axis
    v = dx * math.cos(pa) + dy * math.sin(pa)      # along the minor axis
    k = np.exp(-0.5 * ((u / s_maj) ** 2 + (v / s_min) ** 2))
    return k / k.sum()


def convolve(cube: np.ndarray, bmaj: float, bmin: float, bpa_deg: float) -> np.ndarray:
    """out[c, y, x] = sum_{dy, dx} K[dy, dx] in[c, y - dy, x - dx] (zero outside)."""
    cube = np.asarray(cube, np.float64)
    k = kernel(bmaj, bmin, bpa_deg)
    R = (k.shape[0] - 1) // 2
    nch, ny, nx = cube.shape
    pad = np.zeros((nch, ny + 2 * R, nx + 2 * R))
    pad[:, R:R + ny, R:R + nx] = cube
    out = np.zeros((nch, ny, nx))
    for iy in range(2 * R + 1):
        for ix in range(2 * R + 1):
            # offset (dy, dx) = (iy - R, ix - R) reads in[y - dy, x - dx]
            dy, dx = iy - R, ix - R
            out += k[iy, ix] * pad[:, R - dy:R - dy + ny, R - dx:R - dx + nx]
    return out
