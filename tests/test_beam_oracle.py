"""Pins of the beam-convolution oracle (oracle/beam.py): flux conservation,
a Gaussian source broadened to the quadrature sum of widths, the separable
form of an axis-aligned beam, and the mirror and transpose symmetries that
fix the position-angle convention."""
import math

import numpy as np
import pytest

from oracle import beam as B

FW = 2.0 * math.sqrt(2.0 * math.log(2.0))


def test_kernel_unit_sum_and_half_maximum():
    k = B.kernel(6.0, 6.0, 0.0)
    R = (k.shape[0] - 1) // 2
    assert k.sum() == pytest.approx(1.0, rel=1e-15)
    assert R == math.ceil(3 * 6.0 / FW)
    # FWHM: the kernel falls to half its peak 3 pixels from the centre
    assert k[R, R + 3] / k[R, R] == pytest.approx(0.5, rel=1e-12)
    assert k[R + 3, R] / k[R, R] == pytest.approx(0.5, rel=1e-12)


def test_flux_conserved_away_from_edges():
    rng = np.random.default_rng(1)
    img = np.zeros((2, 64, 64))
    img[:, 20:44, 20:44] = rng.random((2, 24, 24))
    out = B.convolve(img, 7.0, 4.0, 30.0)
    np.testing.assert_allclose(out.sum(axis=(1, 2)), img.sum(axis=(1, 2)), rtol=1e-13)


def test_gaussian_source_widths_add_in_quadrature():
    """A circular Gaussian source of width s convolved with a circular beam of
    width b is a Gaussian of width sqrt(s^2 + b^2) (continuous result; the
    sampled widths here are several pixels, truncation at 3 sigma)."""
    n = 129
    y, x = np.mgrid[0:n, 0:n] - 64.0
    s, b = 3.0, 4.0
    src = np.exp(-0.5 * (x ** 2 + y ** 2) / s ** 2)[None] / (2 * math.pi * s ** 2)
    out = B.convolve(src, b * FW, b * FW, 0.0)[0]
    w = math.hypot(s, b)
    ref = np.exp(-0.5 * (x ** 2 + y ** 2) / w ** 2) / (2 * math.pi * w ** 2)
    assert np.abs(out - ref).max() <= 4e-3 * ref.max()


def test_axis_aligned_beam_is_separable():
    """bpa = 0: major axis along y, so the kernel is a product of 1-D
    Gaussians of sigma_maj in y and sigma_min in x on the same support."""
    rng = np.random.default_rng(2)
    img = rng.random((1, 40, 50))
    bmaj, bmin = 9.0, 5.0
    out = B.convolve(img, bmaj, bmin, 0.0)[0]
    R = math.ceil(3 * bmaj / FW)
    d = np.arange(-R, R + 1)
    gy = np.exp(-0.5 * (d * FW / bmaj) ** 2)
    gx = np.exp(-0.5 * (d * FW / bmin) ** 2)
    gy, gx = gy / gy.sum(), gx / gx.sum()
    pad = np.zeros((40 + 2 * R, 50 + 2 * R))
    pad[R:R + 40, R:R + 50] = img[0]
    tmp = np.zeros((40 + 2 * R, 50))
    for i, w in enumerate(gx):
        tmp += w * pad[:, 2 * R - i:2 * R - i + 50]
    ref = np.zeros((40, 50))
    for i, w in enumerate(gy):
        ref += w * tmp[2 * R - i:2 * R - i + 40, :]
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-15)


def test_position_angle_mirror_and_transpose():
    rng = np.random.default_rng(3)
    img = rng.random((1, 48, 48))
    a = B.convolve(img, 8.0, 3.0, 25.0)
    # mirror x -> -x flips the sense of the position angle
    b = B.convolve(img[:, :, ::-1], 8.0, 3.0, -25.0)[:, :, ::-1]
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)
    # major axis along y (PA 0) on the transpose = major axis along x (PA 90)
    c = B.convolve(img, 8.0, 3.0, 90.0)
    d = np.swapaxes(B.convolve(np.swapaxes(img, 1, 2), 8.0, 3.0, 0.0), 1, 2)
    np.testing.assert_allclose(c, d, rtol=1e-12, atol=1e-15)
    # PA 90: the kernel is wider in x than in y
    k = B.kernel(8.0, 3.0, 90.0)
    R = (k.shape[0] - 1) // 2
    assert k[R, R + 3] > k[R + 3, R]


def test_position_angle_sense():
    """PA is measured from +y towards -x: at 45 degrees the major axis runs
    up and to the left."""
    k = B.kernel(8.0, 3.0, 45.0)
    R = (k.shape[0] - 1) // 2
    assert k[R + 3, R - 3] > 10 * k[R + 3, R + 3]     # (dy, dx) = (3, -3) on the axis, (3, 3) across it
