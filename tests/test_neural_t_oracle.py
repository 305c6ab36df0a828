"""Pins of the neural-temperature oracle (oracle/neural_t.py): exact values of
the encoding, a network small enough to evaluate by hand, the sigmoid range,
Adam's closed form under a constant gradient, and central differences of the
FP64 forward for its gradient."""
import math

import numpy as np
import pytest
import torch

from oracle import neural_t as N


def test_encoding_values_at_exact_points():
    f = N.features(3, 5).numpy()           # x_r in {0, 1/2, 1}, x_z in {0, 1/4, ..., 1}
    node = lambda i, j: f[i * 5 + j]
    # x = 0: sines 0, cosines 1
    np.testing.assert_allclose(node(0, 0), [0] * 4 + [1] * 4 + [0] * 4 + [1] * 4, atol=1e-15)
    # x_r = 1/2: sin(pi/2) = 1, sin(pi) = 0, ...; cos(pi/2) = 0, cos(pi) = -1, cos(2 pi) = 1
    np.testing.assert_allclose(node(1, 0)[:8], [1, 0, 0, 0, 0, -1, 1, 1], atol=1e-15)
    # x_z = 1/4: sin(pi/4), sin(pi/2), sin(pi), sin(2 pi)
    s = math.sqrt(0.5)
    np.testing.assert_allclose(node(0, 1)[8:], [s, 1, 0, 0, s, 0, -1, 1], atol=1e-15)


def test_hand_evaluated_network():
    """One active path: feature 4 (cos(pi x_r)) -> unit 0 of every hidden
    layer with weight 2 and bias 0.5 -> output weight -1, bias 0.25."""
    w = np.zeros(sum(o * i + o for o, i in N.layer_shapes()))
    off = 0
    for li, (o, i) in enumerate(N.layer_shapes()):
        W = np.zeros((o, i))
        b = np.zeros(o)
        if li == 0:
            W[0, 4], b[0] = 2.0, 0.5
        elif li < 4:
            W[0, 0], b[0] = 2.0, 0.5
        else:
            W[0, 0], b[0] = -1.0, 0.25
        w[off:off + o * i] = W.ravel()
        off += o * i
        w[off:off + o] = b
        off += o
    T = N.temperature(torch.tensor(w), 3, 2).numpy()
    for i, xr in enumerate((0.0, 0.5, 1.0)):
        h = max(2.0 * math.cos(math.pi * xr) + 0.5, 0.0)
        for _ in range(3):
            h = max(2.0 * h + 0.5, 0.0)
        o = -h + 0.25
        np.testing.assert_allclose(T[i], 5.0 + 395.0 / (1.0 + math.exp(-o)), rtol=1e-14)


def test_temperature_range_and_zero_network():
    w = torch.zeros(sum(o * i + o for o, i in N.layer_shapes()), dtype=torch.float64)
    np.testing.assert_allclose(N.temperature(w, 4, 3).numpy(), 5.0 + 395.0 / 2.0, rtol=1e-15)
    rng = np.random.default_rng(1)
    T = N.temperature(torch.tensor(50.0 * rng.standard_normal(w.shape)), 7, 9).numpy()
    assert T.min() >= 5.0 and T.max() <= 400.0


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias corrections are exact: every step
    moves by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    lrs = [1e-3, 5e-4, 2e-4, 1e-4]
    for t, lr in enumerate(lrs, start=1):
        p, m, v = N.adam(p, m, v, g, t, lr)
    np.testing.assert_allclose(p, -sum(lrs) * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert N.poly_lr(0, 100) == pytest.approx(1e-4) and N.poly_lr(100, 100) == pytest.approx(1e-6)
    assert N.poly_lr(50, 100) == pytest.approx(0.5 * (1e-4 + 1e-6))


def test_gradient_matches_central_differences():
    import synth.mlp as SM
    w0 = SM.make_neural_t_weights(3).astype(np.float64)
    rng = np.random.default_rng(2)
    c = torch.tensor(rng.standard_normal((6, 5)))
    w = torch.tensor(w0, requires_grad=True)
    (N.temperature(w, 6, 5) * c).sum().backward()
    g = w.grad.numpy()
    for p in rng.choice(len(w0), size=12, replace=False):
        h = 1e-6 * max(1.0, abs(w0[p]))
        wp, wm = w0.copy(), w0.copy()
        wp[p] += h
        wm[p] -= h
        fd = ((N.temperature(torch.tensor(wp), 6, 5) - N.temperature(torch.tensor(wm), 6, 5)) * c).sum().item() / (2 * h)
        assert g[p] == pytest.approx(fd, rel=1e-6, abs=1e-8 * np.abs(g).max()), p
