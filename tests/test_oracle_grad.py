"""Pins of the oracle's gradient (float64 torch autograd of the discrete march)
against central finite differences of the independent C forward, against
exact scaling identities, and a dot-product (directional derivative) test."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import torch_ref

FIELDS = ["ln_nh2", "temp_k", "vphi_kms", "z_lo_au", "z_up_au"]


def _problem(mlp_seed=None):
    prob = synth.small_problem(nx=14, ny=12, nch=6, nsamp=40, nr=20, nz=10, seed=5, dv=0.3,
                               mlp_seed=mlp_seed)
    return prob.replace(intensity_scale=synth.disk.rj_kelvin_scale(prob.line))


def _target(prob):
    tgt = synth.perturb_surfaces(prob, seed=30)
    if prob.mlp_w is not None:
        tgt = tgt.replace(mlp_w=synth.make_mlp_weights(99))
    return synth.disk.add_noise(oracle.render(tgt), 0.05, seed=31)


def _loss_c(prob, target, **fields):
    p2 = prob.replace(**fields) if fields else prob
    return oracle.loss(oracle.render(p2), target)


def _fd(prob, target, name, idx, h):
    """Central difference through the C forward.  The C oracle reads float32
    inputs, so the step actually taken is the float32-rounded one."""
    arr = getattr(prob, name)
    plus = arr.copy()
    minus = arr.copy()
    plus.flat[idx] = np.float32(float(arr.flat[idx]) + h)
    minus.flat[idx] = np.float32(float(arr.flat[idx]) - h)
    step = float(plus.flat[idx]) - float(minus.flat[idx])
    assert step > 0
    return (_loss_c(prob, target, **{name: plus}) - _loss_c(prob, target, **{name: minus})) / step


def _loss_c64(prob, target, name, arr64):
    # the torch mirror equals the C forward to ~1e-15 (checked below), and it
    # takes float64 fields directly, so it serves for the perturbed forward
    leaves = torch_ref.as_leaves(prob, requires_grad=False)
    leaves[name] = torch.tensor(arr64)
    cube = torch_ref.cube(prob, leaves).numpy()
    return oracle.loss(cube, target)


def test_torch_mirror_equals_c_forward():
    for mlp in (None, 4):
        prob = _problem(mlp)
        c = oracle.render(prob)
        t = torch_ref.cube(prob).detach().numpy()
        assert c.max() > 1.0
        np.testing.assert_allclose(t, c, rtol=0, atol=1e-12 * c.max())


@pytest.mark.parametrize("name", FIELDS)
def test_gradient_matches_central_differences(name):
    prob = _problem()
    target = _target(prob)
    L, grads = torch_ref.loss_and_grad(prob, target)
    assert L == pytest.approx(oracle.loss(oracle.render(prob), target), rel=1e-12)
    g = grads[name]
    rng = np.random.Generator(np.random.PCG64(32))
    cand = np.nonzero(np.abs(g).ravel() >= 1e-3 * np.abs(g).max())[0]
    assert len(cand) >= 4
    for idx in rng.choice(cand, size=min(6, len(cand)), replace=False):
        fd = _fd(prob, target, name, int(idx), 1e-4)
        assert g.flat[idx] == pytest.approx(fd, rel=1e-4, abs=1e-7 * np.abs(g).max()), (name, idx)


def test_scaling_identities():
    """n -> lambda n:  sum_ij dL/d ln n_ij = dL/d ln lambda;
    T -> lambda T:     sum_ij T_ij dL/dT_ij = dL/d ln lambda."""
    prob = _problem()
    target = _target(prob)
    _, grads = torch_ref.loss_and_grad(prob, target)
    h = 1e-5
    ln = prob.ln_nh2.astype(np.float64)
    dn = (_loss_c64(prob, target, "ln_nh2", ln + h) - _loss_c64(prob, target, "ln_nh2", ln - h)) / (2 * h)
    assert grads["ln_nh2"].sum() == pytest.approx(dn, rel=1e-6)
    t = prob.temp_k.astype(np.float64)
    dt = (_loss_c64(prob, target, "temp_k", t * math.exp(h)) -
          _loss_c64(prob, target, "temp_k", t * math.exp(-h))) / (2 * h)
    assert float(np.sum(t * grads["temp_k"])) == pytest.approx(dt, rel=1e-6)


def test_directional_derivative():
    """<grad L, d> equals the derivative of L along a random direction d."""
    prob = _problem()
    target = _target(prob)
    _, grads = torch_ref.loss_and_grad(prob, target)
    rng = np.random.Generator(np.random.PCG64(77))
    dirs = {k: rng.standard_normal(getattr(prob, k).shape) * s
            for k, s in zip(FIELDS, [0.1, 1.0, 0.05, 0.5, 0.5])}
    pred = sum(float(np.sum(grads[k] * dirs[k])) for k in FIELDS)
    h = 1e-5

    def loss_at(eps):
        leaves = torch_ref.as_leaves(prob, requires_grad=False)
        for k in FIELDS:
            leaves[k] = torch.tensor(getattr(prob, k).astype(np.float64) + eps * dirs[k])
        return oracle.loss(torch_ref.cube(prob, leaves).numpy(), target)

    fd = (loss_at(h) - loss_at(-h)) / (2 * h)
    assert pred == pytest.approx(fd, rel=1e-6)


def test_mlp_c_loops_match_torch_library():
    w = synth.make_mlp_weights(4)
    rng = np.random.Generator(np.random.PCG64(1))
    pts = rng.uniform(-0.05, 1.05, size=(16, 2))
    ref = torch_ref.mlp_eval(torch.tensor(w, dtype=torch.float64), torch.tensor(pts[:, 0]),
                             torch.tensor(pts[:, 1])).numpy()
    for k in range(len(pts)):
        np.testing.assert_allclose(oracle.mlp(w, pts[k, 0], pts[k, 1]), ref[k], rtol=1e-12, atol=1e-12)


def test_mlp_weight_gradient_matches_central_differences():
    prob = _problem(mlp_seed=4)
    target = _target(prob)
    _, grads = torch_ref.loss_and_grad(prob, target)
    g = grads["mlp_w"]
    rng = np.random.Generator(np.random.PCG64(33))
    cand = np.nonzero(np.abs(g) >= 1e-2 * np.abs(g).max())[0]
    for idx in rng.choice(cand, size=4, replace=False):
        fd = _fd(prob, target, "mlp_w", int(idx), 1e-4)
        assert g[idx] == pytest.approx(fd, rel=1e-4, abs=1e-7 * np.abs(g).max()), idx
