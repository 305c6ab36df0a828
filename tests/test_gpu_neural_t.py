"""GPU neural temperature field, its adjoint and the Adam step against the
FP64 oracle (oracle/neural_t.py); the weight gradient through the network,
the derived fields and the render against float64 autograd through the three
oracles; and a short fit that lowers chi^2.

Bars: T within 1e-4 relative of FP64; gradients ||dg||_2 <= 1e-3 ||g||_2
(end to end 2e-3: the GPU render reads its own FP32 fields) and every entry
with |g| >= 1e-2 max within 1e-3 (end to end 5e-3)."""
import numpy as np
import pytest
import torch

import synth
from oracle import chain as OC
from oracle import neural_t as ON
from oracle import torch_ref

pytestmark = pytest.mark.gpu

PHYS = dict(mstar_msun=2.0, mgas_msun=0.09, rc_au=150.0, gamma=1.0, mu=2.37, t_freeze_k=20.0, n_dissoc=1e21)


def _rt():
    import paper_2509_03623_amd as rt
    return rt


def _phys(rt):
    p = PHYS
    return rt.DiskPhysics(p["mstar_msun"], p["mgas_msun"], p["rc_au"], p["gamma"], p["mu"], p["t_freeze_k"],
                          p["n_dissoc"])


def _check_grad(name, got, ref, rel=1e-3, rel_entry=1e-3):
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    l2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    big = np.abs(ref) >= 1e-2 * np.abs(ref).max()
    worst = (np.abs(got - ref)[big] / np.abs(ref)[big]).max()
    print(f"{name}: L2 rel {l2:.2e}; worst entry >= 1e-2 max {worst:.2e} (n={big.sum()})")
    assert l2 <= rel, (name, l2)
    assert worst <= rel_entry, (name, worst)


@pytest.mark.parametrize("grid", [(48, 24, 1.0, 600.0, 0.5), (256, 128, 1.0, 600.0, 0.5), (37, 19, 5.0, 300.0, 0.4)])
def test_neural_temperature_matches_oracle(grid):
    rt = _rt()
    print(f"[gpu] neural temperature grid {grid}", flush=True)
    w = synth.mlp.make_neural_t_weights(7)
    ref = ON.temperature(torch.tensor(w.astype(np.float64)), grid[0], grid[1]).numpy()
    got = rt.neural_temperature(grid, torch.tensor(w, device="cuda"))
    torch.cuda.synchronize()
    np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-4)


def test_neural_temperature_adjoint_matches_autograd():
    rt = _rt()
    grid = (48, 24, 1.0, 600.0, 0.5)
    w = synth.mlp.make_neural_t_weights(8)
    wt = torch.tensor(w.astype(np.float64), requires_grad=True)
    c = np.random.default_rng(3).standard_normal((48, 24)).astype(np.float32)
    (ON.temperature(wt, 48, 24) * torch.tensor(c.astype(np.float64))).sum().backward()
    got = rt.neural_temperature_adjoint(grid, torch.tensor(w, device="cuda"), torch.tensor(c, device="cuda"))
    torch.cuda.synchronize()
    _check_grad("dW", got.cpu().numpy(), wt.grad.numpy())


def test_adam_steps_match_oracle():
    rt = _rt()
    rng = np.random.default_rng(4)
    p0 = rng.standard_normal(1000).astype(np.float32)
    p = torch.tensor(p0, device="cuda")
    opt = rt.Adam(p)
    P, M, V = p0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for t, lr in enumerate((1e-2, 5e-3, 2e-3, 1e-3), start=1):
        g = rng.standard_normal(1000).astype(np.float32)
        opt.step(torch.tensor(g, device="cuda"), lr, grad_scale=0.5)
        P, M, V = ON.adam(P, M, V, 0.5 * g.astype(np.float64), t, lr)
    torch.cuda.synchronize()
    np.testing.assert_allclose(p.cpu().numpy(), P, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(opt.m.cpu().numpy(), M, rtol=1e-5, atol=1e-7)


def _problem():
    prob = synth.small_problem(nx=18, ny=14, nch=10, nsamp=40, nr=40, nz=20, seed=12, dv=0.25)
    return prob.replace(intensity_scale=synth.disk.rj_kelvin_scale(prob.line))


def test_weight_gradient_through_fields_and_render():
    """chi^2 of the render of the fields derived from the network's T: GPU
    dchi^2/dweights (autograd functions over the library's adjoints) against
    float64 autograd through the network, derived-field and render oracles."""
    rt = _rt()
    prob = _problem()
    gs = prob.grid
    grid = (gs.nr, gs.nz, gs.r_min_au, gs.r_max_au, gs.zr_max)
    w = synth.mlp.make_neural_t_weights(9)
    sigma = 0.05
    with torch.no_grad():
        T0 = torch.tensor(prob.temp_k.astype(np.float64))
        o0 = OC.derive_fields(T0, grid, **PHYS)
        target = torch_ref.cube(prob, dict(ln_nh2=o0["ln_nh2"], temp_k=T0, vphi_kms=o0["vphi_kms"],
                                           z_lo_au=o0["z_lo_au"], z_up_au=o0["z_up_au"])).numpy()
    wt = torch.tensor(w.astype(np.float64), requires_grad=True)
    T = ON.temperature(wt, gs.nr, gs.nz)
    o = OC.derive_fields(T, grid, **PHYS)
    cube = torch_ref.cube(prob, dict(ln_nh2=o["ln_nh2"], temp_k=T, vphi_kms=o["vphi_kms"], z_lo_au=o["z_lo_au"],
                                     z_up_au=o["z_up_au"]))
    (((cube - torch.tensor(target)) / sigma) ** 2).sum().backward()
    sc = rt.scene_from_problem(prob)
    wg = torch.tensor(w, device="cuda", requires_grad=True)
    Tg = rt.NeuralTemperature.apply(grid, wg)
    ln_n, vphi, zlo, zup = rt.DeriveFields.apply(grid, _phys(rt), Tg)
    c = rt.render_differentiable(sc, ln_nh2=ln_n, temp_k=Tg, vphi_kms=vphi, z_lo_au=zlo, z_up_au=zup)
    (((c - torch.tensor(target, dtype=torch.float32, device="cuda")) / sigma) ** 2).sum().backward()
    torch.cuda.synchronize()
    _check_grad("end-to-end dchi2/dW", wg.grad.cpu().numpy(), wt.grad.numpy(), rel=2e-3, rel_entry=5e-3)


def test_fit_lowers_chi2():
    """The paper's loop on a small disk: random batches of half the channels,
    Adam with a decaying learning rate; chi^2 over all channels must fall to
    a fraction of its start."""
    rt = _rt()
    prob = synth.small_problem(nx=24, ny=20, nch=16, nsamp=48, nr=40, nz=20, seed=13, dv=0.2)
    prob = prob.replace(intensity_scale=synth.disk.rj_kelvin_scale(prob.line))
    gs = prob.grid
    grid = (gs.nr, gs.nz, gs.r_min_au, gs.r_max_au, gs.zr_max)
    sc = rt.scene_from_problem(prob)
    phys = _phys(rt)
    T_true = torch.tensor(prob.temp_k, device="cuda")
    target = rt.render(sc.replace(temp_k=T_true, **rt.derive_fields(grid, T_true, phys)))
    sigma = 0.015 * float(target.abs().max())
    w = torch.tensor(synth.mlp.make_neural_t_weights(10), device="cuda")
    opt = rt.Adam(w)
    rng = np.random.Generator(np.random.PCG64(14))
    all_ch = np.arange(sc.nch)

    def chi2_all():
        T = rt.neural_temperature(grid, w)
        c = rt.render(sc.replace(temp_k=T, **rt.derive_fields(grid, T, phys)))
        return float((((c - target) / sigma) ** 2).sum())

    start = chi2_all()
    steps = 60
    for t in range(steps):
        ch = np.sort(rng.choice(all_ch, size=sc.nch // 2, replace=False))
        rt.fit_step(sc, grid, phys, opt, target, ch, sigma, rt.poly_lr(t, steps, 3e-3, 3e-4))
    end = chi2_all()
    print(f"chi2 over all channels: start {start:.4g}, after {steps} steps {end:.4g}")
    assert np.isfinite(end) and end < 0.3 * start
