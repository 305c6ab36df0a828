"""GPU derived fields (rt_derive_fields and its adjoint) against the FP64
oracle of oracle/chain.py, and the temperature gradient through the derived
fields and the render against float64 autograd through both oracles.

Bars: FP32 forward within the stated absolute / relative tolerances of the
FP64 values; gradients ||dg||_2 <= 1e-3 ||g||_2 and every entry with
|g| >= 1e-2 max within 1e-3 of it (end to end: 2e-3, since the render there
reads the GPU's own FP32 fields)."""
import numpy as np
import pytest
import torch

import synth
from oracle import chain as OC
from oracle import torch_ref

pytestmark = pytest.mark.gpu

PHYS = dict(mstar_msun=2.0, mgas_msun=0.09, rc_au=150.0, gamma=1.0, mu=2.37, t_freeze_k=20.0, n_dissoc=1e21)


def _rt():
    import paper_2509_03623_amd as rt
    return rt


def _phys(rt, p=PHYS):
    return rt.DiskPhysics(p["mstar_msun"], p["mgas_msun"], p["rc_au"], p["gamma"], p["mu"], p["t_freeze_k"],
                          p["n_dissoc"])


def _temperature(grid, seed, noise=0.1):
    """Two-layer disk temperature on the node grid with lognormal noise."""
    nr, nz, r_min, r_max, zr_max = grid
    r, zr = OC.nodes(nr, nz, r_min, r_max, zr_max)
    R, ZR = np.meshgrid(r, zr, indexing="ij")
    T, _ = synth.disk._temperature(R, ZR * R, synth.disk.DiskParams())
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(T * np.exp(noise * rng.standard_normal(T.shape)), dtype=np.float32)


def _oracle(T32, grid, p=PHYS, requires_grad=False):
    T = torch.tensor(T32.astype(np.float64), requires_grad=requires_grad)
    return T, OC.derive_fields(T, grid, **p)


def _check_grad(name, got, ref, rel=1e-3):
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    l2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    big = np.abs(ref) >= 1e-2 * np.abs(ref).max()
    worst = (np.abs(got - ref)[big] / np.abs(ref)[big]).max()
    print(f"{name}: L2 rel {l2:.2e}; worst entry >= 1e-2 max {worst:.2e} (n={big.sum()})")
    assert l2 <= rel, (name, l2)
    assert worst <= rel, (name, worst)


@pytest.mark.parametrize("grid,seed", [((48, 24, 1.0, 600.0, 0.5), 1), ((256, 128, 1.0, 600.0, 0.5), 2),
                                       ((37, 19, 5.0, 300.0, 0.4), 3)])
def test_derived_fields_match_oracle(grid, seed):
    rt = _rt()
    print(f"[gpu] derived fields grid {grid} seed {seed}", flush=True)
    T32 = _temperature(grid, seed)
    _, ref = _oracle(T32, grid)
    got = rt.derive_fields(grid, torch.tensor(T32, device="cuda"), _phys(rt))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    r = {k: v.detach().numpy() for k, v in ref.items()}
    r_au = OC.nodes(*grid)[0]
    # ln n: absolute (ln n reaches -10^2 where the hydrostatic sum is large)
    assert np.abs(g["ln_nh2"] - r["ln_nh2"]).max() <= 1e-5 * np.abs(r["ln_nh2"]).max() + 2e-5
    assert np.abs(g["vphi_kms"] - r["vphi_kms"]).max() <= 1e-5 * np.abs(r["vphi_kms"]).max()
    for k in ("z_lo_au", "z_up_au"):
        assert np.all(np.abs(g[k] - r[k]) <= 1e-5 * r_au + 1e-6), k


# column lengths below one node per lane, two per lane, and a ragged three
# per lane (the top lanes of the wave own no nodes)
@pytest.mark.parametrize("grid,seed", [((48, 24, 1.0, 600.0, 0.5), 4), ((256, 128, 1.0, 600.0, 0.5), 6),
                                       ((40, 150, 5.0, 300.0, 0.4), 7)])
def test_derived_fields_adjoint_matches_oracle_autograd(grid, seed):
    rt = _rt()
    print(f"[gpu] derived-field adjoint grid {grid} seed {seed}", flush=True)
    T32 = _temperature(grid, seed)
    T, ref = _oracle(T32, grid, requires_grad=True)
    rng = np.random.Generator(np.random.PCG64(44))
    cot = {k: rng.standard_normal(tuple(v.shape)).astype(np.float32) for k, v in ref.items()}
    sum((ref[k] * torch.tensor(cot[k].astype(np.float64))).sum() for k in ref).backward(retain_graph=True)
    got = rt.derive_fields_adjoint(grid, torch.tensor(T32, device="cuda"), _phys(rt),
                                   {k: torch.tensor(v, device="cuda") for k, v in cot.items()})
    torch.cuda.synchronize()
    _check_grad("dT through derived fields", got.cpu().numpy(), T.grad.numpy())
    # the accumulating form adds the same product onto what the buffer holds
    base = torch.tensor(rng.standard_normal(T32.shape).astype(np.float32), device="cuda")
    acc = base.clone()
    rt.derive_fields_adjoint(grid, torch.tensor(T32, device="cuda"), _phys(rt),
                             {k: torch.tensor(v, device="cuda") for k, v in cot.items()}, add_to=acc)
    torch.cuda.synchronize()
    want = base.double() + got.double()
    assert float((acc.double() - want).abs().max()) <= 1e-6 * float(want.abs().max())
    # one output at a time (NULL cotangents for the others)
    for k in cot:
        T.grad = None
        (ref[k] * torch.tensor(cot[k].astype(np.float64))).sum().backward(retain_graph=True)
        one = rt.derive_fields_adjoint(grid, torch.tensor(T32, device="cuda"), _phys(rt),
                                       {k: torch.tensor(cot[k], device="cuda")})
        torch.cuda.synchronize()
        _check_grad(f"dT via {k}", one.cpu().numpy(), T.grad.numpy())


def test_temperature_gradient_through_derived_fields_and_render():
    """L = sum (cube - D)^2 with the fields derived from T: GPU dL/dT (render
    adjoint + derived-field adjoint, chained through the autograd functions)
    against float64 autograd through the oracle chain and the oracle render."""
    rt = _rt()
    prob = synth.small_problem(nx=20, ny=16, nch=10, nsamp=48, nr=40, nz=20, seed=9, dv=0.2)
    prob = prob.replace(intensity_scale=synth.disk.rj_kelvin_scale(prob.line))
    gs = prob.grid
    grid = (gs.nr, gs.nz, gs.r_min_au, gs.r_max_au, gs.zr_max)
    T32 = _temperature(grid, 5)
    # target: the oracle cube of a perturbed temperature
    with torch.no_grad():
        Tt, out_t = _oracle(T32 * np.float32(1.05), grid)
        lt = dict(ln_nh2=out_t["ln_nh2"], temp_k=Tt, vphi_kms=out_t["vphi_kms"], z_lo_au=out_t["z_lo_au"],
                  z_up_au=out_t["z_up_au"])
        target = torch_ref.cube(prob, lt).numpy()
    T, out = _oracle(T32, grid, requires_grad=True)
    leaves = dict(ln_nh2=out["ln_nh2"], temp_k=T, vphi_kms=out["vphi_kms"], z_lo_au=out["z_lo_au"],
                  z_up_au=out["z_up_au"])
    cube = torch_ref.cube(prob, leaves)
    ((cube - torch.tensor(target)) ** 2).sum().backward()
    ref = T.grad.numpy()
    # GPU: fields from rt.DeriveFields, cube from rt.Render, torch autograd chains the two adjoints
    sc = rt.scene_from_problem(prob)
    Tg = torch.tensor(T32, device="cuda", requires_grad=True)
    ln_n, vphi, zlo, zup = rt.DeriveFields.apply(grid, _phys(rt), Tg)
    c = rt.render_differentiable(sc, ln_nh2=ln_n, temp_k=Tg, vphi_kms=vphi, z_lo_au=zlo, z_up_au=zup)
    ((c - torch.tensor(target, dtype=torch.float32, device="cuda")) ** 2).sum().backward()
    torch.cuda.synchronize()
    _check_grad("end-to-end dL/dT", Tg.grad.cpu().numpy(), ref, rel=2e-3)


@pytest.mark.parametrize("grid,args", [((64, 48, 1.0, 600.0, 0.5), (30.0, 60.0, -0.5, 100.0, 70.0, 2.0)),
                                       ((33, 21, 5.0, 300.0, 0.4), (18.0, 45.0, -0.3, 150.0, 40.0, 1.0))])
def test_parametric_temperature_matches_oracle(grid, args):
    rt = _rt()
    T = rt.parametric_temperature(grid, *args)
    torch.cuda.synchronize()
    ref = OC.parametric_temperature(*grid, *args)
    np.testing.assert_allclose(T.cpu().numpy(), ref, rtol=2e-6)
