"""Neural CO layer (network evaluated at every pixel-sample on the matrix
cores) vs the FP64 oracle.

Bars: FP32 path -- cube max |dI| <= 1e-5 peak is the FP32 norm; gradients
L2 <= 1e-3 per block.  BF16 path -- cube relative L2 <= 1e-2 and gradient
cosine >= 0.99 against FP64."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import torch_ref

pytestmark = pytest.mark.gpu


def _rt():
    import paper_2509_03623_amd as rt
    return rt


def mlp_problem(**kw):
    args = dict(nx=24, ny=20, nch=12, nsamp=64, nr=48, nz=24, seed=5, dv=0.2, mlp_seed=4)
    args.update(kw)
    prob = synth.small_problem(**args)
    return prob.replace(intensity_scale=synth.disk.rj_kelvin_scale(prob.line))


def gpu_cube(prob, precision):
    rt = _rt()
    print(f"[gpu] neural render {prob.camera.nx}x{prob.camera.ny}x{prob.nch} ns={prob.nsamp} prec={precision}",
          flush=True)
    sc = rt.scene_from_problem(prob, mlp_precision=precision)
    cube = rt.render(sc)
    torch.cuda.synchronize()
    return cube.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("incl", [45.0, 62.0])
def test_fp32_network_forward(incl):
    rt = _rt()
    prob = mlp_problem(incl=incl)
    ref = oracle.render(prob)
    got = gpu_cube(prob, rt.RT_MLP_FP32)
    err = float(np.abs(got - ref).max() / ref.max())
    l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"fp32 network: max|dI|/peak {err:.2e}, rel L2 {l2:.2e}")
    assert ref.max() > 1.0
    assert err <= 1e-5


def test_bf16_network_forward():
    rt = _rt()
    prob = mlp_problem()
    ref = oracle.render(prob)
    got = gpu_cube(prob, rt.RT_MLP_BF16)
    l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"bf16 network: rel L2 {l2:.2e}, max|dI|/peak {np.abs(got - ref).max() / ref.max():.2e}")
    assert l2 <= 1e-2


def _grads(prob, precision, cotangent):
    rt = _rt()
    sc = rt.scene_from_problem(prob, mlp_precision=precision)
    dl = torch.as_tensor(np.ascontiguousarray(cotangent, np.float32), device="cuda")
    g = rt.render_adjoint(sc, dl, want=("ln_nh2", "temp_k", "vphi_kms", "mlp_w"))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}


def _cos(a, b):
    a, b = a.ravel(), b.ravel()
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_network_gradients_fp32_and_bf16():
    rt = _rt()
    prob = mlp_problem(nx=20, ny=16, nch=10, nsamp=48)
    tgt = synth.disk.add_noise(oracle.render(prob.replace(mlp_w=synth.make_mlp_weights(99))), 0.05, seed=31)
    _, ref = torch_ref.loss_and_grad(prob, tgt)
    cot = 2.0 * (oracle.render(prob) - tgt)
    g32 = _grads(prob, rt.RT_MLP_FP32, cot)
    g16 = _grads(prob, rt.RT_MLP_BF16, cot)
    for k in ("ln_nh2", "temp_k", "vphi_kms", "mlp_w"):
        l2 = float(np.linalg.norm(g32[k] - ref[k]) / np.linalg.norm(ref[k]))
        c16 = _cos(g16[k], ref[k])
        print(f"{k}: fp32 L2 rel {l2:.2e}; bf16 cosine {c16:.5f}")
        assert l2 <= 1e-3, (k, l2)
        assert c16 >= 0.99, (k, c16)
    assert np.abs(g32["mlp_w"]).max() > 0


def test_network_surface_gradients_are_zero():
    """With the network the grid surfaces are not used: their gradients are 0."""
    rt = _rt()
    prob = mlp_problem(nx=12, ny=10, nch=6, nsamp=32)
    sc = rt.scene_from_problem(prob, mlp_precision=rt.RT_MLP_BF16)
    cube = rt.render(sc)
    g = rt.render_adjoint(sc, torch.ones_like(cube), want=("z_lo_au", "z_up_au"))
    torch.cuda.synchronize()
    assert float(g["z_lo_au"].abs().max()) == 0.0 and float(g["z_up_au"].abs().max()) == 0.0


def test_network_adjoint_in_row_bands():
    """The network adjoint differentiated in bands of one row equals the
    single-pass adjoint (network outputs indexed image-wide in every band)."""
    rt = _rt()
    from paper_2509_03623_amd import _lib as L
    prob = mlp_problem(nx=14, ny=11, nch=9, nsamp=40)
    cot = np.random.Generator(np.random.PCG64(7)).standard_normal((9, 11, 14))
    whole = _grads(prob, rt.RT_MLP_FP32, cot)
    rt.set_option(L.RT_OPT_ADJ_SCRATCH_CAP, 1)
    try:
        banded = _grads(prob, rt.RT_MLP_FP32, cot)
    finally:
        rt.set_option(L.RT_OPT_ADJ_SCRATCH_CAP, 0)
    for k in whole:
        scale = np.abs(whole[k]).max()
        assert scale > 0, k
        assert np.abs(banded[k] - whole[k]).max() <= 1e-5 * scale, k


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_size_network_render_sampled_pixels(precision):
    """The 256 x 256 x 32-channel x 256-sample network render in the launch
    configuration the benchmark times, checked on 96 seeded pixels against
    the FP64 oracle (network evaluated in float64 at every sample): the FP32
    path at the FP32 bar (max |dI| <= 1e-5 peak of the sample), the BF16
    path at relative L2 <= 1e-2."""
    rt = _rt()
    prob = synth.config4()
    prec = rt.RT_MLP_FP32 if precision == "fp32" else rt.RT_MLP_BF16
    print(f"[gpu] full-size network render prec={precision}", flush=True)
    sc = rt.scene_from_problem(prob, mlp_precision=prec)
    cube = rt.render(sc)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(44))
    # pixels over the disk (the inner two thirds of the image) plus a few anywhere
    px = np.concatenate([rng.integers(43, 213, 80), rng.integers(0, 256, 16)])
    py = np.concatenate([rng.integers(43, 213, 80), rng.integers(0, 256, 16)])
    ref = oracle.render_pixels(prob, px, py)
    got = cube.cpu().numpy().astype(np.float64)[:, py, px].T
    assert ref.max() > 0
    err = float(np.abs(got - ref).max() / ref.max())
    l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"{precision}: max|dI|/peak {err:.2e}, rel L2 {l2:.2e}")
    if precision == "fp32":
        assert err <= 1e-5
    else:
        assert l2 <= 1e-2


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_network_adjoint_returns_the_forward_cube(precision):
    """The cube the network adjoint writes (cube_out) is the render's: one
    call gives the forward and the gradients."""
    rt = _rt()
    prec = rt.RT_MLP_FP32 if precision == "fp32" else rt.RT_MLP_BF16
    prob = mlp_problem(nx=22, ny=17, nch=11, nsamp=56)
    print(f"[gpu] neural adjoint cube_out {precision}", flush=True)
    sc = rt.scene_from_problem(prob, mlp_precision=prec)
    cube = rt.render(sc)
    cube2 = torch.full_like(cube, float("nan"))
    rt.render_adjoint(sc, torch.ones_like(cube), want=("temp_k", "mlp_w"), cube_out=cube2)
    torch.cuda.synchronize()
    a, b = cube.cpu().numpy(), cube2.cpu().numpy()
    assert np.isfinite(b).all()
    assert a.max() > 1.0
    assert np.abs(a - b).max() <= 1e-6 * np.abs(a).max()
