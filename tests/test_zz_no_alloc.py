"""rt_render_cube_l2_adjoint_noalloc (no allocation; scratch in one fixed
device array) against rt_render_cube_l2_adjoint on the same inputs: two calls
in a row (the second smaller), an image whose scratch needs several bands of
the fixed array, and the size check.

Bars: the cube within 1e-6 of the allocating call's peak (same kernels, so
in practice identical), the loss within 1e-9 relative, each gradient block
within 1e-5 of its largest entry (the accumulation order of the atomics
differs), and the gradients against the FP64 oracle at the adjoint's bar
(L2 <= 1e-3 per block)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import torch_ref

pytestmark = pytest.mark.gpu

BLOCKS = ("ln_nh2", "temp_k", "vphi_kms", "z_lo_au", "z_up_au")


def _rt():
    import paper_2509_03623_amd as rt
    return rt


def kscale(prob):
    return prob.replace(intensity_scale=synth.disk.rj_kelvin_scale(prob.line))


def run_both(prob, target):
    rt = _rt()
    sc = rt.scene_from_problem(prob)
    tgt = torch.as_tensor(np.ascontiguousarray(target, np.float32), device="cuda")
    cube_a, loss_a, g_a = rt.render_l2_adjoint(sc, tgt, want=BLOCKS)
    # outputs allocated before the call, so only the library call runs
    cube_b = torch.full_like(cube_a, float("nan"))
    loss_b = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    g_b = {k: torch.full_like(v, float("nan")) for k, v in g_a.items()}
    torch.cuda.synchronize()
    print(f"[gpu] noalloc fused adjoint {sc.nx}x{sc.ny}x{sc.nch} ns={sc.nsamp} grid {sc.nr}x{sc.nz}", flush=True)
    rt.render_l2_adjoint(sc, tgt, cube_out=cube_b, loss_out=loss_b, grads_out=g_b, noalloc=True)
    torch.cuda.synchronize()
    return (cube_a.cpu().numpy(), float(loss_a.item()), {k: v.cpu().numpy().astype(np.float64) for k, v in g_a.items()},
            cube_b.cpu().numpy(), float(loss_b.item()), {k: v.cpu().numpy().astype(np.float64) for k, v in g_b.items()})


def compare(res):
    cube_a, loss_a, g_a, cube_b, loss_b, g_b = res
    scale = float(np.abs(cube_a).max())
    assert scale > 0
    assert float(np.abs(cube_b - cube_a).max()) <= 1e-6 * scale
    assert loss_b == pytest.approx(loss_a, rel=1e-9)
    for k in BLOCKS:
        s = float(np.abs(g_a[k]).max())
        assert s > 0, k
        d = float(np.abs(g_b[k] - g_a[k]).max())
        print(f"{k}: max |noalloc - alloc| / max {d / s:.2e}")
        assert d <= 1e-5 * s, k


def test_two_calls_in_a_row_second_smaller():
    big = kscale(synth.small_problem(nx=40, ny=36, nch=24, nsamp=96, nr=64, nz=32, seed=21, dv=0.1))
    small = kscale(synth.small_problem(nx=19, ny=17, nch=13, nsamp=61, nr=40, nz=20, seed=8, dv=0.2))
    for prob in (big, small):
        target = synth.disk.add_noise(oracle.render(synth.perturb_surfaces(prob, seed=30)), 0.05, seed=31)
        res = run_both(prob, target)
        compare(res)
        _, oref = torch_ref.loss_and_grad(prob, target)
        for k in BLOCKS:
            r, g = oref[k].ravel(), res[5][k].ravel()
            l2 = float(np.linalg.norm(g - r) / np.linalg.norm(r))
            print(f"{k}: noalloc vs oracle L2 rel {l2:.2e}")
            assert l2 <= 1e-3, k


def test_image_in_bands_of_the_fixed_array():
    """512 x 512 x 64 x 512: one row of scratch is 8.4 MB, so the fixed array
    takes the image in ~18 bands of rows."""
    prob = kscale(synth.config2(2001))
    rt = _rt()
    sc = rt.scene_from_problem(prob)
    target = rt.render(sc.replace(z_up_au=sc.z_up_au * 1.05)).cpu().numpy()
    compare(run_both(prob, target))


def test_too_big_for_the_fixed_array():
    rt = _rt()
    from paper_2509_03623_amd import _lib as L
    prob = synth.small_problem(nx=2048, ny=1, nch=64, nsamp=4096, nr=32, nz=16)
    sc = rt.scene_from_problem(prob)
    tgt = torch.zeros(sc.nch, sc.ny, sc.nx, device="cuda")
    with pytest.raises(rt.RtError) as ei:
        rt.render_l2_adjoint(sc, tgt, want=("temp_k",), noalloc=True)
    assert ei.value.status == L.RT_ETOOBIG
    assert int(L.lib().rt_noalloc_scratch_bytes()) == 256 << 20
