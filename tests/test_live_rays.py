"""The ray-sample count of the measurements comes from the library's census
(rt_render_census / rt_render_census_3d: the march's own ray set-up): its
mask marks exactly the pixels whose chord through the bounding volume is
non-empty in the FP64 oracle (a ray outside has no samples and zero
intensity), and its thin-sample count is exact on slabs whose samples are
all thin or thick by construction."""
import numpy as np
import pytest

import oracle
import synth
from synth import disk3d as S3

pytestmark = pytest.mark.gpu


def _chords(prob, dump):
    ny, nx = prob.camera.ny, prob.camera.nx
    return np.array([[dump(prob, p, q)[3][2] > 0.0 for p in range(nx)] for q in range(ny)])


@pytest.mark.parametrize("incl,pa", [(0.0, 0.0), (35.0, 20.0), (62.0, -110.0), (90.0, 45.0)])
def test_axisymmetric_live_mask_matches_oracle_chords(incl, pa):
    import paper_2509_03623_amd as rt
    prob = synth.small_problem(nx=41, ny=33, nch=2, nsamp=8, nr=24, nz=12, seed=7, incl=incl)
    prob.camera.pa_deg = pa
    prob.camera.fov_au *= 1.4          # leave rays outside the cylinder in every corner
    sc = rt.scene_from_problem(prob)
    want = _chords(prob, oracle.ray_dump)
    print(f"[gpu] census incl={incl} pa={pa}", flush=True)
    got = sc.census()
    assert 0 < want.sum() < want.size
    assert np.array_equal(got["mask"], want)
    assert got["rays"] == int(want.sum())
    assert sc.ray_samples == int(want.sum()) * sc.nch * sc.nsamp


def test_spherical_live_mask_matches_oracle_chords():
    import paper_2509_03623_amd as rt
    grid = S3.Grid3Spec(16, 8, 8)
    prob = S3.uniform_problem3(grid, nx=37, ny=29, nch=2, nsamp=8, incl=50.0, pa=30.0, fov_au=3.0 * grid.r_max_au)
    want = _chords(prob, oracle.ray_dump3)
    sc = rt.scene3d_from_problem(prob)
    print("[gpu] census 3-D", flush=True)
    got = sc.census()
    assert 0 < want.sum() < want.size
    assert np.array_equal(got["mask"], want)
    assert sc.ray_samples == int(want.sum()) * sc.nch * sc.nsamp
    # uniform fields: every sample inside the grid's fade has opacity, none beyond it
    n = got["pixel_samples"]
    assert 0 < got["emitting_pixel_samples"] == got["shaded_pixel_samples"] < n
    assert got["thin_pixel_samples"] >= n - got["emitting_pixel_samples"]


@pytest.mark.parametrize("x_co", [1e-2, 1e-12])
def test_thin_sample_count_on_slabs(x_co):
    """Face-on slabs with a hard mask, so every sample's line-centre depth is
    either 0 (outside the layer, or beyond the grid's top z/r row near the
    axis) or far from the threshold: the census's thin count equals the
    number of samples whose depth in the oracle's central channel (v_los = 0
    face-on) is below 1/32 in natural units, its count of samples with any
    opacity the number whose depth there is not vanishing (the FP64 oracle
    also keeps a few below 1e-45, which FP32 holds as 0), and with a
    negligible abundance every sample is thin."""
    import paper_2509_03623_amd as rt
    prob = synth.slab_problem(nsamp=128, m=24, x_co=x_co, nx=8, ny=8, nch=3)
    sc = rt.scene_from_problem(prob)
    print(f"[gpu] census slab x_co={x_co:g}", flush=True)
    got = sc.census()
    rays = int(got["mask"].sum())
    assert rays > 0 and got["pixel_samples"] == rays * prob.nsamp
    want = 0
    depths = []
    for q in range(prob.camera.ny):
        for p in range(prob.camera.nx):
            _, _, dt, ch = oracle.ray_dump(prob, p, q)
            if ch[2] > 0.0:
                want += int((dt[:, 1] < 1.0 / 32.0).sum())
                depths.append(dt[:, 1])
    depths = np.concatenate(depths)
    emit = int((depths > 1e-30 * depths.max()).sum())
    print(f"thin pixel-samples: census {got['thin_pixel_samples']}, oracle {want} of {got['pixel_samples']}; "
          f"with opacity: census {got['emitting_pixel_samples']}, oracle {emit}")
    assert got["thin_pixel_samples"] == want
    # with opacity: the depths split into those the FP32 march holds (here
    # above 1e-10 in natural units) and a handful of vanishing ones (below
    # 1e-45, zero in FP32, some even in FP64), so the count above 1e-30 of
    # the largest is the march's count of samples with K > 0
    assert depths[(depths > 0.0) & (depths <= 1e-30 * depths.max())].max(initial=0.0) < 1e-40
    assert got["emitting_pixel_samples"] == emit
    # samples with opacity lie inside the grid's edge taper, which the march shades
    assert emit <= got["shaded_pixel_samples"] <= got["pixel_samples"]
    if x_co < 1e-10:
        assert want == got["pixel_samples"]
    else:
        assert 0 < want < got["pixel_samples"]
