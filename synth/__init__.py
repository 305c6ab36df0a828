"""Seeded synthetic inputs for the line radiative-transfer ray march.

This package only builds input arrays (disk fields on the (r, z/r) grid,
camera, channel list, line data, MLP weights, request traces).  It holds none
of the ray-march arithmetic: the oracle and the GPU library both consume what
it produces, and neither is imported here.
"""
from .disk import (  # noqa: F401
    GridSpec, DiskParams, Camera, LineData, Problem,
    co21_line, make_disk, make_problem,
    config1, config2, config3, config3_target_disk, config4, small_problem,
    slab_problem, ring_problem, perturb_surfaces,
)
from .mlp import mlp_param_count, make_mlp_weights, MLP_WIDTH, MLP_DEPTH, MLP_NFREQ  # noqa: F401
from .trace import make_trace  # noqa: F401
from . import disk3d  # noqa: F401
