"""MI355X-native line radiative-transfer ray march (HIP, gfx950).

The renderer lives in librtcube.so behind the C ABI of include/rtcube.h;
this package is its thin Python binding (ctypes + torch for device memory
and streams).
"""
from ._lib import RtError, lib, RT_MLP_BF16, RT_MLP_FP32, RT_MLP_PARAMS  # noqa: F401
from .render import (  # noqa: F401
    Scene, scene_from_problem, render, render_adjoint, render_l2_adjoint, Render, render_differentiable,
    set_option, get_option, constants, DiskPhysics, derive_fields, derive_fields_adjoint, DeriveFields, parametric_temperature,
    Scene3d, pack_fields3d, scene3d_from_problem, render3d, beam_convolve, BeamConvolve,
)
from .server import Server  # noqa: F401
from .fit import (  # noqa: F401
    neural_temperature, neural_temperature_adjoint, NeuralTemperature, Adam, poly_lr, fit_step,
)
