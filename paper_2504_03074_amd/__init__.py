"""MI355X-native WaveHoltz: explicit leapfrog + fused trapezoid time filter,
fixed-point and GMRES outer solvers, hand-written HIP kernels for gfx950.

The compute path is the C ABI in ``include/wh.h`` (``libwh.so``); ``wh``
is its Python binding and ``Solver`` a convenience object over torch tensors.
"""
from .wh import (  # noqa: F401
    Batch, Solver, WhError, library, wh_compute_time_params, wh_version,
    WH_FP64, WH_FP32_STATE, WH_SOLVER_FPI, WH_SOLVER_GMRES, WH_SOLVER_CG,
)

__all__ = ["Batch", "Solver", "WhError", "library", "wh_compute_time_params", "wh_version",
           "WH_FP64", "WH_FP32_STATE", "WH_SOLVER_FPI", "WH_SOLVER_GMRES", "WH_SOLVER_CG"]
