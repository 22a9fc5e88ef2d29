"""MI355X-native solver for the Gross-Pitaevskii equation on selectively
sampled semi-structured grids (arXiv:2603.05447).

The compute path is libgpe.so (HIP for gfx950, C ABI in include/gpe.h);
this package is its thin Python binding.
"""
from ._lib import GPEError, load as load_library, LIB_PATH
from ._lib import (GPE_C128, GPE_C64, GPE_MODE_ITP, GPE_MODE_RT, GPE_MODE_ADJ, GPE_MODE_RT_RKHE3,
                   GPE_MODE_RT_RKCK, GPE_MODE_ITP_REAL, GPE_POT_STATIC, GPE_POT_RF_RAMP, GPE_POT_LERP, GPE_POT_SHELL_RAMP,
                   GPE_RK4, GPE_RKHE3, GPE_RKCK, GPE_MAX_KNOTS)
from .api import (Grid, Batch, Potential, FidelityGrad, BatchFidelityGrad, KernelTimer, config_count,
                  config_describe, make_params, staged_ramp, stream_copy, INTEGRATORS)

__all__ = ["GPEError", "load_library", "LIB_PATH", "Grid", "Batch", "Potential", "FidelityGrad", "BatchFidelityGrad",
           "KernelTimer",
           "config_count", "config_describe", "make_params", "staged_ramp", "stream_copy", "INTEGRATORS", "GPE_C128", "GPE_C64",
           "GPE_MODE_ITP", "GPE_MODE_RT", "GPE_MODE_ADJ", "GPE_MODE_RT_RKHE3", "GPE_MODE_RT_RKCK",
           "GPE_MODE_ITP_REAL", "GPE_POT_STATIC", "GPE_POT_RF_RAMP", "GPE_POT_LERP", "GPE_POT_SHELL_RAMP", "GPE_RK4", "GPE_RKHE3",
           "GPE_RKCK", "GPE_MAX_KNOTS"]
