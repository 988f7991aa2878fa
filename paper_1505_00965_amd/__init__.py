"""MI355X-native multilevel Monte Carlo level sampler (HIP, gfx950).

The computation lives in libmlmc.so (include/mlmc.h); this package is its
ctypes binding plus the named workload presets.
"""
from . import mlmc  # noqa: F401
from .mlmc import Context, MLMCError, model, payoff  # noqa: F401
