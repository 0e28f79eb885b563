"""MI355X (gfx950) batched per-level sample solve of the inexact MLMC method.

The compute path is the HIP library libmlmc.so (C ABI in include/mlmc.h);
``mlmc`` is its thin Python binding.
"""
from .mlmc import (Config, MLMC, MLMCError, MLMCQoI, LevelPlan, DTYPES, SOLVERS,  # noqa: F401
                   EXPORTS, LIB_PATH, load_library)
