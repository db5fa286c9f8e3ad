"""MI355X-native adaptive fast multipole Poisson solver for AMR hierarchies.

The solver itself is the HIP library ``libafmm.so`` (C ABI in include/afmm.h);
this package is its thin Python binding.
"""
from ._lib import AFMM_ALL_LEVELS, AfmmError, lib
from .afmm import AFMMSolve, Batch, Plan, hierarchy_check, make_options, release_cached_memory, solve

__all__ = ["AFMM_ALL_LEVELS", "AfmmError", "AFMMSolve", "Batch", "Plan", "hierarchy_check", "lib", "make_options", "release_cached_memory", "solve"]
