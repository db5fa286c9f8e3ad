"""Seeded synthetic AMR hierarchies and cell masses.

This package feeds both the HIP solver and the CPU oracle.  It holds no part of
the multipole method itself: it only builds graded octree hierarchies (levels,
cell coordinates, refinement flags) and midpoint-rule cell masses from analytic
densities, with seeded noise.
"""
from .hierarchy import (
    Hierarchy,
    unigrid,
    build_graded,
    shuffle_order,
    mirror_x,
)
from .density import plummer, gaussian_clumps, uniform_sphere, cell_masses
from . import configs

__all__ = [
    "Hierarchy",
    "unigrid",
    "build_graded",
    "shuffle_order",
    "mirror_x",
    "plummer",
    "gaussian_clumps",
    "uniform_sphere",
    "cell_masses",
    "configs",
]
