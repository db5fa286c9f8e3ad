"""Analytic densities and midpoint-rule cell masses with seeded noise.

Cell masses are m = rho(x_c) h^3 (1 + noise * u), u ~ U[-1, 1) drawn from
NumPy's PCG64(seed) in flat level-major caller order.  Refined cells get the
same formula: the solver ignores their entries, which lets tests check that.
"""
from __future__ import annotations

from typing import Callable, Sequence

import numpy as np

from .hierarchy import Hierarchy


def plummer(total_mass: float = 1.0, a: float = 0.1, centre=(0.5, 0.5, 0.5)) -> Callable:
    """Plummer sphere rho(r) = 3M / (4 pi a^3) (1 + r^2/a^2)^(-5/2)."""
    c = np.asarray(centre, dtype=np.float64)
    rho0 = 3.0 * total_mass / (4.0 * np.pi * a ** 3)

    def rho(x):
        x = np.asarray(x, dtype=np.float64)
        d = x[..., 0] - c[0]
        r2 = d * d
        d = x[..., 1] - c[1]
        r2 += d * d
        d = x[..., 2] - c[2]
        r2 += d * d
        return rho0 * (1.0 + r2 / (a * a)) ** (-2.5)

    return rho


def gaussian_clumps(centres: np.ndarray, sigmas: Sequence[float], masses: Sequence[float]) -> Callable:
    """Sum of isotropic Gaussians, each normalised to its mass."""
    centres = np.asarray(centres, dtype=np.float64)
    sig = np.asarray(sigmas, dtype=np.float64)
    ms = np.asarray(masses, dtype=np.float64)
    norm = ms / ((2.0 * np.pi) ** 1.5 * sig ** 3)

    def rho(x):
        x = np.asarray(x, dtype=np.float64)
        x0, x1, x2 = x[..., 0], x[..., 1], x[..., 2]
        out = np.zeros(x.shape[:-1], dtype=np.float64)
        for c, s, n in zip(centres, sig, norm):
            d = x0 - c[0]
            r2 = d * d
            d = x1 - c[1]
            r2 += d * d
            d = x2 - c[2]
            r2 += d * d
            out += n * np.exp(-0.5 * r2 / (s * s))
        return out

    return rho


def uniform_sphere(radius: float, centre, rho0: float = 1.0) -> Callable:
    c = np.asarray(centre, dtype=np.float64)

    def rho(x):
        r2 = np.sum((np.asarray(x, dtype=np.float64) - c) ** 2, axis=-1)
        return np.where(r2 <= radius * radius, rho0, 0.0)

    return rho


def sum_density(*fns: Callable) -> Callable:
    def rho(x):
        out = fns[0](x)
        for f in fns[1:]:
            out = out + f(x)
        return out

    return rho


def cell_masses(h: Hierarchy, rho: Callable, noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Flat level-major masses: midpoint rule times (1 + noise * U[-1, 1))."""
    out = []
    for i, a in enumerate(h.ijk):
        hl = h.cell_size(h.levelmin + i)
        x = (a.astype(np.float64) + 0.5) * hl
        out.append(rho(x) * hl ** 3)
    m = np.concatenate(out).astype(np.float64)
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        m = m * (1.0 + noise * rng.uniform(-1.0, 1.0, size=m.shape[0]))
    return np.ascontiguousarray(m)
