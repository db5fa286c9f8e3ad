"""The five synthetic workloads (and reduced-size variants used in tests).

1. unigrid 32^3 (level 5), Plummer M=1, a=0.1 at the box centre, 1% noise, seed 1, p=4, FP64.
2. level 6 complete + level 7 over the level-6 cells whose centre is within 0.15 of
   the box centre; Plummer a=0.05 + 1% noise, seed 2; p=6, FP32.
3. level 7 base, up to level 11, refined where the midpoint mass of
   (Plummer a=0.05 + 32 Gaussian clumps) exceeds k * M_total / 128^3, k = CFG3_K
   (chosen so that the hierarchy holds about 8M leaves); 1% noise, seed 3; p=6, FP32.
4. 256 hierarchies: base level U{4,5,6}, 0-3 extra levels refined where the mass
   exceeds 8x the mean base-cell mass; Plummer (a ~ U[0.05,0.15], centre
   U[0.35,0.65]^3) or 8 clumps; seed 4000+i; p=4 and p=8, FP32.
5. level 7 + level 8 over centres within r<0.2 + level 9 within r<0.1 (graded),
   Plummer a=0.05 + 1% noise, seed 5; p=6, FP32.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np

from .density import cell_masses, gaussian_clumps, plummer, sum_density
from .hierarchy import Hierarchy, build_graded, refine_mass, refine_sphere, unigrid

CENTRE = (0.5, 0.5, 0.5)
# Refinement threshold factor of workload 3 (mass > k * M_total / 128^3); the
# value is chosen so the hierarchy lands near 8M leaves.
CFG3_K = 1.25


@dataclass
class Workload:
    name: str
    hierarchy: Hierarchy
    mass: np.ndarray
    p: int
    precision: str          # "fp64" or "fp32"
    seed: int
    description: str = ""


def cfg1(level: int = 5, seed: int = 1, p: int = 4) -> Workload:
    h = unigrid(level)
    rho = plummer(1.0, 0.1, CENTRE)
    m = cell_masses(h, rho, noise=0.01, seed=seed)
    return Workload(f"unigrid{1 << level}^3_p{p}", h, m, p, "fp64", seed,
                    f"unigrid {1 << level}^3, Plummer a=0.1, 1% noise")


def cfg2(base: int = 6, radius: float = 0.15, seed: int = 2, p: int = 6) -> Workload:
    want = refine_sphere(CENTRE, {base: radius})
    h = build_graded(base, base + 1, want)
    rho = plummer(1.0, 0.05, CENTRE)
    m = cell_masses(h, rho, noise=0.01, seed=seed)
    return Workload(f"amr2_{1 << base}^3+1_p{p}", h, m, p, "fp32", seed,
                    f"level {base} + level {base + 1} within r<={radius}, Plummer a=0.05")


def cfg3_density(seed: int = 3, nclumps: int = 32) -> Callable:
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.1, 0.9, size=(nclumps, 3))
    sig = rng.uniform(0.005, 0.02, size=nclumps)
    ms = 10.0 ** rng.uniform(-3.0, -2.0, size=nclumps)
    return sum_density(plummer(1.0, 0.05, CENTRE), gaussian_clumps(centres, sig, ms))


def cfg3(base: int = 7, extra: int = 4, k: float = CFG3_K, seed: int = 3, p: int = 6) -> Workload:
    rho = cfg3_density(seed)
    thr = k * 1.0 / float((1 << base) ** 3)
    h = build_graded(base, base + extra, refine_mass(rho, thr, base + extra))
    m = cell_masses(h, rho, noise=0.01, seed=seed)
    return Workload(f"deep_{1 << base}^3+{extra}_p{p}", h, m, p, "fp32", seed,
                    f"level {base} base, up to {extra} levels refined on mass > {k} x mean")


def cfg5(base: int = 7, r1: float = 0.2, r2: float = 0.1, seed: int = 5, p: int = 6) -> Workload:
    want = refine_sphere(CENTRE, {base: r1, base + 1: r2})
    h = build_graded(base, base + 2, want)
    rho = plummer(1.0, 0.05, CENTRE)
    m = cell_masses(h, rho, noise=0.01, seed=seed)
    return Workload(f"diff_{1 << base}^3+2_p{p}", h, m, p, "fp32", seed,
                    f"level {base} + r<{r1} + r<{r2}, Plummer a=0.05")


def cfg4_member(i: int, p: int = 4, base_choices=(4, 5, 6), max_extra: int = 3) -> Workload:
    seed = 4000 + i
    rng = np.random.Generator(np.random.PCG64(seed))
    base = int(rng.choice(base_choices))
    extra = int(rng.integers(0, max_extra + 1))
    if rng.uniform() < 0.5:
        a = rng.uniform(0.05, 0.15)
        c = rng.uniform(0.35, 0.65, size=3)
        rho = plummer(1.0, a, c)
    else:
        centres = rng.uniform(0.2, 0.8, size=(8, 3))
        sig = rng.uniform(0.01, 0.04, size=8)
        ms = np.full(8, 1.0 / 8.0)
        rho = gaussian_clumps(centres, sig, ms)
    thr = 8.0 / float((1 << base) ** 3)
    h = build_graded(base, base + extra, refine_mass(rho, thr, base + extra))
    m = cell_masses(h, rho, noise=0.01, seed=seed)
    return Workload(f"batch_member{i}", h, m, p, "fp32", seed, "")


def cfg4(n: int = 256, p: int = 4, **kw) -> List[Workload]:
    return [cfg4_member(i, p=p, **kw) for i in range(n)]
