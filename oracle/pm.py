"""Plain CPU reference of the particle-mesh time loop (the binary-orbit workload).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): used by the tests to
check the library's particle-mesh calls and its time loop.  Shares no code with
the HIP path: cloud-in-cell weights, the cell lookup and the leapfrog are
written out here in numpy; the hierarchy comes from ``synth.build_graded``
with a particle predicate; the cell fields from the FP64 oracle FMM.

- Cloud-in-cell (Sec. 1: particle masses deposited onto the AMR cells): a
  particle at x spreads its mass over the 8 cells of level L whose centres are
  within one cell size h of it, with weights prod_d (1 - |x_d/h - (c_d + 1/2)|).
- Interpolation back to the particles uses the same weights.
- Leapfrog, kick-drift-kick with a fixed step (Sec. 4, Fig. fig:binary).
"""
from __future__ import annotations

import numpy as np


def particle_refinement(pos: np.ndarray, nexpand: int):
    """Predicate for ``synth.build_graded``: refine the level-l cells within
    `nexpand` cells (Chebyshev distance) of a particle's 2x2x2 cloud at level l."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)

    def want(level, ijk, h):
        ijk = np.asarray(ijk, dtype=np.int64)
        out = np.zeros(ijk.shape[0], dtype=bool)
        for x in pos:
            c0 = np.floor(x / h - 0.5).astype(np.int64)
            lo, hi = c0 - nexpand, c0 + 1 + nexpand
            out |= np.all((ijk >= lo) & (ijk <= hi), axis=1)
        return out
    return want


def _index(h):
    """(level, i, j, k) -> flat index of the hierarchy's cells."""
    lev = h.level_of()
    ijk = h.flat_ijk()
    return {(int(l), int(a), int(b), int(c)): n for n, (l, (a, b, c)) in enumerate(zip(lev, ijk))}


def cloud(x, level, boxlen=1.0):
    """The 8 (cell, weight) pairs of a particle at level `level`."""
    h = boxlen / (1 << level)
    u = np.asarray(x, dtype=np.float64) / h - 0.5
    c0 = np.floor(u).astype(np.int64)
    f = u - c0
    out = []
    for o in range(8):
        d = np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1])
        w = float(np.prod(np.where(d == 1, f, 1.0 - f)))
        out.append((tuple(int(v) for v in c0 + d), w))
    return out


def deposit(h, level, pos, pmass, boxlen=1.0, index=None):
    index = index or _index(h)
    m = np.zeros(h.total)
    ref = h.flat_refined()
    for x, mp in zip(np.asarray(pos).reshape(-1, 3), pmass):
        for c, w in cloud(x, level, boxlen):
            n = index[(level, *c)]          # KeyError: the cloud cell is not in the hierarchy
            assert ref[n] == 0, "cloud cell is refined"
            m[n] += w * mp
    return m


def interpolate(h, level, pos, field, boxlen=1.0, index=None):
    index = index or _index(h)
    field = np.asarray(field)
    out = np.zeros((len(pos),) + field.shape[1:])
    for p, x in enumerate(np.asarray(pos).reshape(-1, 3)):
        for c, w in cloud(x, level, boxlen):
            out[p] += w * field[index[(level, *c)]]
    return out


def run(pos, vel, mass, levelmin, levelmax, nexpand, p, dt, nsteps, G=1.0, boxlen=1.0):
    """The kick-drift-kick loop with the oracle FMM; returns positions and
    velocities after every step ([nsteps + 1][np][3] each)."""
    import oracle
    from synth.hierarchy import build_graded

    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)

    def accel(x):
        h = build_graded(levelmin, levelmax, particle_refinement(x, nexpand), boxlen)
        idx = _index(h)
        L = h.levelmax
        m = deposit(h, L, x, mass, boxlen, idx)
        _, ac = oracle.Oracle(h, p, G).solve_all(m)
        return interpolate(h, L, x, ac, boxlen, idx)

    a = accel(pos)
    P, V = [pos.copy()], [vel.copy()]
    for _ in range(nsteps):
        vel += 0.5 * dt * a
        pos += dt * vel
        a = accel(pos)
        vel += 0.5 * dt * a
        P.append(pos.copy())
        V.append(vel.copy())
    return np.array(P), np.array(V)
