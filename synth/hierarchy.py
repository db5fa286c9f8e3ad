"""Graded AMR octree hierarchies on the unit (or `boxlen`) cube.

Level l has 2**l cells per dimension; cell (i, j, k) at level l has centre
((i, j, k) + 1/2) * boxlen / 2**l.  The coarsest level `levelmin` is complete
(8**levelmin cells).  A refined cell at level l owns its 8 children at l + 1,
and only leaves (unrefined cells) carry mass.

Grading follows the strong reading of the refinement rule in the paper's
nearest-field section (Sec. 3.2): a cell at level l may be refined only if the
3**3 level-(l-1) neighbours of its father (clipped to the box) are all refined.
`build_graded` enforces it by bottom-up dilation and iterates the refinement
predicate to a fixed point.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

MAX_LEVEL = 20


def encode(ijk: np.ndarray, level: int) -> np.ndarray:
    ijk = np.asarray(ijk, dtype=np.int64)
    return (ijk[:, 0] << (2 * level)) | (ijk[:, 1] << level) | ijk[:, 2]


def decode(keys: np.ndarray, level: int) -> np.ndarray:
    keys = np.asarray(keys, dtype=np.int64)
    mask = (1 << level) - 1
    out = np.empty((keys.shape[0], 3), dtype=np.int64)
    out[:, 0] = keys >> (2 * level)
    out[:, 1] = (keys >> level) & mask
    out[:, 2] = keys & mask
    return out


_OFFS27 = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)],
                   dtype=np.int64)
_OCT = np.array([(o & 1, (o >> 1) & 1, (o >> 2) & 1) for o in range(8)], dtype=np.int64)


def children_keys(keys: np.ndarray, level: int) -> np.ndarray:
    """Keys (level + 1) of the 8 children of every key, sorted."""
    if keys.size == 0:
        return keys.astype(np.int64)
    ijk = decode(keys, level)
    ch = (2 * ijk[:, None, :] + _OCT[None, :, :]).reshape(-1, 3)
    return np.sort(encode(ch, level + 1))


def neighbours27(keys: np.ndarray, level: int, periodic: bool = False) -> np.ndarray:
    """Unique keys of the 27-neighbourhoods (inclusive) of `keys`, clipped to the box
    (or wrapped around it when `periodic`)."""
    if keys.size == 0:
        return keys.astype(np.int64)
    ijk = decode(keys, level)
    nb = (ijk[:, None, :] + _OFFS27[None, :, :]).reshape(-1, 3)
    n = 1 << level
    if periodic:
        return np.unique(encode(nb % n, level))
    ok = np.all((nb >= 0) & (nb < n), axis=1)
    return np.unique(encode(nb[ok], level))


@dataclass
class Hierarchy:
    """Per-level cell lists in caller order (the order the arrays are given in)."""

    levelmin: int
    levelmax: int
    ijk: List[np.ndarray]        # per level: int32 [n, 3]
    refined: List[np.ndarray]    # per level: uint8 [n]
    boxlen: float = 1.0
    meta: dict = field(default_factory=dict)

    # -- sizes and flat (level-major) views ---------------------------------
    @property
    def nlevels(self) -> int:
        return self.levelmax - self.levelmin + 1

    @property
    def ncell(self) -> np.ndarray:
        return np.array([a.shape[0] for a in self.ijk], dtype=np.int64)

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.ncell)]).astype(np.int64)

    @property
    def total(self) -> int:
        return int(self.ncell.sum())

    def level_of(self) -> np.ndarray:
        return np.concatenate([np.full(n, self.levelmin + i, dtype=np.int32)
                               for i, n in enumerate(self.ncell)])

    def flat_ijk(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate(self.ijk, axis=0).astype(np.int32))

    def flat_refined(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate(self.refined).astype(np.uint8))

    def leaf_mask(self) -> np.ndarray:
        return self.flat_refined() == 0

    def nleaves(self) -> int:
        return int(self.leaf_mask().sum())

    def leaves_per_level(self) -> List[int]:
        return [int((r == 0).sum()) for r in self.refined]

    def cell_size(self, level: int) -> float:
        return self.boxlen / float(1 << level)

    def centres(self) -> np.ndarray:
        """Physical cell centres, flat level-major [N, 3] float64."""
        out = []
        for i, a in enumerate(self.ijk):
            h = self.cell_size(self.levelmin + i)
            out.append((a.astype(np.float64) + 0.5) * h)
        return np.concatenate(out, axis=0)

    def level_slice(self, level: int) -> slice:
        o = self.offsets
        i = level - self.levelmin
        return slice(int(o[i]), int(o[i + 1]))

    def summary(self) -> dict:
        return {
            "levelmin": self.levelmin,
            "levelmax": self.levelmax,
            "ncell": [int(x) for x in self.ncell],
            "leaves": self.leaves_per_level(),
            "refined": [int(r.sum()) for r in self.refined],
            "total_leaves": self.nleaves(),
        }


def _from_refined_sets(levelmin: int, levelmax: int, refined_keys: List[np.ndarray],
                       boxlen: float) -> Hierarchy:
    """Assemble a hierarchy (Morton-free, key-sorted caller order) from refined key sets."""
    n0 = 1 << levelmin
    g = np.arange(n0, dtype=np.int64)
    ii, jj, kk = np.meshgrid(g, g, g, indexing="ij")
    cells = np.sort(encode(np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1), levelmin))
    ijk, ref = [], []
    for lev in range(levelmin, levelmax + 1):
        rk = refined_keys[lev - levelmin] if lev < levelmax else np.zeros(0, np.int64)
        flags = np.isin(cells, rk, assume_unique=True).astype(np.uint8)
        ijk.append(decode(cells, lev).astype(np.int32))
        ref.append(flags)
        if lev < levelmax:
            cells = children_keys(cells[flags.astype(bool)], lev)
    # drop trailing empty levels
    while len(ijk) > 1 and ijk[-1].shape[0] == 0:
        ijk.pop()
        ref.pop()
    lmax = levelmin + len(ijk) - 1
    return Hierarchy(levelmin, lmax, ijk, ref, boxlen)


def unigrid(level: int, boxlen: float = 1.0) -> Hierarchy:
    return _from_refined_sets(level, level, [], boxlen)


def build_graded(levelmin: int, levelmax: int,
                 want: Callable[[int, np.ndarray, float], np.ndarray],
                 boxlen: float = 1.0, max_iter: int = 50, periodic: bool = False) -> Hierarchy:
    """Refine where `want(level, ijk[n,3], h) -> bool[n]` asks, then grade.

    The predicate is applied top-down to the cells that exist; the strong
    grading rule is then closed bottom-up (refined cell at l => the 27
    neighbours of its father at l-1 are refined; on a periodic box the
    neighbours wrap around).  Both steps only add refinement, so alternating
    them reaches a fixed point.
    """
    assert 1 <= levelmin <= levelmax <= MAX_LEVEL
    R = [np.zeros(0, np.int64) for _ in range(levelmin, levelmax)]
    for _ in range(max_iter):
        changed = False
        # top-down: predicate on existing cells
        n0 = 1 << levelmin
        g = np.arange(n0, dtype=np.int64)
        ii, jj, kk = np.meshgrid(g, g, g, indexing="ij")
        cells = np.sort(encode(np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1), levelmin))
        for lev in range(levelmin, levelmax):
            i = lev - levelmin
            if cells.size:
                m = np.asarray(want(lev, decode(cells, lev), boxlen / (1 << lev)), dtype=bool)
                new = np.union1d(R[i], cells[m])
            else:
                new = R[i]
            new = np.intersect1d(new, cells, assume_unique=False)
            if new.size != R[i].size:
                changed = True
            R[i] = new
            cells = children_keys(R[i], lev)
        # bottom-up grading closure
        for lev in range(levelmax - 1, levelmin, -1):
            i = lev - levelmin
            if R[i].size == 0:
                continue
            fk = np.unique(encode(decode(R[i], lev) // 2, lev - 1))
            req = neighbours27(fk, lev - 1, periodic)
            merged = np.union1d(R[i - 1], req)
            if merged.size != R[i - 1].size:
                changed = True
                R[i - 1] = merged
        if not changed:
            break
    else:
        raise RuntimeError("graded refinement did not converge")
    return _from_refined_sets(levelmin, levelmax, R, boxlen)


def shuffle_order(h: Hierarchy, seed: int) -> Hierarchy:
    """Same hierarchy with every level's cells in a seeded random caller order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ijk, ref = [], []
    for a, r in zip(h.ijk, h.refined):
        perm = rng.permutation(a.shape[0])
        ijk.append(np.ascontiguousarray(a[perm]))
        ref.append(np.ascontiguousarray(r[perm]))
    out = Hierarchy(h.levelmin, h.levelmax, ijk, ref, h.boxlen, dict(h.meta))
    return out


def mirror_x(h: Hierarchy) -> Hierarchy:
    """Mirror image under x -> boxlen - x, keeping each cell's caller position."""
    ijk = []
    for i, a in enumerate(h.ijk):
        lev = h.levelmin + i
        b = a.copy()
        b[:, 0] = (1 << lev) - 1 - b[:, 0]
        ijk.append(b)
    return Hierarchy(h.levelmin, h.levelmax, ijk, [r.copy() for r in h.refined], h.boxlen,
                     dict(h.meta))


def refine_sphere(centre, radii: dict) -> Callable:
    """Predicate: refine level-l cells whose centre is within radii[l] of `centre`."""
    c = np.asarray(centre, dtype=np.float64)

    def want(level, ijk, h):
        r = radii.get(level)
        if r is None:
            return np.zeros(ijk.shape[0], dtype=bool)
        x = (ijk.astype(np.float64) + 0.5) * h
        return np.sum((x - c) ** 2, axis=1) <= r * r

    return want


def refine_mass(density: Callable, threshold: float, levelmax: int) -> Callable:
    """Predicate: refine cells whose midpoint-rule mass rho(x_c) h^3 exceeds `threshold`."""

    def want(level, ijk, h):
        if level >= levelmax:
            return np.zeros(ijk.shape[0], dtype=bool)
        x = (ijk.astype(np.float64) + 0.5) * h
        return density(x) * h ** 3 > threshold

    return want


def check_graded(h: Hierarchy) -> Optional[str]:
    """Independent checker of completeness and strong grading; returns an error or None."""
    if h.ijk[0].shape[0] != 8 ** h.levelmin:
        return "coarsest level incomplete"
    keysets = [np.sort(encode(a.astype(np.int64), h.levelmin + i)) for i, a in enumerate(h.ijk)]
    for i in range(h.nlevels):
        lev = h.levelmin + i
        if np.unique(keysets[i]).size != keysets[i].size:
            return f"duplicate cells at level {lev}"
        rk = np.sort(encode(h.ijk[i][h.refined[i].astype(bool)].astype(np.int64), lev))
        if i + 1 < h.nlevels:
            ch = children_keys(rk, lev)
            if ch.size != keysets[i + 1].size or np.any(ch != keysets[i + 1]):
                return f"level {lev + 1} is not exactly the children of refined level-{lev} cells"
        elif rk.size:
            return "refined cells at levelmax"
        if i >= 1 and rk.size:
            fk = np.unique(encode(decode(rk, lev) // 2, lev - 1))
            req = neighbours27(fk, lev - 1)
            prev_ref = np.sort(encode(h.ijk[i - 1][h.refined[i - 1].astype(bool)].astype(np.int64),
                                      lev - 1))
            if not np.all(np.isin(req, prev_ref)):
                return f"grading violated at level {lev}"
    return None
