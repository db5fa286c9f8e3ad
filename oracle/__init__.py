"""ctypes wrapper of the FP64 CPU oracle (``afmm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and
by the benchmark's CPU-baseline leg, never by the solver.  It shares no code
with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "afmm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ERRORS = {0: "ok", -1: "invalid argument", -2: "not graded", -3: "incomplete oct",
          -4: "unsupported", -5: "out of memory", -7: "bad state / call order"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2); returns the library path."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-Wno-unused-parameter", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        L.oracle_create.argtypes = [C.c_int, C.c_int, lp, ip, up, C.c_int, C.c_double, C.c_double,
                                    C.POINTER(P)]
        L.oracle_destroy.argtypes = [P]
        L.oracle_destroy.restype = None
        L.oracle_set_merged_all.argtypes = [P, C.c_int]
        L.oracle_set_merged_all.restype = None
        L.oracle_rebuild.argtypes = [P, C.c_int, dp]
        L.oracle_eval.argtypes = [P, C.c_int, C.c_int64, lp, dp, dp, P]
        L.oracle_solve.argtypes = [P, C.c_int, C.c_int, dp, dp, dp]
        L.oracle_solve_all.argtypes = [P, dp, dp, dp]
        L.oracle_direct.argtypes = [C.c_int64, dp, dp, C.c_int64, dp, C.c_double, dp, dp]
        L.oracle_nmi.argtypes = [C.c_int]
        L.oracle_multi_index.argtypes = [C.c_int, ip]
        L.oracle_derivs.argtypes = [C.c_int, dp, dp]
        L.oracle_multipole.argtypes = [C.c_int, C.c_int64, dp, dp, dp, dp]
        L.oracle_m2m.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_m2l.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_l2l.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_l2p.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_m2p.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_chain_check.argtypes = [P, C.c_int, C.POINTER(C.c_double)]
        L.oracle_num_threads.argtypes = []
        L.oracle_set_options.argtypes = [P, C.c_int, C.c_int]
        L.oracle_self_constant.argtypes = []
        L.oracle_self_constant.restype = C.c_double
        L.oracle_set_periodic.argtypes = [P, C.c_int]
        L.oracle_lattice.argtypes = [C.c_int, C.c_double, C.c_double, dp]
        L.oracle_lattice_at.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.oracle_direct_periodic.argtypes = [C.c_int64, dp, dp, C.c_int64, dp, C.c_double, C.c_double,
                                             C.c_double, dp, dp]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(rc, f"{what}: {ERRORS.get(rc, rc)}")


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def nmi(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def multi_index(p: int) -> np.ndarray:
    out = np.zeros(3 * nmi(p), dtype=np.int32)
    _check(lib().oracle_multi_index(p, out), "multi_index")
    return out.reshape(-1, 3)


def derivs(n: int, R) -> np.ndarray:
    """D_g(R) = d^g(-1/|R|) for |g| <= n, in `multi_index` order."""
    out = np.zeros(nmi(n), dtype=np.float64)
    _check(lib().oracle_derivs(n, np.ascontiguousarray(R, dtype=np.float64), out), "derivs")
    return out


def multipole(p: int, x, m, c) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    m = np.ascontiguousarray(m, dtype=np.float64)
    out = np.zeros(nmi(p))
    lib().oracle_multipole(p, x.shape[0], x.ravel(), m, np.ascontiguousarray(c, dtype=np.float64), out)
    return out


def _op(name, p, v, A):
    out = np.zeros(nmi(p) if name in ("m2m", "m2l", "l2l") else 4)
    getattr(lib(), "oracle_" + name)(p, np.ascontiguousarray(v, dtype=np.float64),
                                     np.ascontiguousarray(A, dtype=np.float64), out)
    return out


def m2m(p, t, M):
    return _op("m2m", p, t, M)


def m2l(p, R, M):
    return _op("m2l", p, R, M)


def l2l(p, a, L):
    return _op("l2l", p, a, L)


def l2p(p, u, L):
    return _op("l2p", p, u, L)


def m2p(p, R, M):
    return _op("m2p", p, R, M)


def direct(xs, ms, xt, G: float = 1.0):
    """O(N^2) sum over point masses; coincident points are skipped."""
    xs = np.ascontiguousarray(xs, dtype=np.float64).reshape(-1, 3)
    xt = np.ascontiguousarray(xt, dtype=np.float64).reshape(-1, 3)
    ms = np.ascontiguousarray(ms, dtype=np.float64)
    phi = np.zeros(xt.shape[0])
    acc = np.zeros(3 * xt.shape[0])
    lib().oracle_direct(xs.shape[0], xs.ravel(), ms, xt.shape[0], xt.ravel(), G, phi, acc)
    return phi, acc.reshape(-1, 3)


def direct_periodic(xs, ms, xt, G: float = 1.0, boxlen: float = 1.0, alpha: Optional[float] = None):
    """Ewald sum on the periodic box with a neutralising background (zero-mean
    potential); a source at a target's own position adds its images and the
    background only.  ``alpha`` is the split parameter (default 2.5 / boxlen)."""
    xs = np.ascontiguousarray(xs, dtype=np.float64).reshape(-1, 3)
    xt = np.ascontiguousarray(xt, dtype=np.float64).reshape(-1, 3)
    ms = np.ascontiguousarray(ms, dtype=np.float64)
    phi = np.zeros(xt.shape[0])
    acc = np.zeros(3 * xt.shape[0])
    al = 2.5 / boxlen if alpha is None else alpha
    _check(lib().oracle_direct_periodic(xs.shape[0], xs.ravel(), ms, xt.shape[0], xt.ravel(), G, boxlen, al,
                                        phi, acc), "direct_periodic")
    return phi, acc.reshape(-1, 3)


def lattice(n: int, boxlen: float = 1.0, alpha: Optional[float] = None, at=None) -> np.ndarray:
    """Lattice tensors D^lat_g (|g| <= n, the oracle's multi-index order): derivatives
    at ``at`` (default 0) of minus (the Ewald sum less the 27 nearest images of
    1/r); ``alpha`` defaults to 1.8 / boxlen, the value the periodic FMM uses."""
    out = np.zeros(nmi(n))
    al = 1.8 / boxlen if alpha is None else alpha
    if at is None:
        _check(lib().oracle_lattice(n, boxlen, al, out), "lattice")
    else:
        d = np.ascontiguousarray(at, dtype=np.float64).reshape(3)
        _check(lib().oracle_lattice_at(n, boxlen, al, d, out), "lattice_at")
    return out


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def self_constant() -> float:
    """Integral of 1/|r| over the unit cube centred at the origin (the oracle's quadrature)."""
    return float(lib().oracle_self_constant())


class Oracle:
    """Literal per-level-tree FMM on one hierarchy (see ``afmm_oracle.c``)."""

    def __init__(self, h, p: int, G: float = 1.0, quad_cap: bool = False, self_potential: bool = False,
                 periodic: bool = False):
        self.h = h
        self.p = p
        self.G = G
        self._ptr = C.c_void_p()
        ijk = np.ascontiguousarray(h.flat_ijk(), dtype=np.int32).ravel()
        ref = np.ascontiguousarray(h.flat_refined(), dtype=np.uint8)
        ncell = np.ascontiguousarray(h.ncell, dtype=np.int64)
        _check(lib().oracle_create(h.levelmin, h.levelmax, ncell, ijk, ref, p, G, h.boxlen,
                                   C.byref(self._ptr)), "create")
        # the paper's multipole cap (order p - 1) and the optional self-potential term
        _check(lib().oracle_set_options(self._ptr, int(bool(quad_cap)), int(bool(self_potential))), "set_options")
        # periodic box with a neutralising background (an extension of the paper's isolated box)
        if periodic:
            _check(lib().oracle_set_periodic(self._ptr, 1), "set_periodic")
        self.N = h.total
        self.offsets = h.offsets

    def close(self):
        if self._ptr:
            lib().oracle_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_merged_all(self, on: bool):
        lib().oracle_set_merged_all(self._ptr, int(bool(on)))

    def rebuild(self, level: int, mass: np.ndarray):
        _check(lib().oracle_rebuild(self._ptr, level, np.ascontiguousarray(mass, dtype=np.float64)),
               "rebuild")

    def eval(self, level: int, targets: np.ndarray, parts: bool = False):
        """phi[n], acc[n,3] (and optionally parts[n,4,4]) for level-`level` leaf flat indices."""
        t = np.ascontiguousarray(targets, dtype=np.int64)
        phi = np.zeros(t.shape[0])
        acc = np.zeros(3 * t.shape[0])
        part = np.zeros(16 * t.shape[0]) if parts else None
        pp = part.ctypes.data_as(C.c_void_p) if parts else None
        _check(lib().oracle_eval(self._ptr, level, t.shape[0], t, phi, acc, pp), "eval")
        if parts:
            return phi, acc.reshape(-1, 3), part.reshape(-1, 4, 4)
        return phi, acc.reshape(-1, 3)

    def eval_sample(self, flat_targets: np.ndarray):
        """Evaluate arbitrary leaf flat indices (any levels) with the current trees."""
        flat_targets = np.asarray(flat_targets, dtype=np.int64)
        lev = self.h.level_of()[flat_targets]
        phi = np.zeros(flat_targets.shape[0])
        acc = np.zeros((flat_targets.shape[0], 3))
        for L in np.unique(lev):
            sel = np.nonzero(lev == L)[0]
            p_, a_ = self.eval(int(L), flat_targets[sel])
            phi[sel] = p_
            acc[sel] = a_
        return phi, acc

    def solve(self, level: int, icount: int, mass: np.ndarray, phi: np.ndarray, acc: np.ndarray):
        """Alg. 1 Solve(level, icount): writes level-`level` leaves of flat phi[N], acc[N,3]."""
        _check(lib().oracle_solve(self._ptr, level, icount, np.ascontiguousarray(mass, dtype=np.float64),
                                  phi, acc.reshape(-1)), "solve")

    def solve_all(self, mass: np.ndarray):
        phi = np.zeros(self.N)
        acc = np.zeros(3 * self.N)
        _check(lib().oracle_solve_all(self._ptr, np.ascontiguousarray(mass, dtype=np.float64), phi, acc),
               "solve_all")
        return phi, acc.reshape(-1, 3)

    def chain_check(self, j: int) -> float:
        v = C.c_double()
        _check(lib().oracle_chain_check(self._ptr, j, C.byref(v)), "chain_check")
        return v.value
