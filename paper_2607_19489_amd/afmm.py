"""Python binding of the C ABI (argument marshalling only).

Every step of a solve runs in the HIP library; PyTorch supplies device memory
and the current stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from ._lib import (AFMM_ALL_LEVELS, AFMM_CHECK_INPUT, AFMM_FP32_MIXED, AFMM_FP64, AFMM_GRAPH, AFMM_OVERLAP, AFMM_PAPER_QUAD_CAP,
                   AFMM_PERIODIC, AFMM_SELF_POTENTIAL, AFMM_SERIAL, HierarchyC, Options, PlanInfo, StageTime, TuneResult, check, lib)

PRECISIONS = {"fp64": AFMM_FP64, "fp32": AFMM_FP32_MIXED, "mixed": AFMM_FP32_MIXED}


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _hierarchy_arrays(h):
    """(levelmin, levelmax, ncell[int64], ijk[int32 flat], refined[uint8]) from a hierarchy object."""
    ncell = np.ascontiguousarray(np.asarray(h.ncell, dtype=np.int64))
    ijk = np.ascontiguousarray(np.asarray(h.flat_ijk(), dtype=np.int32).reshape(-1))
    ref = np.ascontiguousarray(np.asarray(h.flat_refined(), dtype=np.uint8))
    return int(h.levelmin), int(h.levelmax), ncell, ijk, ref


def _hier_struct(levelmin, levelmax, ncell, ijk, ref):
    hc = HierarchyC()
    hc.levelmin = levelmin
    hc.levelmax = levelmax
    hc.ncell = ncell.ctypes.data_as(C.POINTER(C.c_int64))
    hc.ijk = ijk.ctypes.data_as(C.POINTER(C.c_int32))
    hc.refined = ref.ctypes.data_as(C.POINTER(C.c_uint8))
    return hc


def make_options(p: int = 4, precision: str = "fp64", G: float = 1.0, boxlen: float = 1.0,
                 fp64_levels: int = 3, check_input: bool = False, max_device_bytes: int = 0,
                 tap_split: int = 0, serial: bool = False, overlap: bool = False,
                 quad_cap: bool = False, self_potential: bool = False, graph: bool = False,
                 m2p_shape: int = 0, periodic: bool = False) -> Options:
    o = Options()
    lib().afmm_options_default(C.byref(o))
    o.p = p
    o.precision = PRECISIONS[precision]
    o.G = G
    o.boxlen = boxlen
    o.fp64_levels = fp64_levels
    o.tap_split = tap_split
    o.flags = ((AFMM_CHECK_INPUT if check_input else 0) | (AFMM_SERIAL if serial else 0)
               | (AFMM_OVERLAP if overlap else 0) | (AFMM_PAPER_QUAD_CAP if quad_cap else 0)
               | (AFMM_SELF_POTENTIAL if self_potential else 0) | (AFMM_GRAPH if graph else 0)
               | (AFMM_PERIODIC if periodic else 0))
    o.max_device_bytes = max_device_bytes
    o.m2p_shape = m2p_shape
    return o


def hierarchy_check(h, p: int = 4, precision: str = "fp64", **opts) -> dict:
    """Host-only validation and work counts (no device needed)."""
    arrs = _hierarchy_arrays(h)
    hc = _hier_struct(*arrs)
    info = PlanInfo()
    o = make_options(p, precision, boxlen=float(getattr(h, "boxlen", 1.0)), **opts)
    check(lib().afmm_hierarchy_check(C.byref(hc), C.byref(o), C.byref(info)), "afmm_hierarchy_check")
    return info.as_dict()


def _profile(fn, handle, what) -> dict:
    buf = (StageTime * 16)()
    n = C.c_int32()
    check(fn(handle, buf, 16, C.byref(n)), what)
    return {buf[i].name.decode(): {"launches": buf[i].launches, "ms": buf[i].ms, "flops": buf[i].flops,
                                   "bytes": buf[i].bytes} for i in range(min(n.value, 16))}


class Plan:
    """A solver plan for one AMR hierarchy (afmm_plan)."""

    def __init__(self, h, p: int = 4, precision: str = "fp64", G: float = 1.0,
                 boxlen: Optional[float] = None, fp64_levels: int = 3, check_input: bool = False,
                 max_device_bytes: int = 0, tap_split: int = 0, serial: bool = False,
                 overlap: bool = False, quad_cap: bool = False, self_potential: bool = False,
                 graph: bool = False, m2p_shape: int = 0, periodic: bool = False,
                 stream: Optional[torch.cuda.Stream] = None):
        self._ptr = C.c_void_p()
        arrs = _hierarchy_arrays(h)
        self.levelmin, self.levelmax, self.ncell = arrs[0], arrs[1], arrs[2]
        self.N = int(self.ncell.sum())
        hc = _hier_struct(*arrs)
        bl = float(boxlen if boxlen is not None else getattr(h, "boxlen", 1.0))
        self.options = make_options(p, precision, G, bl, fp64_levels, check_input, max_device_bytes, tap_split,
                                    serial, overlap, quad_cap, self_potential, graph, m2p_shape, periodic)
        check(lib().afmm_plan_create(C.byref(hc), C.byref(self.options), _stream_handle(stream),
                                     C.byref(self._ptr)), "afmm_plan_create")
        self.p = p
        self.precision = precision

    def replan(self, h, level: int, stream: Optional[torch.cuda.Stream] = None) -> "Plan":
        """afmm_plan_replan: a plan for `h`, whose levels below `level` are this
        plan's, carrying over the stale trees' masses; this plan stays valid."""
        arrs = _hierarchy_arrays(h)
        hc = _hier_struct(*arrs)
        new = Plan.__new__(Plan)
        new._ptr = C.c_void_p()
        check(lib().afmm_plan_replan(self._ptr, C.byref(hc), level, _stream_handle(stream), C.byref(new._ptr)),
              "afmm_plan_replan")
        new.levelmin, new.levelmax, new.ncell = arrs[0], arrs[1], arrs[2]
        new.N = int(new.ncell.sum())
        new.options, new.p, new.precision = self.options, self.p, self.precision
        return new

    def close(self):
        if self._ptr:
            lib().afmm_plan_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> C.c_void_p:
        return self._ptr

    def info(self) -> dict:
        info = PlanInfo()
        check(lib().afmm_plan_get_info(self._ptr, C.byref(info)), "afmm_plan_get_info")
        return info.as_dict()

    def set_profiling(self, enable: bool):
        check(lib().afmm_plan_set_profiling(self._ptr, int(bool(enable))), "afmm_plan_set_profiling")

    def get_profile(self) -> dict:
        """Per kernel family: launches, summed event ms, algorithmic flops and bytes (resets)."""
        return _profile(lib().afmm_plan_get_profile, self._ptr, "afmm_plan_get_profile")

    def _check_tensor(self, t: torch.Tensor, shape, name: str):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def solve(self, mass: torch.Tensor, level: int = AFMM_ALL_LEVELS, icount: int = 1,
              phi: Optional[torch.Tensor] = None, acc: Optional[torch.Tensor] = None,
              stream: Optional[torch.cuda.Stream] = None):
        """afmm_solve: returns (phi[N], acc[N, 3]) (only solved leaves are written)."""
        self._check_tensor(mass, (self.N,), "mass")
        if phi is None:
            phi = torch.zeros(self.N, dtype=torch.float64, device=mass.device)
        if acc is None:
            acc = torch.zeros(self.N, 3, dtype=torch.float64, device=mass.device)
        self._check_tensor(phi, (self.N,), "phi")
        self._check_tensor(acc, (self.N, 3), "acc")
        check(lib().afmm_solve(self._ptr, level, icount, C.c_void_p(mass.data_ptr()),
                               C.c_void_p(phi.data_ptr()), C.c_void_p(acc.data_ptr()), _stream_handle(stream)),
              "afmm_solve")
        return phi, acc

    def solve_drift(self, mass: torch.Tensor, mass_rate: torch.Tensor, time: float, level: int = AFMM_ALL_LEVELS,
                    icount: int = 1, phi: Optional[torch.Tensor] = None, acc: Optional[torch.Tensor] = None,
                    stream: Optional[torch.cuda.Stream] = None):
        """afmm_solve_drift: afmm_solve with the stale trees advanced to `time`
        by the mass rates their last rebuild recorded; returns (phi, acc)."""
        self._check_tensor(mass, (self.N,), "mass")
        self._check_tensor(mass_rate, (self.N,), "mass_rate")
        if phi is None:
            phi = torch.zeros(self.N, dtype=torch.float64, device=mass.device)
        if acc is None:
            acc = torch.zeros(self.N, 3, dtype=torch.float64, device=mass.device)
        self._check_tensor(phi, (self.N,), "phi")
        self._check_tensor(acc, (self.N, 3), "acc")
        check(lib().afmm_solve_drift(self._ptr, level, icount, float(time), C.c_void_p(mass.data_ptr()),
                                     C.c_void_p(mass_rate.data_ptr()), C.c_void_p(phi.data_ptr()),
                                     C.c_void_p(acc.data_ptr()), _stream_handle(stream)), "afmm_solve_drift")
        return phi, acc

    def autotune(self, mass: torch.Tensor, phi: Optional[torch.Tensor] = None, acc: Optional[torch.Tensor] = None,
                 stream: Optional[torch.cuda.Stream] = None) -> dict:
        """afmm_plan_autotune: pick the M2L / M2P tap splits by timing; leaves a full solve in phi/acc."""
        self._check_tensor(mass, (self.N,), "mass")
        if phi is None:
            phi = torch.zeros(self.N, dtype=torch.float64, device=mass.device)
        if acc is None:
            acc = torch.zeros(self.N, 3, dtype=torch.float64, device=mass.device)
        res = TuneResult()
        check(lib().afmm_plan_autotune(self._ptr, C.c_void_p(mass.data_ptr()), C.c_void_p(phi.data_ptr()),
                                       C.c_void_p(acc.data_ptr()), _stream_handle(stream), C.byref(res)),
              "afmm_plan_autotune")
        return res.as_dict()

    def solve_adjoint(self, phi_bar: torch.Tensor, acc_bar: torch.Tensor, level: int = AFMM_ALL_LEVELS,
                      mass_bar: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
        """afmm_solve_adjoint: returns mass_bar[N] = A^T (phi_bar, acc_bar)."""
        self._check_tensor(phi_bar, (self.N,), "phi_bar")
        self._check_tensor(acc_bar, (self.N, 3), "acc_bar")
        if mass_bar is None:
            mass_bar = torch.zeros(self.N, dtype=torch.float64, device=phi_bar.device)
        self._check_tensor(mass_bar, (self.N,), "mass_bar")
        check(lib().afmm_solve_adjoint(self._ptr, level, C.c_void_p(phi_bar.data_ptr()),
                                       C.c_void_p(acc_bar.data_ptr()), C.c_void_p(mass_bar.data_ptr()),
                                       _stream_handle(stream)), "afmm_solve_adjoint")
        return mass_bar


def _check_f64(t: torch.Tensor, shape, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Batch:
    """Independent hierarchies solved as one forest, replayed as one hipGraph (afmm_batch)."""

    def __init__(self, plans: Sequence[Plan], stream: Optional[torch.cuda.Stream] = None):
        self._ptr = C.c_void_p()
        self.sizes = [pl.N for pl in plans]
        arr = (C.c_void_p * len(plans))(*[pl.handle.value for pl in plans])
        check(lib().afmm_batch_create(arr, len(plans), _stream_handle(stream), C.byref(self._ptr)),
              "afmm_batch_create")

    def close(self):
        if self._ptr:
            lib().afmm_batch_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        info = PlanInfo()
        check(lib().afmm_batch_get_info(self._ptr, C.byref(info)), "afmm_batch_get_info")
        return info.as_dict()

    def set_profiling(self, enable: bool):
        """While enabled, solves run eagerly with per-launch events (no graph)."""
        check(lib().afmm_batch_set_profiling(self._ptr, int(bool(enable))), "afmm_batch_set_profiling")

    def get_profile(self) -> dict:
        return _profile(lib().afmm_batch_get_profile, self._ptr, "afmm_batch_get_profile")

    def _arrays(self, masses, phis, accs):
        n = len(self.sizes)
        if len(masses) != n:
            raise ValueError(f"expected {n} mass tensors")
        if phis is None:
            phis = [torch.zeros(N, dtype=torch.float64, device=masses[0].device) for N in self.sizes]
        if accs is None:
            accs = [torch.zeros(N, 3, dtype=torch.float64, device=masses[0].device) for N in self.sizes]
        for i, N in enumerate(self.sizes):
            _check_f64(masses[i], (N,), f"masses[{i}]")
            _check_f64(phis[i], (N,), f"phis[{i}]")
            _check_f64(accs[i], (N, 3), f"accs[{i}]")
        mp = (C.c_void_p * n)(*[t.data_ptr() for t in masses])
        pp = (C.c_void_p * n)(*[t.data_ptr() for t in phis])
        ap = (C.c_void_p * n)(*[t.data_ptr() for t in accs])
        return phis, accs, mp, pp, ap

    def autotune(self, masses: Sequence[torch.Tensor], stream: Optional[torch.cuda.Stream] = None) -> dict:
        """afmm_batch_autotune: pick the tap splits by timing and capture the graph again."""
        # phis/accs stay referenced until the call returns: the table holds their addresses
        phis, accs, mp, pp, ap = self._arrays(masses, None, None)
        res = TuneResult()
        check(lib().afmm_batch_autotune(self._ptr, mp, pp, ap, _stream_handle(stream), C.byref(res)),
              "afmm_batch_autotune")
        del phis, accs
        return res.as_dict()

    def solve(self, masses: Sequence[torch.Tensor], phis: Optional[Sequence[torch.Tensor]] = None,
              accs: Optional[Sequence[torch.Tensor]] = None, stream: Optional[torch.cuda.Stream] = None):
        """afmm_batch_solve: returns the lists (phis, accs)."""
        phis, accs, mp, pp, ap = self._arrays(masses, phis, accs)
        check(lib().afmm_batch_solve(self._ptr, mp, pp, ap, _stream_handle(stream)), "afmm_batch_solve")
        return phis, accs


class AFMMSolve(torch.autograd.Function):
    """(phi, acc) = FMM(mass) with the hand-written adjoint as backward."""

    @staticmethod
    def forward(ctx, mass: torch.Tensor, plan: Plan):
        ctx.plan = plan
        phi, acc = plan.solve(mass.detach().contiguous())
        return phi, acc

    @staticmethod
    def backward(ctx, phi_bar, acc_bar):
        plan = ctx.plan
        if phi_bar is None:
            phi_bar = torch.zeros(plan.N, dtype=torch.float64, device=acc_bar.device)
        if acc_bar is None:
            acc_bar = torch.zeros(plan.N, 3, dtype=torch.float64, device=phi_bar.device)
        mbar = plan.solve_adjoint(phi_bar.contiguous(), acc_bar.contiguous())
        return mbar, None


def solve(mass: torch.Tensor, plan: Plan):
    """Differentiable full solve."""
    return AFMMSolve.apply(mass, plan)


def release_cached_memory():
    """Free the device buffers that destroyed plans left in the library's cache."""
    check(lib().afmm_release_cached_memory(), "afmm_release_cached_memory")
