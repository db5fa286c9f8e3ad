"""Loader of the in-tree HIP library ``libafmm.so`` (C ABI of include/afmm.h).

There is no fallback: if the library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafmm.so")

AFMM_OK = 0
AFMM_FP64 = 0
AFMM_FP32_MIXED = 1
AFMM_CHECK_INPUT = 1
AFMM_SERIAL = 2
AFMM_OVERLAP = 4
AFMM_PAPER_QUAD_CAP = 8
AFMM_GRAPH = 32
AFMM_SELF_POTENTIAL = 16
AFMM_PERIODIC = 64
AFMM_ALL_LEVELS = -1

STATUS = {
    0: "AFMM_OK", -1: "AFMM_E_INVALID_ARG", -2: "AFMM_E_NOT_GRADED", -3: "AFMM_E_INCOMPLETE_OCT",
    -4: "AFMM_E_UNSUPPORTED", -5: "AFMM_E_OUT_OF_MEMORY", -6: "AFMM_E_DEVICE", -7: "AFMM_E_ATS_ORDER",
    -8: "AFMM_E_NONFINITE",
}

# every symbol the header declares
SYMBOLS = [
    "afmm_options_default", "afmm_plan_create", "afmm_plan_destroy", "afmm_plan_get_info", "afmm_solve",
    "afmm_solve_adjoint", "afmm_batch_create", "afmm_batch_solve", "afmm_batch_get_info",
    "afmm_batch_destroy", "afmm_hierarchy_check", "afmm_status_string", "afmm_last_error",
    "afmm_plan_set_profiling", "afmm_plan_get_profile", "afmm_batch_set_profiling", "afmm_batch_get_profile",
    "afmm_plan_autotune", "afmm_batch_autotune", "afmm_solve_adjoint_noalloc",
    "afmm_particle_hierarchy_create", "afmm_particle_hierarchy_view", "afmm_particle_hierarchy_destroy",
    "afmm_cic_deposit", "afmm_cic_interpolate", "afmm_particles_update", "afmm_plan_replan", "afmm_solve_drift",
    "afmm_release_cached_memory",
]


class Options(C.Structure):
    _fields_ = [("p", C.c_int32), ("precision", C.c_int32), ("G", C.c_double), ("boxlen", C.c_double),
                ("flags", C.c_uint32), ("fp64_levels", C.c_int32), ("tap_split", C.c_int32),
                ("max_device_bytes", C.c_size_t), ("m2p_shape", C.c_int32)]


class HierarchyC(C.Structure):
    _fields_ = [("levelmin", C.c_int32), ("levelmax", C.c_int32), ("ncell", C.POINTER(C.c_int64)),
                ("ijk", C.POINTER(C.c_int32)), ("refined", C.POINTER(C.c_uint8))]


class PlanInfo(C.Structure):
    _fields_ = [("levelmin", C.c_int32), ("levelmax", C.c_int32), ("p", C.c_int32), ("K", C.c_int32),
                ("precision", C.c_int32), ("nhier", C.c_int32),
                ("ncell", C.c_int64), ("nleaves", C.c_int64), ("nrefined", C.c_int64),
                ("leaves_per_level", C.c_int64 * 21),
                ("m2l_targets", C.c_int64), ("m2l_pairs", C.c_int64), ("m2p_pairs", C.c_int64),
                ("p2p_pairs", C.c_int64), ("near_m2p_pairs", C.c_int64), ("nearest_pairs", C.c_int64),
                ("flops_m2l", C.c_double), ("flops_m2p", C.c_double), ("flops_p2p", C.c_double),
                ("flops_updown", C.c_double), ("bytes_min", C.c_double), ("device_bytes", C.c_size_t)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "leaves_per_level" else v
        return d


class StageTime(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("launches", C.c_int32), ("ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("m2l_split", C.c_int32 * 2), ("m2p_split", C.c_int32 * 2), ("ms_before", C.c_double),
                ("ms_after", C.c_double), ("candidates", C.c_int32), ("m2p_shape", C.c_int32 * 2)]

    def as_dict(self):
        return {"m2l_split": list(self.m2l_split), "m2p_split": list(self.m2p_split),
                "m2p_shape": list(self.m2p_shape), "ms_before": self.ms_before, "ms_after": self.ms_after,
                "candidates": self.candidates}


class AfmmError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str):
        super().__init__(f"{what}: {STATUS.get(code, code)} ({detail})")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(paper_2607_19489_amd/build.py); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.afmm_options_default.argtypes = [C.POINTER(Options)]
    L.afmm_options_default.restype = None
    L.afmm_plan_create.argtypes = [C.POINTER(HierarchyC), C.POINTER(Options), vp, C.POINTER(vp)]
    L.afmm_plan_destroy.argtypes = [vp]
    L.afmm_release_cached_memory.argtypes = []
    L.afmm_plan_replan.argtypes = [vp, C.POINTER(HierarchyC), C.c_int32, vp, C.POINTER(vp)]
    L.afmm_plan_get_info.argtypes = [vp, C.POINTER(PlanInfo)]
    L.afmm_solve.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, vp]
    L.afmm_solve_drift.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, vp, vp, vp, vp, vp]
    L.afmm_solve_adjoint.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.afmm_solve_adjoint_noalloc.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.afmm_batch_create.argtypes = [C.POINTER(vp), C.c_int32, vp, C.POINTER(vp)]
    L.afmm_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp]
    L.afmm_batch_get_info.argtypes = [vp, C.POINTER(PlanInfo)]
    L.afmm_batch_destroy.argtypes = [vp]
    L.afmm_hierarchy_check.argtypes = [C.POINTER(HierarchyC), C.POINTER(Options), C.POINTER(PlanInfo)]
    L.afmm_plan_set_profiling.argtypes = [vp, C.c_int32]
    L.afmm_plan_get_profile.argtypes = [vp, C.POINTER(StageTime), C.c_int32, C.POINTER(C.c_int32)]
    L.afmm_batch_set_profiling.argtypes = [vp, C.c_int32]
    L.afmm_batch_get_profile.argtypes = [vp, C.POINTER(StageTime), C.c_int32, C.POINTER(C.c_int32)]
    L.afmm_plan_autotune.argtypes = [vp, vp, vp, vp, vp, C.POINTER(TuneResult)]
    L.afmm_batch_autotune.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp, C.POINTER(TuneResult)]
    L.afmm_particle_hierarchy_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int64, vp, C.c_double,
                                                 C.POINTER(vp)]
    L.afmm_particle_hierarchy_view.argtypes = [vp, C.POINTER(HierarchyC)]
    L.afmm_particle_hierarchy_destroy.argtypes = [vp]
    L.afmm_cic_deposit.argtypes = [vp, C.c_int32, C.c_int64, vp, vp, vp, vp]
    L.afmm_cic_interpolate.argtypes = [vp, C.c_int32, C.c_int64, vp, vp, vp, vp, vp, vp]
    L.afmm_particles_update.argtypes = [C.c_int64, C.c_double, vp, vp, vp]
    L.afmm_status_string.argtypes = [C.c_int32]
    L.afmm_status_string.restype = C.c_char_p
    L.afmm_last_error.argtypes = []
    L.afmm_last_error.restype = C.c_char_p
    for name in ("afmm_plan_create", "afmm_plan_destroy", "afmm_plan_get_info", "afmm_solve",
                 "afmm_solve_adjoint", "afmm_solve_adjoint_noalloc", "afmm_batch_create", "afmm_batch_solve", "afmm_batch_get_info",
                 "afmm_batch_destroy", "afmm_hierarchy_check", "afmm_plan_set_profiling",
                 "afmm_plan_get_profile", "afmm_batch_set_profiling", "afmm_batch_get_profile",
                 "afmm_plan_autotune", "afmm_batch_autotune", "afmm_particle_hierarchy_create",
                 "afmm_particle_hierarchy_view", "afmm_particle_hierarchy_destroy", "afmm_cic_deposit",
                 "afmm_cic_interpolate", "afmm_particles_update", "afmm_plan_replan", "afmm_solve_drift",
                 "afmm_release_cached_memory"):
        getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def check(rc: int, what: str):
    if rc != AFMM_OK:
        detail = lib().afmm_last_error().decode(errors="replace")
        raise AfmmError(rc, what, detail)
