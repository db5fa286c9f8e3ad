"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
its host-only validation returns the documented status codes and counts."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2607_19489_amd as A
from paper_2607_19489_amd import _lib
from synth import configs, unigrid
from synth.hierarchy import Hierarchy, build_graded, refine_sphere

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "afmm.h")).read()
    return sorted(set(re.findall(r"\b(afmm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.SYMBOLS) == names


def test_status_strings():
    L = _lib.lib()
    assert L.afmm_status_string(-2) == b"hierarchy not graded"
    assert L.afmm_status_string(0) == b"ok"


def _chain(levelmin, depth):
    from test_oracle_fmm import _single_chain
    return _single_chain(levelmin, depth)


def test_validation_codes():
    A.hierarchy_check(_chain(3, 1))
    with pytest.raises(A.AfmmError) as e:
        A.hierarchy_check(_chain(3, 2))
    assert e.value.code == -2
    h = build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {3: 0.3, 4: 0.2}))
    inc = Hierarchy(h.levelmin, h.levelmax, [h.ijk[0], h.ijk[1][1:], h.ijk[2]],
                    [h.refined[0], h.refined[1][1:], h.refined[2]])
    with pytest.raises(A.AfmmError) as e:
        A.hierarchy_check(inc)
    assert e.value.code == -3
    bad = Hierarchy(h.levelmin, h.levelmax, [a.copy() for a in h.ijk], [r.copy() for r in h.refined])
    bad.ijk[0][0, 0] = 99
    with pytest.raises(A.AfmmError) as e:
        A.hierarchy_check(bad)
    assert e.value.code == -1
    with pytest.raises(A.AfmmError) as e:
        A.hierarchy_check(h, p=9)
    assert e.value.code == -4


def test_validation_reports_the_first_bad_cell_in_cell_order():
    # the host checks run over ranges of cells on several threads; the error
    # names the first offending cell whichever range finds it
    u = unigrid(6)
    for first, second in ((50000, 200000), (3, 262000), (131071, 131072)):
        bad = Hierarchy(u.levelmin, u.levelmax, [a.copy() for a in u.ijk], [r.copy() for r in u.refined])
        bad.ijk[0][second, 1] = 64
        bad.ijk[0][first, 2] = -1
        with pytest.raises(A.AfmmError) as e:
            A.hierarchy_check(bad)
        assert e.value.code == -1 and f"cell {first} of level 6 out of range" in str(e.value), str(e.value)


def test_counts_unigrid():
    info = A.hierarchy_check(unigrid(5), p=4)
    assert info["nleaves"] == 32768 and info["nrefined"] == 0
    # every leaf: 189 (interior) or fewer intermediate sources; near P2P <= 215
    assert 0 < info["m2p_pairs"] <= 32768 * 189
    assert info["p2p_pairs"] <= 32768 * 215
    assert info["nearest_pairs"] == 0 and info["near_m2p_pairs"] == 0
    # a 4^3 grid is near field only
    i2 = A.hierarchy_check(unigrid(2), p=4)
    assert i2["m2p_pairs"] == 0 and i2["p2p_pairs"] == 64 * 63


def test_counts_cfg2():
    info = A.hierarchy_check(configs.cfg2().hierarchy, p=6)
    assert info["nleaves"] == 287680 and info["nrefined"] == 3648
    assert info["nearest_pairs"] > 0 and info["near_m2p_pairs"] > 0


def test_model_flags_accepted_and_unknown_flag_refused():
    h = build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {3: 0.3, 4: 0.2}))
    a = A.hierarchy_check(h, p=3)
    b = A.hierarchy_check(h, p=3, quad_cap=True, self_potential=True)
    assert a["nleaves"] == b["nleaves"] and a["flops_m2p"] == b["flops_m2p"]
    o = A.make_options(p=3)
    o.flags = 1 << 9
    arrs = A.afmm._hierarchy_arrays(h)  # kept alive: hc points into them
    hc = A.afmm._hier_struct(*arrs)
    info = _lib.PlanInfo()
    assert _lib.lib().afmm_hierarchy_check(C.byref(hc), C.byref(o), C.byref(info)) == -4


def test_max_device_bytes_gives_out_of_memory_before_any_device_call():
    """A cap smaller than the first allocation fails plan creation with
    AFMM_E_OUT_OF_MEMORY; the check precedes hipMalloc, so it runs without a GPU."""
    h = build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {3: 0.3, 4: 0.2}))
    o = A.make_options(p=4, max_device_bytes=1)
    arrs = A.afmm._hierarchy_arrays(h)
    hc = A.afmm._hier_struct(*arrs)
    ptr = C.c_void_p()
    rc = _lib.lib().afmm_plan_create(C.byref(hc), C.byref(o), None, C.byref(ptr))
    assert rc == -5 and not ptr.value
    assert b"max_device_bytes" in _lib.lib().afmm_last_error()


def test_release_of_an_empty_buffer_cache_touches_no_device():
    """afmm_release_cached_memory with nothing cached returns AFMM_OK without a GPU,
    also when called twice (the capped plan above never put a buffer in the cache)."""
    assert _lib.lib().afmm_release_cached_memory() == 0
    A.release_cached_memory()


def test_m2p_shape_option_validated():
    h = build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {3: 0.3, 4: 0.2}))
    a = A.hierarchy_check(h, p=4, precision="fp32")
    for shape in (1, 2, 3):
        assert A.hierarchy_check(h, p=4, precision="fp32", m2p_shape=shape)["flops_m2p"] == a["flops_m2p"]
    # an unsupported combination (two tiles per wave at p = 8, FP64) falls back to shape 0 at plan time
    assert A.hierarchy_check(h, p=8, m2p_shape=2)["nleaves"] == a["nleaves"]
    for bad in (-1, 4):
        with pytest.raises(A.AfmmError):
            A.hierarchy_check(h, p=4, m2p_shape=bad)


def test_periodic_hierarchy_validation_and_counts():
    """Periodic boxes: neighbour lists wrap, so every leaf of a unigrid has all
    189 interaction-list sources and 215 near neighbours; levelmin < 3 and a
    hierarchy graded only inside the box are refused."""
    i3 = A.hierarchy_check(unigrid(3), p=4, periodic=True)
    assert i3["m2p_pairs"] == 512 * 189 and i3["p2p_pairs"] == 512 * 215
    i4 = A.hierarchy_check(unigrid(4), p=4, periodic=True)
    assert i4["m2l_targets"] == 512 and i4["m2l_pairs"] == 512 * 189 and i4["p2p_pairs"] == 4096 * 215
    iso = A.hierarchy_check(unigrid(3), p=4)
    assert iso["m2p_pairs"] < i3["m2p_pairs"]
    with pytest.raises(A.AfmmError, match="UNSUPPORTED"):
        A.hierarchy_check(unigrid(2), p=4, periodic=True)

    def face(level, ijk, h):
        x = (ijk.astype(np.float64) + 0.5) * h
        r = {3: 0.2, 4: 0.1}.get(level)
        if r is None:
            return np.zeros(len(x), bool)
        return (x[:, 0] < r) & (np.abs(x[:, 1] - 0.5) < 0.2) & (np.abs(x[:, 2] - 0.5) < 0.2)
    with pytest.raises(A.AfmmError, match="NOT_GRADED"):
        A.hierarchy_check(build_graded(3, 5, face), p=4, periodic=True)
    assert A.hierarchy_check(build_graded(3, 5, face, periodic=True), p=4, periodic=True)["nleaves"] > 0
