"""Seeded synthetic inputs: determinism, completeness, strong grading, counts."""
import numpy as np

from synth import configs, shuffle_order, unigrid
from synth.hierarchy import build_graded, check_graded, refine_sphere


def test_unigrid_and_cfg1():
    w = configs.cfg1()
    assert w.hierarchy.total == 32768 and w.hierarchy.nleaves() == 32768
    assert check_graded(w.hierarchy) is None
    w2 = configs.cfg1()
    np.testing.assert_array_equal(w.mass, w2.mass)
    assert abs(w.mass.sum() - 0.96) < 0.01


def test_cfg2_counts():
    h = configs.cfg2().hierarchy
    assert h.summary()["leaves"] == [258496, 29184]
    assert h.summary()["refined"] == [3648, 0]
    assert check_graded(h) is None


def test_grading_closure_small():
    h = build_graded(3, 6, refine_sphere((0.31, 0.52, 0.77), {3: 0.1, 4: 0.06, 5: 0.04}))
    assert check_graded(h) is None
    assert h.levelmax == 6
    hs = shuffle_order(h, 5)
    assert check_graded(hs) is None


def test_noise_is_seeded():
    a = configs.cfg2(base=4, seed=2).mass
    b = configs.cfg2(base=4, seed=2).mass
    c = configs.cfg2(base=4, seed=3).mass
    np.testing.assert_array_equal(a, b)
    assert np.any(a != c)
