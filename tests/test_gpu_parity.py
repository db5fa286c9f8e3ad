"""HIP path vs the FP64 oracle, element by element on the same seeded inputs.

Tolerances (relative L2 over the evaluated leaves, max-normalised at most 10x):
FP64 form 1e-10, FP32 mixed form 1e-4 (the stated force-error target).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import compare, gpu_solve, max_rel, rel_l2  # noqa: E402

import oracle  # noqa: E402
from synth import cell_masses, configs, plummer, shuffle_order, unigrid  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


def _amr(lmin, radii, centre=(0.5, 0.5, 0.5)):
    return build_graded(lmin, lmin + len(radii), refine_sphere(centre, radii))


@pytest.mark.parametrize("level", [1, 2, 3])
def test_tiny_unigrid_fp64(level):
    h = unigrid(level)
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, level)
    print(f"unigrid level {level}", flush=True)
    compare(h, m, 4, "fp64", 1e-12)


def test_cfg1_unigrid32_fp64_all_targets():
    w = configs.cfg1()
    print("cfg1 32^3 p=4 fp64", flush=True)
    ep, ea = compare(w.hierarchy, w.mass, w.p, "fp64", 1e-10)
    print("errors", ep, ea)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_small_amr_all_orders(p):
    h = _amr(3, {3: 0.3, 4: 0.2})
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, p)
    print(f"amr p={p}", flush=True)
    compare(h, m, p, "fp64", 1e-10)
    compare(h, m, p, "fp32", 1e-4)


_SPLIT_CASE = {}


def _split_case(p):
    """A two-level AMR hierarchy and its oracle solution, computed once per order."""
    if p not in _SPLIT_CASE:
        h = _amr(3, {3: 0.3, 4: 0.2})
        m = cell_masses(h, plummer(1.0, 0.1), 0.01, 40 + p)
        po, ao = oracle.Oracle(h, p).solve_all(m)
        _SPLIT_CASE[p] = (h, m, po, ao)
    return _SPLIT_CASE[p]


@pytest.mark.parametrize("p", [4, 6])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("split", [1, 2, 3, 7, 21])
def test_explicit_tap_splits(p, precision, split):
    """Every tap split (1 to 21 blocks per tile, ranges of 8 to 189 taps, the
    per-launch LDS source table of M2P sized from them) against the oracle."""
    h, m, po, ao = _split_case(p)
    print(f"tap split {split} p={p} {precision}", flush=True)
    phi, acc, _ = gpu_solve(h, m, p, precision, tap_split=split)
    leaf = h.leaf_mask()
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert rel_l2(acc[leaf], ao[leaf]) <= tol and rel_l2(phi[leaf], po[leaf]) <= tol
    assert max_rel(acc[leaf], ao[leaf]) <= 10 * tol
    # a split changes only the order of the partial sums
    phi1, acc1, _ = gpu_solve(h, m, p, precision, tap_split=1)
    assert rel_l2(acc[leaf], acc1[leaf]) <= (1e-13 if precision == "fp64" else 1e-5)


def test_three_level_amr_fp32_and_fp64():
    h = _amr(4, {4: 0.25, 5: 0.15, 6: 0.08})
    m = cell_masses(h, plummer(1.0, 0.05), 0.01, 9)
    print("amr 4+3", flush=True)
    compare(h, m, 6, "fp64", 1e-10)
    compare(h, m, 6, "fp32", 1e-4)


def test_refinement_touching_box_corner_and_shuffled_order():
    h = shuffle_order(_amr(3, {3: 0.35, 4: 0.2, 5: 0.1}, centre=(0.02, 0.03, 0.97)), 17)
    m = cell_masses(h, plummer(1.0, 0.1, (0.1, 0.1, 0.9)), 0.01, 4)
    print("corner amr", flush=True)
    compare(h, m, 5, "fp64", 1e-10)
    compare(h, m, 5, "fp32", 1e-4)


def test_cfg2_full_size_sampled():
    w = configs.cfg2()
    print("cfg2 fp32 sampled", flush=True)
    ep, ea = compare(w.hierarchy, w.mass, w.p, "fp32", 1e-4, sample=1500, seed=2)
    print("fp32 errors", ep, ea)
    ep, ea = compare(w.hierarchy, w.mass, w.p, "fp64", 1e-10, sample=600, seed=3)
    print("fp64 errors", ep, ea)


def test_nearest_pair_antisymmetry_gpu():
    from test_oracle_fmm import _nearest_pair
    h = _amr(4, {4: 0.25, 5: 0.12})
    ci, fi = _nearest_pair(h)
    m = np.zeros(h.total)
    m[ci], m[fi] = 0.7, 0.3
    for prec, tol in (("fp64", 1e-14), ("fp32", 1e-6)):
        phi, acc, _ = gpu_solve(h, m, 6, prec)
        mom = m[ci] * acc[ci] + m[fi] * acc[fi]
        assert np.linalg.norm(mom) <= tol * m[ci] * np.linalg.norm(acc[ci]), prec


def test_deterministic_and_untouched_entries():
    import torch as T
    import paper_2607_19489_amd as A
    h = _amr(3, {3: 0.3, 4: 0.2})
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 1)
    plan = A.Plan(h, p=6, precision="fp32")
    mt = T.from_numpy(m).cuda()
    phi1 = T.full((h.total,), 7.0, dtype=T.float64, device="cuda")
    acc1 = T.full((h.total, 3), 7.0, dtype=T.float64, device="cuda")
    plan.solve(mt, phi=phi1, acc=acc1)
    phi2, acc2 = plan.solve(mt)
    T.cuda.synchronize()
    leaf = T.from_numpy(h.leaf_mask()).cuda()
    assert T.equal(phi1[leaf], phi2[leaf]) and T.equal(acc1[leaf], acc2[leaf])
    assert bool((phi1[~leaf] == 7.0).all()) and bool((acc1[~leaf] == 7.0).all())
    # the two-stream schedule, serial launches and profiled solves run the same arithmetic
    plan_s = A.Plan(h, p=6, precision="fp32", serial=True)
    phi3, acc3 = plan_s.solve(mt)
    plan_o = A.Plan(h, p=6, precision="fp32", overlap=True)
    phi5, acc5 = plan_o.solve(mt)
    T.cuda.synchronize()
    assert T.equal(phi5[leaf], phi2[leaf]) and T.equal(acc5[leaf], acc2[leaf])
    plan.set_profiling(True)
    phi4, acc4 = plan.solve(mt)
    T.cuda.synchronize()
    prof = plan.get_profile()
    assert T.equal(phi3[leaf], phi2[leaf]) and T.equal(acc3[leaf], acc2[leaf])
    assert T.equal(phi4[leaf], phi2[leaf]) and T.equal(acc4[leaf], acc2[leaf])
    assert prof["upward"]["launches"] >= 1 and sum(v["ms"] for v in prof.values()) > 0
    assert any(k.startswith("near_") for k in prof) and any(k.startswith("m2p_") for k in prof)


def test_ats_sequence_matches_oracle():
    import paper_2607_19489_amd as A
    h = _amr(3, {3: 0.3, 4: 0.2})
    rng = np.random.default_rng(4)
    m0 = cell_masses(h, plummer(1.0, 0.1), 0.01, 1)
    seq = [(3, 1), (4, 1), (5, 1), (5, 2), (4, 2), (5, 1), (5, 2)]
    plan = A.Plan(h, p=4, precision="fp64")
    o = oracle.Oracle(h, 4)
    N = h.total
    po = np.zeros(N)
    ao = np.zeros((N, 3))
    lev = h.level_of()
    m = m0.copy()
    for (l, ic) in seq:
        m = m * (1 + 1e-3 * rng.uniform(-1, 1, N))
        phi, acc, _ = gpu_solve(h, m, 4, level=l, icount=ic, plan=plan)
        o.solve(l, ic, m, po, ao)
        sel = (lev == l) & h.leaf_mask()
        assert rel_l2(acc[sel], ao[sel]) < 1e-10, (l, ic)
        assert rel_l2(phi[sel], po[sel]) < 1e-10, (l, ic)
    mt = torch.from_numpy(m).cuda()
    for bad in ((4, 0), (2, 1), (6, 1)):
        with pytest.raises(A.AfmmError):
            plan.solve(mt, level=bad[0], icount=bad[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_level_solve_without_rebuild_reproduces_the_full_solve(precision):
    """Alg. 1: solve(l, icount=1) for l > levelmin rebuilds no tree, so right after a
    full solve it must give the full solve's level-l values whatever masses it is
    handed: the device keeps the trees, and the level's restricted M2L/L2L chain
    computes every needed local expansion with the same per-column arithmetic."""
    import paper_2607_19489_amd as A
    h = _amr(4, {4: 0.25, 5: 0.15, 6: 0.08})
    m = cell_masses(h, plummer(1.0, 0.05), 0.01, 21)
    plan = A.Plan(h, p=5, precision=precision, tap_split=2)
    phi, acc, _ = gpu_solve(h, m, 5, plan=plan)
    lev = h.level_of()
    junk = m * 3.0 + 1.0
    for l in (5, 6, 7):
        pl, al, _ = gpu_solve(h, junk, 5, level=l, icount=1, plan=plan)
        sel = (lev == l) & h.leaf_mask()
        assert sel.any()
        assert np.array_equal(pl[sel], phi[sel]) and np.array_equal(al[sel], acc[sel]), l
    # a rebuild (icount 2) takes the new masses of levels >= l: level l changes
    pl, al, _ = gpu_solve(h, junk, 5, level=6, icount=2, plan=plan)
    sel = (lev == 6) & h.leaf_mask()
    assert not np.allclose(al[sel], acc[sel])
