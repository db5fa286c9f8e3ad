"""Autotuner of the tap splits: every candidate is a valid configuration, the
chosen one reproduces the solve (up to FP rounding order) and the oracle, and
a tuned batch still matches its members' solves."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import max_rel, rel_l2  # noqa: E402

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, configs, plummer  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


def _amr():
    return build_graded(4, 7, refine_sphere((0.5, 0.5, 0.5), {4: 0.25, 5: 0.15, 6: 0.08}))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_plan_autotune(precision, tol):
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.05), 0.01, 9)
    mt = torch.from_numpy(m).cuda()
    plan = A.Plan(h, p=6, precision=precision)
    phi0, acc0 = plan.solve(mt)
    res = plan.autotune(mt)
    print(precision, res, flush=True)
    for k in ("m2l_split", "m2p_split"):
        assert all(1 <= v <= 21 for v in res[k])
    assert res["ms_after"] > 0 and res["candidates"] >= 10
    phi1, acc1 = plan.solve(mt)
    torch.cuda.synchronize()
    leaf = h.leaf_mask()
    a0, a1 = acc0.cpu().numpy()[leaf], acc1.cpu().numpy()[leaf]
    assert rel_l2(a1, a0) <= (1e-13 if precision == "fp64" else 1e-6)
    po, ao = oracle.Oracle(h, 6).solve_all(m)
    assert rel_l2(a1, ao[leaf]) <= tol and max_rel(a1, ao[leaf]) <= 10 * tol
    assert rel_l2(phi1.cpu().numpy()[leaf], po[leaf]) <= tol
    # the adjoint follows the tuned plan
    pb = torch.randn(h.total, dtype=torch.float64, device="cuda")
    ab = torch.randn(h.total, 3, dtype=torch.float64, device="cuda")
    mb = plan.solve_adjoint(pb, ab)
    torch.cuda.synchronize()
    assert torch.isfinite(mb).all()


def test_batch_autotune():
    ws = [configs.cfg4_member(i, p=4, base_choices=(3, 4), max_extra=2) for i in range(5)]
    plans = [A.Plan(w.hierarchy, p=4, precision="fp64") for w in ws]
    batch = A.Batch(plans)
    masses = [torch.from_numpy(w.mass).cuda() for w in ws]
    res = batch.autotune(masses)
    print("batch", res, flush=True)
    phis, accs = batch.solve(masses)
    for i, pl in enumerate(plans):
        phi, acc = pl.solve(masses[i])
        torch.cuda.synchronize()
        leaf = ws[i].hierarchy.leaf_mask()
        assert rel_l2(accs[i].cpu().numpy()[leaf], acc.cpu().numpy()[leaf]) <= 1e-13
        assert rel_l2(phis[i].cpu().numpy()[leaf], phi.cpu().numpy()[leaf]) <= 1e-13


def test_level_solve_after_autotune_matches_oracle():
    """The autotuner's solves rebuild every tree from the tuned masses: a level
    solve without a rebuild right after it evaluates those trees."""
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.05), 0.01, 13)
    plan = A.Plan(h, p=5, precision="fp64")
    plan.autotune(torch.from_numpy(m).cuda())
    o = oracle.Oracle(h, 5)
    o.rebuild(h.levelmin, m)
    lev = h.level_of()
    for l in (5, 6):
        phi, acc = plan.solve(torch.from_numpy(m * 2.0).cuda(), level=l, icount=1)
        torch.cuda.synchronize()
        sel = np.nonzero((lev == l) & h.leaf_mask())[0]
        po, ao = o.eval(l, sel)
        assert rel_l2(acc.cpu().numpy()[sel], ao) <= 1e-10 and rel_l2(phi.cpu().numpy()[sel], po) <= 1e-10
