"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same input.

Error metrics (over the evaluated leaves):
  rel_l2        ||x - x_ref|| / ||x_ref||                 (gate: 1e-10 FP64, 1e-4 FP32)
  max_rel       max |x - x_ref| / max |x_ref|              (at most 10x the gate)
  p99_cell      99th percentile of |a_i - a_ref_i| / |a_ref_i| over cells (at most 10x the gate)
The FP32 form also has a regression bound far below its gate: the mixed path
measures a few 1e-7 of relative L2 force error, so an FP32-only defect that
stays under 1e-4 still fails at FP32_REGRESSION.
"""
import numpy as np
import torch

import oracle
import paper_2607_19489_amd as A

FP32_REGRESSION = 5e-6


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def p99_cell(a, b):
    """99th percentile of the per-cell relative error of vectors (rows) or scalars."""
    if a.ndim == 1:
        d, r = np.abs(a - b), np.abs(b)
    else:
        d, r = np.linalg.norm(a - b, axis=1), np.linalg.norm(b, axis=1)
    ok = r > 0
    return float(np.percentile(d[ok] / r[ok], 99)) if ok.any() else 0.0


def gate(precision):
    return 1e-10 if precision == "fp64" else 1e-4


def check_errors(phi, acc, po, ao, precision, tol=None, regression=True, what=""):
    """Assert the error bars of one comparison; returns the measured metrics."""
    tol = gate(precision) if tol is None else tol
    e = {"rel_l2_acc": rel_l2(acc, ao), "rel_l2_phi": rel_l2(phi, po), "max_rel_acc": max_rel(acc, ao),
         "p99_cell_acc": p99_cell(acc, ao), "p99_cell_phi": p99_cell(phi, po)}
    print(f"{what} {precision}: " + " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert e["rel_l2_acc"] <= tol, (what, e)
    assert e["rel_l2_phi"] <= tol, (what, e)
    assert e["max_rel_acc"] <= 10 * tol, (what, e)
    assert e["p99_cell_acc"] <= 10 * tol, (what, e)
    if precision == "fp32" and regression:
        assert e["rel_l2_acc"] <= FP32_REGRESSION and e["rel_l2_phi"] <= FP32_REGRESSION, (what, e)
    return e


def gpu_solve(h, m, p, precision="fp64", level=A.AFMM_ALL_LEVELS, icount=1, plan=None, **kw):
    plan = plan or A.Plan(h, p=p, precision=precision, **kw)
    mt = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    phi, acc = plan.solve(mt, level=level, icount=icount)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), acc.cpu().numpy(), plan


def compare(h, m, p, precision, tol, sample=None, seed=0, oracle_kw=None, regression=True, **plan_kw):
    """GPU full solve vs oracle on all leaves (or a seeded sample of leaves)."""
    phi, acc, _ = gpu_solve(h, m, p, precision, **plan_kw)
    o = oracle.Oracle(h, p, **(oracle_kw or {}))
    leaf = np.nonzero(h.leaf_mask())[0]
    if sample is None or sample >= leaf.size:
        po, ao = o.solve_all(m)
        sel = leaf
        po, ao = po[sel], ao[sel]
    else:
        o.rebuild(h.levelmin, m)
        rng = np.random.default_rng(seed)
        sel = np.sort(rng.choice(leaf, size=sample, replace=False))
        po, ao = o.eval_sample(sel)
    e = check_errors(phi[sel], acc[sel], po, ao, precision, tol, regression=regression,
                     what=f"{h.levelmin}..{h.levelmax} p={p}")
    return e["rel_l2_phi"], e["rel_l2_acc"]
