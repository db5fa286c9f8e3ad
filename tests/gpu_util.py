"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same input."""
import numpy as np
import torch

import oracle
import paper_2607_19489_amd as A


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def gpu_solve(h, m, p, precision="fp64", level=A.AFMM_ALL_LEVELS, icount=1, plan=None, **kw):
    plan = plan or A.Plan(h, p=p, precision=precision, **kw)
    mt = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    phi, acc = plan.solve(mt, level=level, icount=icount)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), acc.cpu().numpy(), plan


def compare(h, m, p, precision, tol, sample=None, seed=0):
    """GPU full solve vs oracle on all leaves (or a seeded sample of leaves)."""
    phi, acc, _ = gpu_solve(h, m, p, precision)
    o = oracle.Oracle(h, p)
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
    ea = rel_l2(acc[sel], ao)
    ep = rel_l2(phi[sel], po)
    assert ea <= tol, f"force rel L2 {ea:.3e} > {tol:.1e}"
    assert ep <= tol, f"potential rel L2 {ep:.3e} > {tol:.1e}"
    assert max_rel(acc[sel], ao) <= 10 * tol
    return ep, ea
