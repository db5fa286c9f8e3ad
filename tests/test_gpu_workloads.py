"""The measured workloads at full size against the FP64 oracle.

- Deep AMR (level 7 base + 4 mass-refined levels, about 8.08M leaves, p = 6):
  a seeded sample of 450 leaves on every level 7..11 (2,250 leaves), FP32 mixed
  and FP64 forms, with the launch configuration the benchmark times (autotuned
  tap splits).
- Adaptive time steps in the FP32 form with rebuilds (icount = 2) against
  Alg. 1 run by the oracle on the same mass sequence.
- The FP32 adjoint: oracle unit-mass column probes (A^T bar)_i = <A e_i, bar>.
- Differentiation workload (level 7 + r < 0.2 + r < 0.1, 3,081,632 leaves, p = 6,
  FP32): autograd of W = 1/2 sum m phi and of an MSE loss on accelerations
  against central finite differences (h = 1e-4) on 64 seeded cells.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import FP32_REGRESSION, check_errors, gpu_solve, rel_l2  # noqa: E402

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, configs, plummer  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


@pytest.fixture(scope="module")
def deep():
    print("generating the deep AMR workload", flush=True)
    return configs.cfg3()


@pytest.mark.timeout(900)
def test_deep_amr_full_size_sampled_every_level(deep):
    h, m = deep.hierarchy, deep.mass
    lev, leaf = h.level_of(), h.leaf_mask()
    rng = np.random.default_rng(7)
    sel = np.concatenate([np.sort(rng.choice(np.nonzero(leaf & (lev == l))[0], 450, replace=False))
                          for l in range(h.levelmin, h.levelmax + 1)])
    assert sel.size >= 2000 and set(np.unique(lev[sel])) == set(range(7, 12))
    mt = torch.from_numpy(m).cuda()
    outs = {}
    for prec in ("fp32", "fp64"):
        print(f"deep AMR {prec}: plan + autotune + solve", flush=True)
        plan = A.Plan(h, p=deep.p, precision=prec)
        plan.autotune(mt)
        phi, acc = plan.solve(mt)
        torch.cuda.synchronize()
        outs[prec] = (phi.cpu().numpy()[sel], acc.cpu().numpy()[sel])
        plan.close()
        del phi, acc
    print("oracle rebuild + sample", flush=True)
    o = oracle.Oracle(h, deep.p)
    o.rebuild(h.levelmin, m)
    po, ao = o.eval_sample(sel)
    for prec, (phi, acc) in outs.items():
        check_errors(phi, acc, po, ao, prec, what="deep AMR sample")
        for l in range(h.levelmin, h.levelmax + 1):  # every level on its own
            s = lev[sel] == l
            assert rel_l2(acc[s], ao[s]) <= (FP32_REGRESSION if prec == "fp32" else 1e-10), (prec, l)


def _amr(lmin, radii):
    return build_graded(lmin, lmin + len(radii), refine_sphere((0.5, 0.5, 0.5), radii))


def test_fp32_ats_sequence_with_rebuilds_matches_oracle():
    h = _amr(4, {4: 0.25, 5: 0.15, 6: 0.08})
    lmin = h.levelmin
    rng = np.random.default_rng(14)
    m = cell_masses(h, plummer(1.0, 0.05), 0.01, 13)
    # one coarse step of Alg. 1 with sub-cycling: each level-l step runs two level-(l+1) steps
    seq = []

    def rec(l, ic):
        seq.append((l, ic))
        if l < h.levelmax:
            rec(l + 1, 1)
            rec(l + 1, 2)
    rec(lmin, 1)
    assert sum(ic == 2 for _, ic in seq) >= 3
    plan = A.Plan(h, p=5, precision="fp32", fp64_levels=2)
    o = oracle.Oracle(h, 5)
    po, ao = np.zeros(h.total), np.zeros((h.total, 3))
    lev, leaf = h.level_of(), h.leaf_mask()
    for l, ic in seq:
        m = m * (1 + 1e-3 * rng.uniform(-1, 1, h.total))
        phi, acc, _ = gpu_solve(h, m, 5, level=l, icount=ic, plan=plan)
        o.solve(l, ic, m, po, ao)
        s = (lev == l) & leaf
        check_errors(phi[s], acc[s], po[s], ao[s], "fp32", what=f"ATS solve({l}, {ic})")


@pytest.mark.parametrize("p", [4, 6])
def test_fp32_adjoint_oracle_column_probes(p):
    h = _amr(3, {3: 0.3, 4: 0.2})
    rng = np.random.default_rng(20 + p)
    pb, ab = rng.standard_normal(h.total), rng.standard_normal((h.total, 3))
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 3)
    plan = A.Plan(h, p=p, precision="fp32", fp64_levels=2)
    plan.solve(torch.from_numpy(m).cuda())
    mb = plan.solve_adjoint(torch.from_numpy(pb).cuda(), torch.from_numpy(ab).cuda())
    torch.cuda.synchronize()
    mb = mb.cpu().numpy()
    o = oracle.Oracle(h, p)
    lm = h.leaf_mask()
    errs = []
    for i in rng.choice(np.nonzero(lm)[0], size=8, replace=False):
        e = np.zeros(h.total)
        e[i] = 1.0
        po, ao = o.solve_all(e)
        want = float(np.dot(po[lm], pb[lm]) + np.sum(ao[lm] * ab[lm]))
        scale = float(np.dot(np.abs(po[lm]), np.abs(pb[lm])) + np.sum(np.abs(ao[lm] * ab[lm])))
        errs.append(abs(mb[i] - want) / scale)
    print(f"fp32 adjoint column probes p={p}: max err / scale {max(errs):.2e}", flush=True)
    assert max(errs) <= FP32_REGRESSION


@pytest.mark.timeout(900)
def test_differentiation_workload_fp32_vs_finite_differences():
    """W = 1/2 sum m phi and MSE(a, a*) are quadratic in m, so central
    differences are exact up to rounding; the FP32 form's gradient must match
    them to 1e-3 (relative to the larger of |fd| and the gradient's rms)."""
    w = configs.cfg5()
    h, m0 = w.hierarchy, w.mass
    assert h.nleaves() == 3081632
    plan = A.Plan(h, p=w.p, precision="fp32")
    leaf_np = h.leaf_mask()
    leaf = torch.from_numpy(leaf_np).cuda()
    target_m = cell_masses(h, plummer(1.0, 0.05), 0.01, 55)
    _, a_star = plan.solve(torch.from_numpy(target_m).cuda())
    a_star = a_star.clone()
    nleaf = float(leaf_np.sum())

    def energy(mt):
        phi, _ = A.solve(mt, plan)
        return 0.5 * torch.sum(torch.where(leaf, mt * phi, torch.zeros_like(phi)))

    def force_loss(mt):
        _, acc = A.solve(mt, plan)
        d = torch.where(leaf[:, None], acc - a_star, torch.zeros_like(acc))
        return torch.sum(d * d) / nleaf

    rng = np.random.default_rng(5)
    cells = rng.choice(np.nonzero(leaf_np)[0], size=64, replace=False)
    hstep = 1e-4
    for fn, name in ((energy, "W"), (force_loss, "mse")):
        mt = torch.from_numpy(m0).cuda().requires_grad_(True)
        fn(mt).backward()
        g = mt.grad.detach().cpu().numpy()
        assert np.all(g[~leaf_np] == 0.0)
        rms = float(np.sqrt(np.mean(g[leaf_np] ** 2)))
        worst = 0.0
        for i in cells:
            mp, mm = m0.copy(), m0.copy()
            mp[i] += hstep
            mm[i] -= hstep
            with torch.no_grad():
                fd = (fn(torch.from_numpy(mp).cuda()).double() - fn(torch.from_numpy(mm).cuda()).double()).item()
            fd /= 2 * hstep
            err = abs(g[i] - fd) / max(abs(fd), rms)
            worst = max(worst, err)
            assert err <= 1e-3, (name, int(i), g[i], fd)
        print(f"{name}: 64 cells, worst |grad - fd| / max(|fd|, rms) = {worst:.2e}", flush=True)
