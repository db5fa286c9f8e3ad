"""Adjoint (transposed FMM) pass: dot-product identity, oracle column probes,
autograd against central finite differences, adaptive-time-step adjoint.

The forward map m -> (phi, a) is linear, so <A m, bar> = <m, A^T bar> must
hold to round-off for the adjoint of the FP64 form; the oracle pins A^T
independently through unit-mass columns: (A^T bar)_i = <A e_i, bar>.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, plummer, shuffle_order, unigrid  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


def _amr(lmin, radii, centre=(0.5, 0.5, 0.5)):
    return build_graded(lmin, lmin + len(radii), refine_sphere(centre, radii))


CASES = {
    "unigrid3": lambda: unigrid(3),
    "amr3+2": lambda: _amr(3, {3: 0.3, 4: 0.2}),
    "amr4+3": lambda: _amr(4, {4: 0.25, 5: 0.15, 6: 0.08}),
    "corner": lambda: shuffle_order(_amr(3, {3: 0.35, 4: 0.2, 5: 0.1}, centre=(0.02, 0.03, 0.97)), 17),
}


def _bars(h, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(h.total), rng.standard_normal((h.total, 3))


def _adjoint(plan, m, pb, ab, level=A.AFMM_ALL_LEVELS, icount=1):
    mt = torch.from_numpy(m).cuda()
    phi, acc = plan.solve(mt, level=level, icount=icount)
    mb = plan.solve_adjoint(torch.from_numpy(pb).cuda(), torch.from_numpy(ab).cuda(), level=level)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), acc.cpu().numpy(), mb.cpu().numpy()


@pytest.mark.parametrize("name,p", [("unigrid3", 4), ("amr3+2", 1), ("amr3+2", 3), ("amr3+2", 6), ("amr3+2", 8),
                                    ("amr4+3", 6), ("corner", 5)])
def test_dot_product_identity(name, p):
    h = CASES[name]()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 3)
    pb, ab = _bars(h, 4)
    print(f"adjoint dot {name} p={p}", flush=True)
    plan = A.Plan(h, p=p, precision="fp64")
    phi, acc, mb = _adjoint(plan, m, pb, ab)
    leaf = h.leaf_mask()
    assert np.all(mb[~leaf] == 0.0)
    lhs = float(np.dot(phi[leaf], pb[leaf]) + np.sum(acc[leaf] * ab[leaf]))
    rhs = float(np.dot(m[leaf], mb[leaf]))
    scale = float(np.dot(np.abs(phi[leaf]), np.abs(pb[leaf])) + np.sum(np.abs(acc[leaf] * ab[leaf])))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    # the FP32 form transposes the same operator (its M2P^T / M2L^T run in FP32
    # MFMA below the FP64 levels, like the forward)
    plan32 = A.Plan(h, p=p, precision="fp32", fp64_levels=2)
    phi32, acc32, mb32 = _adjoint(plan32, m, pb, ab)
    assert np.linalg.norm(mb32[leaf] - mb[leaf]) <= 1e-5 * np.linalg.norm(mb[leaf])
    lhs32 = float(np.dot(phi32[leaf], pb[leaf]) + np.sum(acc32[leaf] * ab[leaf]))
    rhs32 = float(np.dot(m[leaf], mb32[leaf]))
    assert abs(lhs32 - rhs32) <= 1e-5 * scale


@pytest.mark.parametrize("name,p", [("amr3+2", 4), ("corner", 6)])
def test_oracle_column_probes(name, p):
    h = CASES[name]()
    pb, ab = _bars(h, 8)
    plan = A.Plan(h, p=p, precision="fp64")
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 3)
    _, _, mb = _adjoint(plan, m, pb, ab)
    leaf = np.nonzero(h.leaf_mask())[0]
    rng = np.random.default_rng(9)
    o = oracle.Oracle(h, p)
    print(f"column probes {name} p={p}", flush=True)
    lm = h.leaf_mask()
    for i in rng.choice(leaf, size=6, replace=False):
        e = np.zeros(h.total)
        e[i] = 1.0
        po, ao = o.solve_all(e)
        want = float(np.dot(po[lm], pb[lm]) + np.sum(ao[lm] * ab[lm]))
        scale = float(np.dot(np.abs(po[lm]), np.abs(pb[lm])) + np.sum(np.abs(ao[lm] * ab[lm])))
        assert abs(mb[i] - want) <= 1e-10 * scale, (i, mb[i], want)


def test_autograd_energy_and_force_loss_vs_finite_differences():
    h = CASES["amr3+2"]()
    m0 = cell_masses(h, plummer(1.0, 0.1), 0.01, 5)
    plan = A.Plan(h, p=6, precision="fp64")
    leaf_np = h.leaf_mask()
    leaf = torch.from_numpy(leaf_np).cuda()
    rng = np.random.default_rng(5)
    target = torch.from_numpy(rng.standard_normal((h.total, 3)) * 0.1).cuda()

    def energy(mt):
        phi, _ = A.solve(mt, plan)
        return 0.5 * torch.sum(torch.where(leaf, mt * phi, torch.zeros_like(phi)))

    def force_loss(mt):
        _, acc = A.solve(mt, plan)
        d = (acc - target)[leaf]
        return torch.mean(d * d)

    for fn, name in ((energy, "W"), (force_loss, "mse")):
        mt = torch.from_numpy(m0).cuda().requires_grad_(True)
        val = fn(mt)
        val.backward()
        g = mt.grad.detach().cpu().numpy()
        assert np.all(g[~leaf_np] == 0.0)
        cells = rng.choice(np.nonzero(leaf_np)[0], size=8, replace=False)
        hstep = 1e-4
        for i in cells:
            mp, mm = m0.copy(), m0.copy()
            mp[i] += hstep
            mm[i] -= hstep
            with torch.no_grad():
                fd = (fn(torch.from_numpy(mp).cuda()) - fn(torch.from_numpy(mm).cuda())).item() / (2 * hstep)
            assert abs(g[i] - fd) <= 1e-7 * max(1.0, abs(fd)), (name, i, g[i], fd)
        print(f"{name}: grad ok on {cells.size} cells", flush=True)
    # dW/dm = (phi + A^T m)/2 differs from phi (the FMM operator is not symmetric)
    mt = torch.from_numpy(m0).cuda().requires_grad_(True)
    energy(mt).backward()
    phi, _ = plan.solve(torch.from_numpy(m0).cuda())
    gap = (mt.grad - phi)[leaf].abs().max().item()
    assert gap > 1e-9 * phi[leaf].abs().max().item()


def test_adaptive_time_step_adjoint():
    h = CASES["amr4+3"]()
    lmin, lmax = h.levelmin, h.levelmax
    m_old = cell_masses(h, plummer(1.0, 0.1), 0.01, 6)
    m_new = m_old * (1.0 + 0.01 * np.random.default_rng(7).standard_normal(h.total))
    plan = A.Plan(h, p=5, precision="fp64")
    plan.solve(torch.from_numpy(m_old).cuda(), level=lmin, icount=1)
    lev = lmin + 1
    pb, ab = _bars(h, 11)
    phi1, acc1, mb = _adjoint(plan, m_new, pb, ab, level=lev, icount=2)
    lv = h.level_of()
    assert np.all(mb[lv < lev] == 0.0)
    rng = np.random.default_rng(12)
    delta = np.where(lv >= lev, rng.standard_normal(h.total) * 1e-3, 0.0)
    phi2, acc2, _ = _adjoint(plan, m_new + delta, pb, ab, level=lev, icount=2)
    sel = (lv == lev) & h.leaf_mask()
    lhs = float(np.dot(phi2[sel] - phi1[sel], pb[sel]) + np.sum((acc2[sel] - acc1[sel]) * ab[sel]))
    rhs = float(np.dot(delta, mb))
    assert abs(lhs - rhs) <= 1e-9 * max(abs(rhs), 1e-30), (lhs, rhs)
    with pytest.raises(A.AfmmError):
        plan.solve_adjoint(torch.from_numpy(pb).cuda(), torch.from_numpy(ab).cuda(), level=A.AFMM_ALL_LEVELS)
