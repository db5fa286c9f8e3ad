"""Model options and error paths of the C ABI on the GPU.

- AFMM_PAPER_QUAD_CAP (the paper's expansion setting, Sec. 2: multipoles to
  order p - 1) and AFMM_SELF_POTENTIAL (reading R11) against the oracle with
  the same options, in both forms; the cap leaves accelerations bit for bit.
- AFMM_CHECK_INPUT -> AFMM_E_NONFINITE for a non-finite leaf mass that the
  solve reads, and no error for slots it does not read.
- AFMM_E_ATS_ORDER for level solves and adjoints before any tree exists.
- An autotune under a device-memory cap keeps a consistent plan (its next
  solve still matches the oracle).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import check_errors, gpu_solve  # noqa: E402

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, plummer  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


def _amr(lmin=3, radii=None):
    radii = radii or {3: 0.3, 4: 0.2}
    return build_graded(lmin, lmin + len(radii), refine_sphere((0.5, 0.5, 0.5), radii))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [3, 6])
def test_paper_quad_cap_matches_oracle(precision, p):
    h = _amr(4, {4: 0.25, 5: 0.12})
    m = cell_masses(h, plummer(1.0, 0.08), 0.01, 31 + p)
    leaf = h.leaf_mask()
    print(f"quad cap p={p} {precision}", flush=True)
    po, ao = oracle.Oracle(h, p, quad_cap=True).solve_all(m)
    phi, acc, _ = gpu_solve(h, m, p, precision, quad_cap=True, fp64_levels=2)
    check_errors(phi[leaf], acc[leaf], po[leaf], ao[leaf], precision, what="capped")
    # accelerations never see order-p multipoles: bit for bit the uncapped ones
    phi_u, acc_u, _ = gpu_solve(h, m, p, precision, fp64_levels=2)
    assert np.array_equal(acc_u[leaf], acc[leaf])
    assert np.linalg.norm(phi_u[leaf] - phi[leaf]) > 1e-9 * np.linalg.norm(phi[leaf])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_self_potential_matches_oracle(precision):
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 41)
    leaf = h.leaf_mask()
    po, ao = oracle.Oracle(h, 5, self_potential=True).solve_all(m)
    phi, acc, _ = gpu_solve(h, m, 5, precision, self_potential=True, fp64_levels=2)
    check_errors(phi[leaf], acc[leaf], po[leaf], ao[leaf], precision, what="self potential")
    phi0, acc0, _ = gpu_solve(h, m, 5, precision, fp64_levels=2)
    assert np.array_equal(acc0[leaf], acc[leaf])


def test_paper_setting_adjoint_dot_product():
    """The cap and the self term are linear in the masses: the adjoint of the
    plan with both options still satisfies <A m, bar> = <m, A^T bar>."""
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 43)
    rng = np.random.default_rng(44)
    pb, ab = rng.standard_normal(h.total), rng.standard_normal((h.total, 3))
    leaf = h.leaf_mask()
    plan = A.Plan(h, p=3, precision="fp64", quad_cap=True, self_potential=True)
    phi, acc = plan.solve(torch.from_numpy(m).cuda())
    mb = plan.solve_adjoint(torch.from_numpy(pb).cuda(), torch.from_numpy(ab).cuda())
    torch.cuda.synchronize()
    phi, acc, mb = phi.cpu().numpy(), acc.cpu().numpy(), mb.cpu().numpy()
    lhs = float(np.dot(phi[leaf], pb[leaf]) + np.sum(acc[leaf] * ab[leaf]))
    rhs = float(np.dot(m[leaf], mb[leaf]))
    scale = float(np.dot(np.abs(phi[leaf]), np.abs(pb[leaf])) + np.sum(np.abs(acc[leaf] * ab[leaf])))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)
    # column probe against the oracle with the same options: (A^T bar)_i = <A e_i, bar>
    o = oracle.Oracle(h, 3, quad_cap=True, self_potential=True)
    for i in rng.choice(np.nonzero(leaf)[0], size=3, replace=False):
        e = np.zeros(h.total)
        e[i] = 1.0
        po, ao = o.solve_all(e)
        want = float(np.dot(po[leaf], pb[leaf]) + np.sum(ao[leaf] * ab[leaf]))
        sc = float(np.dot(np.abs(po[leaf]), np.abs(pb[leaf])) + np.sum(np.abs(ao[leaf] * ab[leaf])))
        assert abs(mb[i] - want) <= 1e-10 * sc, (i, mb[i], want)


def test_check_input_nonfinite():
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 5)
    lev = h.level_of()
    leaf = h.leaf_mask()
    plan = A.Plan(h, p=4, precision="fp64", check_input=True)
    ref_phi, ref_acc, _ = gpu_solve(h, m, 4, plan=plan)
    bad = m.copy()
    i_leaf = int(np.nonzero(leaf & (lev == h.levelmin + 1))[0][0])
    bad[i_leaf] = np.nan
    with pytest.raises(A.AfmmError) as e:
        gpu_solve(h, bad, 4, plan=plan)
    assert e.value.code == -8
    inf = m.copy()
    inf[int(np.nonzero(leaf)[0][-1])] = np.inf
    with pytest.raises(A.AfmmError) as e:
        gpu_solve(h, inf, 4, plan=plan)
    assert e.value.code == -8
    # a refined cell's slot is never read: a NaN there is no error and changes nothing
    junk = m.copy()
    junk[int(np.nonzero(~leaf)[0][0])] = np.nan
    phi, acc, _ = gpu_solve(h, junk, 4, plan=plan)
    assert np.array_equal(phi[leaf], ref_phi[leaf]) and np.array_equal(acc[leaf], ref_acc[leaf])
    # Alg. 1 without a rebuild reads no mass at all
    phi, acc, _ = gpu_solve(h, bad, 4, level=h.levelmin + 1, icount=1, plan=plan)
    # a rebuilding level solve reads levels >= l only: a NaN below is ignored
    below = m.copy()
    below[int(np.nonzero(leaf & (lev == h.levelmin))[0][0])] = np.nan
    gpu_solve(h, below, 4, level=h.levelmin + 1, icount=2, plan=plan)
    with pytest.raises(A.AfmmError) as e:
        gpu_solve(h, bad, 4, level=h.levelmin + 1, icount=2, plan=plan)
    assert e.value.code == -8
    # the plan is still usable
    phi, acc, _ = gpu_solve(h, m, 4, plan=plan)
    assert np.array_equal(phi[leaf], ref_phi[leaf])


def test_ats_order_errors():
    h = _amr()
    m = torch.from_numpy(cell_masses(h, plummer(1.0, 0.1), 0.01, 6)).cuda()
    plan = A.Plan(h, p=4, precision="fp64")
    with pytest.raises(A.AfmmError) as e:
        plan.solve(m, level=h.levelmin + 1, icount=1)
    assert e.value.code == -7
    z = torch.zeros(h.total, dtype=torch.float64, device="cuda")
    z3 = torch.zeros(h.total, 3, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AfmmError) as e:
        plan.solve_adjoint(z, z3)
    assert e.value.code == -7
    plan.solve(m, level=h.levelmin, icount=1)
    plan.solve(m, level=h.levelmin + 1, icount=1)
    torch.cuda.synchronize()


def test_autotune_under_device_memory_cap():
    """A cap just above the plan's own memory: candidates whose partial buffers
    would not fit are skipped, the plan stays consistent, and the next solve
    matches the oracle."""
    h = _amr(4, {4: 0.25, 5: 0.12})
    m = cell_masses(h, plummer(1.0, 0.08), 0.01, 51)
    leaf = h.leaf_mask()
    po, ao = oracle.Oracle(h, 5).solve_all(m)
    for prec in ("fp64", "fp32"):
        probe = A.Plan(h, p=5, precision=prec, fp64_levels=2)
        need = probe.info()["device_bytes"]
        probe.close()
        plan = A.Plan(h, p=5, precision=prec, fp64_levels=2, max_device_bytes=need + 4096)
        mt = torch.from_numpy(m).cuda()
        res = plan.autotune(mt)
        assert plan.info()["device_bytes"] <= need + 4096
        assert res["candidates"] >= 1
        phi, acc, _ = gpu_solve(h, m, 5, plan=plan)
        check_errors(phi[leaf], acc[leaf], po[leaf], ao[leaf], prec, what=f"capped autotune {res}")
