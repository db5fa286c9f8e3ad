"""Device buffers of destroyed plans are kept by the library and handed to later
plans.  A plan built on buffers that an earlier plan of another hierarchy
filled must solve bit for bit like one built on fresh buffers (nothing may
depend on what the memory held), also across re-plans and batches; a plan with
a device-byte cap still counts exactly what it asks for.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import check_errors  # noqa: E402

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, plummer  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


def _amr(lmin, radii, centre=(0.5, 0.5, 0.5)):
    return build_graded(lmin, lmin + len(radii), refine_sphere(centre, radii))


def _solve(h, m, **kw):
    plan = A.Plan(h, **kw)
    mt = torch.from_numpy(m).cuda()
    phi, acc = plan.solve(mt)
    torch.cuda.synchronize()
    out = (phi.cpu().numpy().copy(), acc.cpu().numpy().copy())
    plan.close()
    return out


@pytest.mark.parametrize("precision,p", [("fp32", 6), ("fp64", 4)])
def test_plan_on_reused_buffers_matches_fresh_buffers(precision, p):
    h1 = _amr(4, {4: 0.3, 5: 0.15}, (0.4, 0.55, 0.5))
    h2 = _amr(4, {4: 0.28, 5: 0.14}, (0.55, 0.45, 0.5))
    m1 = cell_masses(h1, plummer(1.0, 0.1), 0.01, 5)
    m2 = cell_masses(h2, plummer(1.0, 0.08), 0.01, 6)
    kw = dict(p=p, precision=precision)
    A.release_cached_memory()
    fresh = _solve(h2, m2, **kw)
    # fill the cache with buffers that hold another hierarchy's trees and fields
    for _ in range(2):
        _solve(h1, m1, **kw)
    reused = _solve(h2, m2, **kw)
    leaf = h2.leaf_mask()
    assert np.array_equal(fresh[0][leaf], reused[0][leaf]) and np.array_equal(fresh[1][leaf], reused[1][leaf])
    po, ao = oracle.Oracle(h2, p).solve_all(m2)
    check_errors(reused[0][leaf], reused[1][leaf], po[leaf], ao[leaf], precision, what=f"reused buffers {precision}")
    A.release_cached_memory()
    again = _solve(h2, m2, **kw)
    assert np.array_equal(again[0][leaf], fresh[0][leaf]) and np.array_equal(again[1][leaf], fresh[1][leaf])


def test_capped_plan_counts_exactly_and_batches_reuse_buffers():
    h = _amr(4, {4: 0.25, 5: 0.12})
    m = cell_masses(h, plummer(1.0, 0.08), 0.01, 9)
    probe = A.Plan(h, p=5, precision="fp32")
    need = probe.info()["device_bytes"]
    probe.close()
    # the cache holds the probe's buffers; a capped plan takes exact buffers of its own
    capped = A.Plan(h, p=5, precision="fp32", max_device_bytes=need)
    assert capped.info()["device_bytes"] == need
    capped.close()
    hs = [h, _amr(3, {3: 0.3, 4: 0.15}), _amr(4, {4: 0.2})]
    ms = [m] + [cell_masses(x, plummer(1.0, 0.1), 0.01, 20 + i) for i, x in enumerate(hs[1:])]
    masses = [torch.from_numpy(x).cuda() for x in ms]
    results = []
    for _ in range(2):  # the second batch is built on the first one's buffers
        plans = [A.Plan(x, p=4, precision="fp32") for x in hs]
        batch = A.Batch(plans)
        phis, accs = batch.solve(masses)
        torch.cuda.synchronize()
        results.append([(a.cpu().numpy().copy(), b.cpu().numpy().copy()) for a, b in zip(phis, accs)])
        batch.close()
        for pl in plans:
            pl.close()
    for x, (p0, a0), (p1, a1) in zip(hs, results[0], results[1]):
        leaf = x.leaf_mask()
        assert np.array_equal(p0[leaf], p1[leaf]) and np.array_equal(a0[leaf], a1[leaf])
