"""Batched solves (one forest, one hipGraph replay) against per-hierarchy solves.

With the same tap split, the batch runs the same arithmetic in the same order
for every hierarchy, so its results must equal the individual solves bit for
bit.  The graph is replayed several times with eager work in between, and each
replay is checked.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import max_rel, rel_l2  # noqa: E402

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, configs, plummer, unigrid  # noqa: E402

SENTINEL = 7.25


def _members(p):
    ws = [configs.cfg4_member(i, p=p, base_choices=(3, 4), max_extra=2) for i in range(6)]
    hs = [w.hierarchy for w in ws] + [unigrid(2), unigrid(3)]
    ms = [w.mass for w in ws] + [cell_masses(unigrid(2), plummer(1.0, 0.2), 0.01, 5),
                                 cell_masses(unigrid(3), plummer(1.0, 0.1), 0.01, 6)]
    return hs, ms


def _plans(hs, p, **kw):
    return [A.Plan(h, p=p, **kw) for h in hs]


def _individual(plans, masses):
    out = []
    for pl, m in zip(plans, masses):
        phi = torch.full((pl.N,), SENTINEL, dtype=torch.float64, device="cuda")
        acc = torch.full((pl.N, 3), SENTINEL, dtype=torch.float64, device="cuda")
        pl.solve(m, phi=phi, acc=acc)
        out.append((phi, acc))
    torch.cuda.synchronize()
    return [(a.cpu().numpy(), b.cpu().numpy()) for a, b in out]


@pytest.mark.parametrize("precision,p", [("fp64", 4), ("fp32", 4), ("fp32", 8), ("fp64", 6)])
def test_batch_equals_individual_bitwise(precision, p):
    hs, ms = _members(p)
    print(f"batch {precision} p={p}: {[h.nleaves() for h in hs]} leaves", flush=True)
    plans = _plans(hs, p, precision=precision, tap_split=3)
    batch = A.Batch(plans)
    info = batch.info()
    assert info["nhier"] == len(hs)
    assert info["nleaves"] == sum(h.nleaves() for h in hs)
    masses = [torch.from_numpy(m).cuda() for m in ms]
    ref = _individual(plans, masses)
    for rep in range(3):
        scale = 1.0 + 0.5 * rep
        ms_r = [m * scale for m in masses]
        phis = [torch.full((pl.N,), SENTINEL, dtype=torch.float64, device="cuda") for pl in plans]
        accs = [torch.full((pl.N, 3), SENTINEL, dtype=torch.float64, device="cuda") for pl in plans]
        batch.solve(ms_r, phis, accs)
        torch.cuda.synchronize()
        ref_r = ref if rep == 0 else _individual(plans, ms_r)
        for i, h in enumerate(hs):
            leaf = h.leaf_mask()
            pb, ab = phis[i].cpu().numpy(), accs[i].cpu().numpy()
            assert np.array_equal(pb[leaf], ref_r[i][0][leaf]), f"member {i} phi differs (replay {rep})"
            assert np.array_equal(ab[leaf], ref_r[i][1][leaf]), f"member {i} acc differs (replay {rep})"
            assert np.all(pb[~leaf] == SENTINEL) and np.all(ab[~leaf] == SENTINEL)
    batch.close()
    # the batch owns a copy of the topology: plans may go first
    for pl in plans:
        pl.close()


def test_batch_outlives_plans_and_matches_oracle():
    hs, ms = _members(5)
    plans = [A.Plan(h, p=5, precision="fp64") for h in hs[:3]]
    batch = A.Batch(plans)
    for pl in plans:
        pl.close()
    masses = [torch.from_numpy(m).cuda() for m in ms[:3]]
    phis, accs = batch.solve(masses)
    torch.cuda.synchronize()
    for i in range(3):
        po, ao = oracle.Oracle(hs[i], 5).solve_all(ms[i])
        leaf = hs[i].leaf_mask()
        a, ph = accs[i].cpu().numpy()[leaf], phis[i].cpu().numpy()[leaf]
        assert rel_l2(a, ao[leaf]) <= 1e-10 and rel_l2(ph, po[leaf]) <= 1e-10
        assert max_rel(a, ao[leaf]) <= 1e-9


def test_batch_of_one_and_mismatched_options():
    h = unigrid(3)
    m = torch.from_numpy(cell_masses(h, plummer(1.0, 0.1), 0.01, 2)).cuda()
    pl = A.Plan(h, p=4, precision="fp32")
    b = A.Batch([pl])
    phis, accs = b.solve([m])
    phi, acc = pl.solve(m)
    torch.cuda.synchronize()
    assert torch.equal(phis[0], phi) and torch.equal(accs[0], acc)
    other = A.Plan(h, p=5, precision="fp32")
    with pytest.raises(A.AfmmError):
        A.Batch([pl, other])
    # the model flags travel into the batch; members must agree on them
    cap = A.Plan(h, p=4, precision="fp32", quad_cap=True, self_potential=True)
    with pytest.raises(A.AfmmError):
        A.Batch([pl, cap])
    bc = A.Batch([cap])
    phis, accs = bc.solve([m])
    phi, acc = cap.solve(m)
    torch.cuda.synchronize()
    assert torch.equal(phis[0], phi) and torch.equal(accs[0], acc)
