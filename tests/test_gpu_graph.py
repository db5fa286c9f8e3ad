"""AFMM_GRAPH: solves replayed from captured hipGraphs give the eager solves'
bits, for full solves and the adaptive-time-step sequence (Alg. 1), over
several replays with eager work in between, with masses updated in place
between replays and with new I/O buffers (a new capture)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, plummer  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


def _amr():
    return build_graded(4, 7, refine_sphere((0.5, 0.5, 0.5), {4: 0.25, 5: 0.15, 6: 0.08}))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_full_solves_equal_eager(precision):
    h = _amr()
    leaf = torch.from_numpy(h.leaf_mask()).cuda()
    eager = A.Plan(h, p=5, precision=precision, tap_split=2)
    graph = A.Plan(h, p=5, precision=precision, tap_split=2, graph=True)
    m = torch.from_numpy(cell_masses(h, plummer(1.0, 0.08), 0.01, 81)).cuda()
    phi = torch.zeros(h.total, dtype=torch.float64, device="cuda")
    acc = torch.zeros(h.total, 3, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(82)
    for rep in range(4):
        # masses change in place: the graph reads the same buffer
        m.copy_(torch.from_numpy(cell_masses(h, plummer(1.0, 0.08), 0.01, 81)
                                 * (1 + 1e-2 * rng.standard_normal(h.total))).cuda())
        graph.solve(m, phi=phi, acc=acc)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        pe, ae = eager.solve(m)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(phi[leaf], pe[leaf]) and torch.equal(acc[leaf], ae[leaf]), rep
    # new output buffers: a second capture, same bits
    p2, a2 = graph.solve(m)
    torch.cuda.synchronize()
    assert torch.equal(p2[leaf], pe[leaf]) and torch.equal(a2[leaf], ae[leaf])
    # profiled solves run eagerly
    graph.set_profiling(True)
    p3, a3 = graph.solve(m)
    torch.cuda.synchronize()
    assert graph.get_profile()["upward"]["launches"] >= 1
    assert torch.equal(p3[leaf], pe[leaf]) and torch.equal(a3[leaf], ae[leaf])


def test_graph_ats_sequence_equals_eager():
    h = _amr()
    lev, leafn = h.level_of(), h.leaf_mask()
    seq = []

    def rec(l, ic):
        seq.append((l, ic))
        if l < h.levelmax:
            rec(l + 1, 1)
            rec(l + 1, 2)
    rec(h.levelmin, 1)
    eager = A.Plan(h, p=4, precision="fp32", fp64_levels=2)
    graph = A.Plan(h, p=4, precision="fp32", fp64_levels=2, graph=True)
    m0 = cell_masses(h, plummer(1.0, 0.08), 0.01, 83)
    rng = np.random.default_rng(84)
    m = torch.from_numpy(m0).cuda()
    pg = torch.zeros(h.total, dtype=torch.float64, device="cuda")
    ag = torch.zeros(h.total, 3, dtype=torch.float64, device="cuda")
    for sweep in range(2):  # the second sweep replays every captured graph
        for l, ic in seq:
            m.mul_(torch.from_numpy(1 + 1e-3 * rng.uniform(-1, 1, h.total)).cuda())
            graph.solve(m, level=l, icount=ic, phi=pg, acc=ag)
            pe, ae = eager.solve(m, level=l, icount=ic)
            torch.cuda.synchronize()
            s = torch.from_numpy((lev == l) & leafn).cuda()
            assert torch.equal(pg[s], pe[s]) and torch.equal(ag[s], ae[s]), (sweep, l, ic)
