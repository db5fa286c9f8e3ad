"""Tile shapes of the intermediate-field launch (afmm_options.m2p_shape).

Shape 0 loads each lane's B fragments itself, shape 1 loads the source rows row
by row and stages them through LDS, shape 2 does the same with two 16-group
tiles of one parity class per wave, shape 3 loads the rows row by row and takes
each lane's fragments from other lanes over the crossbar (FP32 and FP64).  Every
shape runs the same MFMAs in the same order on the same operands, so the solves
must agree bit for bit; shapes 2 and 3 are also checked against the FP64
oracle, on ragged tiles (parity classes whose group counts are not multiples of
32), with tap splits whose ranges cross the kernels' source-table chunks, in a
batch, on periodic plans, and under the autotuner.
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


def _amr(lmin, radii):
    return build_graded(lmin, lmin + len(radii), refine_sphere((0.5, 0.5, 0.5), radii))


H3 = _amr(3, {3: 0.3, 4: 0.2, 5: 0.1})
H4 = _amr(4, {4: 0.22, 5: 0.1})


@pytest.mark.parametrize("h,p,split", [(H3, 4, 0), (H3, 5, 3), (H4, 4, 7), (H3, 2, 0), (H4, 6, 0), (H3, 8, 2)])
def test_shapes_agree_bitwise(h, p, split):
    m = cell_masses(h, plummer(1.0, 0.08), 0.01, 11 * p + split)
    leaf = h.leaf_mask()
    ref = None
    for shape in (0, 1, 2, 3):
        phi, acc, _ = gpu_solve(h, m, p, "fp32", m2p_shape=shape, tap_split=split)
        if ref is None:
            ref = (phi, acc)
            continue
        assert np.array_equal(phi[leaf], ref[0][leaf]) and np.array_equal(acc[leaf], ref[1][leaf]), shape
    print(f"p={p} split={split}: shapes 0..3 bit-identical over {int(leaf.sum())} leaves", flush=True)


@pytest.mark.parametrize("h,p,split", [(H3, 4, 0), (H4, 6, 3), (H3, 7, 0), (H3, 1, 2)])
def test_crossbar_fragments_fp64_bitwise_and_against_oracle(h, p, split):
    m = cell_masses(h, plummer(1.0, 0.08), 0.01, 13 * p + split)
    leaf = h.leaf_mask()
    phi0, acc0, _ = gpu_solve(h, m, p, "fp64", m2p_shape=0, tap_split=split)
    phi3, acc3, _ = gpu_solve(h, m, p, "fp64", m2p_shape=3, tap_split=split)
    assert np.array_equal(phi3[leaf], phi0[leaf]) and np.array_equal(acc3[leaf], acc0[leaf])
    po, ao = oracle.Oracle(h, p).solve_all(m)
    check_errors(phi3[leaf], acc3[leaf], po[leaf], ao[leaf], "fp64", what=f"shape 3 fp64 p={p}")


@pytest.mark.parametrize("p", [3, 4, 5])
def test_two_tiles_per_wave_against_oracle(p):
    h = H3
    m = cell_masses(h, plummer(1.0, 0.08), 0.01, 40 + p)
    phi, acc, _ = gpu_solve(h, m, p, "fp32", m2p_shape=2)
    po, ao = oracle.Oracle(h, p).solve_all(m)
    leaf = h.leaf_mask()
    check_errors(phi[leaf], acc[leaf], po[leaf], ao[leaf], "fp32", 1e-4, what=f"shape 2 p={p}")


def test_batch_with_two_tiles_per_wave_equals_plans():
    hs = [H3, H4, _amr(3, {3: 0.25})]
    ms = [cell_masses(h, plummer(1.0, 0.1), 0.01, 60 + i) for i, h in enumerate(hs)]
    plans = [A.Plan(h, p=4, precision="fp32", tap_split=3, m2p_shape=2) for h in hs]
    masses = [torch.from_numpy(m).cuda() for m in ms]
    ind = [pl.solve(mt) for pl, mt in zip(plans, masses)]
    batch = A.Batch(plans)
    phis, accs = batch.solve(masses)
    torch.cuda.synchronize()
    for h, (p0, a0), p1, a1 in zip(hs, ind, phis, accs):
        leaf = torch.from_numpy(h.leaf_mask()).cuda()
        assert torch.equal(p0[leaf], p1[leaf]) and torch.equal(a0[leaf], a1[leaf])
    batch.close()
    for pl in plans:
        pl.close()


def test_autotune_reports_a_supported_shape_and_stays_correct():
    h = H3
    m = cell_masses(h, plummer(1.0, 0.08), 0.01, 77)
    plan = A.Plan(h, p=4, precision="fp32")
    mt = torch.from_numpy(m).cuda()
    res = plan.autotune(mt)
    assert res["m2p_shape"][0] in (0, 3) and res["m2p_shape"][1] in (0, 1, 2, 3)
    phi, acc = plan.solve(mt)
    torch.cuda.synchronize()
    po, ao = oracle.Oracle(h, 4).solve_all(m)
    leaf = h.leaf_mask()
    check_errors(phi.cpu().numpy()[leaf], acc.cpu().numpy()[leaf], po[leaf], ao[leaf], "fp32", 1e-4,
                 what=f"autotuned shape {res['m2p_shape']}")
    plan.close()


@pytest.mark.parametrize("precision,p", [("fp32", 6), ("fp32", 5), ("fp64", 6), ("fp64", 4)])
def test_crossbar_shape_on_periodic_plans_and_in_batches(precision, p):
    # periodic plans (wrapped tiles, the level-2 far operator) and a batch of
    # plans, each with shape 3 against shape 0: bit for bit
    from test_gpu_periodic import _case
    names = ["corner", "face", "uni4"]
    cases = [_case(n) for n in names]
    masses = [torch.from_numpy(m).cuda() for _, m in cases]
    out = {}
    for shape in (0, 3):
        plans = [A.Plan(h, p=p, precision=precision, periodic=True, m2p_shape=shape, tap_split=1) for h, _ in cases]
        single = [tuple(t.clone() for t in pl.solve(mt)) for pl, mt in zip(plans, masses)]
        batch = A.Batch(plans)
        phis, accs = batch.solve(masses)
        torch.cuda.synchronize()
        for (h, _), (p1, a1), p2, a2 in zip(cases, single, phis, accs):
            leaf = torch.from_numpy(h.leaf_mask()).cuda()
            assert torch.equal(p1[leaf], p2[leaf]) and torch.equal(a1[leaf], a2[leaf]), shape
        out[shape] = single
        batch.close()
        for pl in plans:
            pl.close()
    for (h, _), (p0, a0), (p3, a3) in zip(cases, out[0], out[3]):
        leaf = torch.from_numpy(h.leaf_mask()).cuda()
        assert torch.equal(p0[leaf], p3[leaf]) and torch.equal(a0[leaf], a3[leaf])
