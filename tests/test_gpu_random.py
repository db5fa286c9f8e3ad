"""Randomised parity sweep: seeded random graded hierarchies (levelmin 1..4, one
to three refined levels around random clumps, refinement reaching the box
faces and corners, shuffled caller order) with random order p, precision, tap
split and M2P tile shape, each solved on the GPU and compared with the FP64
oracle over all leaves (FP64 to 1e-10, the FP32 form to its gate).  Plus an
adaptive-time-step sub-step and the adjoint's dot-product identity on the
same cases.  Every case prints its parameters before it runs.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import check_errors, gpu_solve  # noqa: E402

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, plummer  # noqa: E402
from synth.density import gaussian_clumps, sum_density  # noqa: E402
from synth.hierarchy import build_graded, refine_mass, shuffle_order  # noqa: E402


def _case(seed):
    rng = np.random.default_rng(seed)
    lmin = int(rng.integers(1, 5))
    extra = int(rng.integers(1, 4))
    nclump = int(rng.integers(1, 4))
    centres = rng.uniform(0.0, 1.0, size=(nclump, 3))
    sig = rng.uniform(0.03, 0.1, size=nclump)
    mass = rng.uniform(0.2, 1.0, size=nclump)
    rho = sum_density(gaussian_clumps(centres, sig, mass), plummer(0.1, 0.3))
    # refine where a cell holds more than a random multiple of the mean base-cell mass
    thr = float(rng.uniform(1.5, 6.0)) / 8 ** lmin
    h = build_graded(lmin, lmin + extra, refine_mass(rho, thr, lmin + extra))
    h = shuffle_order(h, seed)
    m = cell_masses(h, rho, 0.01, seed)
    p = int(rng.integers(1, 9))
    precision = ["fp64", "fp32"][int(rng.integers(0, 2))]
    split = int(rng.choice([0, 1, 2, 3, 5]))
    shape = int(rng.integers(0, 3)) if precision == "fp32" else 0
    return h, m, p, precision, split, shape


SEEDS = list(range(9100, 9116))


@pytest.mark.parametrize("seed", SEEDS)
def test_random_case_against_oracle(seed):
    h, m, p, precision, split, shape = _case(seed)
    print(f"seed {seed}: levels {h.levelmin}..{h.levelmax}, {h.nleaves()} leaves, p={p} {precision} "
          f"split={split} shape={shape}", flush=True)
    plan = A.Plan(h, p=p, precision=precision, tap_split=split, m2p_shape=shape)
    phi, acc, _ = gpu_solve(h, m, p, precision, plan=plan)
    o = oracle.Oracle(h, p)
    po, ao = o.solve_all(m)
    leaf = h.leaf_mask()
    tol = 1e-10 if precision == "fp64" else 1e-4
    check_errors(phi[leaf], acc[leaf], po[leaf], ao[leaf], precision, tol, what=f"seed {seed}")
    # one adaptive-time-step sub-step without a rebuild at the finest level: the
    # trees of the full solve are kept, so the finest leaves must not change
    lev = h.level_of()
    fine = (lev == h.levelmax) & leaf
    if h.levelmax > h.levelmin and fine.any():
        pl, al, _ = gpu_solve(h, m * 2.0 + 1.0, p, precision, plan=plan, level=h.levelmax, icount=1)
        assert np.array_equal(pl[fine], phi[fine]) and np.array_equal(al[fine], acc[fine])
    # adjoint: <A x, y> = <x, A^T y> on the leaves
    if precision == "fp64":
        rng = np.random.default_rng(seed + 1)
        x = np.where(leaf, rng.standard_normal(h.total), 0.0)
        yp = np.where(leaf, rng.standard_normal(h.total), 0.0)
        ya = np.where(leaf[:, None], rng.standard_normal((h.total, 3)), 0.0)
        px, ax, _ = gpu_solve(h, x, p, precision, plan=plan)
        xb = plan.solve_adjoint(torch.from_numpy(yp).cuda(), torch.from_numpy(ya).cuda()).cpu().numpy()
        lhs = float(np.dot(px[leaf], yp[leaf]) + np.sum(ax[leaf] * ya[leaf]))
        rhs = float(np.dot(x, xb))
        assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-300) + 1e-12, (lhs, rhs)
    plan.close()
