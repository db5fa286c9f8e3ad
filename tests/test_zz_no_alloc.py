"""afmm_solve_adjoint_noalloc (the allocation-free adjoint) against
afmm_solve_adjoint on the same plans: identical bits, nothing allocated.

Two calls in a row on different plans, the second on a smaller hierarchy, so
the second call reuses the static scratch that the first one filled; the
allocation-free call runs first on each plan (no plan workspace exists yet),
then the allocating adjoint gives the reference.  A plan whose adjoint
scratch exceeds the static maximum is refused with AFMM_E_OUT_OF_MEMORY.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_19489_amd as A  # noqa: E402
from paper_2607_19489_amd import _lib  # noqa: E402
from synth import cell_masses, plummer, unigrid  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402


def _noalloc(plan, pb, ab, mb, level=A.AFMM_ALL_LEVELS):
    return _lib.lib().afmm_solve_adjoint_noalloc(plan.handle, level, C.c_void_p(pb.data_ptr()),
                                                 C.c_void_p(ab.data_ptr()), C.c_void_p(mb.data_ptr()),
                                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_adjoint_equals_adjoint_twice_second_smaller(precision):
    cases = [build_graded(4, 7, refine_sphere((0.5, 0.5, 0.5), {4: 0.25, 5: 0.15, 6: 0.08})),
             build_graded(3, 5, refine_sphere((0.4, 0.5, 0.6), {3: 0.3, 4: 0.2}))]
    assert cases[1].total < cases[0].total
    for k, h in enumerate(cases):
        print(f"no-alloc adjoint case {k} ({h.total} cells) {precision}", flush=True)
        m = torch.from_numpy(cell_masses(h, plummer(1.0, 0.1), 0.01, 60 + k)).cuda()
        rng = np.random.default_rng(70 + k)
        pb = torch.from_numpy(rng.standard_normal(h.total)).cuda()
        ab = torch.from_numpy(rng.standard_normal((h.total, 3))).cuda()
        plan = A.Plan(h, p=5, precision=precision, fp64_levels=2)
        plan.solve(m)
        torch.cuda.synchronize()
        before = plan.info()["device_bytes"]
        mb = torch.full((h.total,), 3.5, dtype=torch.float64, device="cuda")
        assert _noalloc(plan, pb, ab, mb) == 0, _lib.lib().afmm_last_error()
        torch.cuda.synchronize()
        assert plan.info()["device_bytes"] == before  # the call allocated nothing
        ref = plan.solve_adjoint(pb, ab)
        torch.cuda.synchronize()
        assert plan.info()["device_bytes"] > before  # the allocating one did
        assert torch.equal(mb, ref)
        # again after the allocating call, and after a level solve (Alg. 1)
        mb2 = torch.zeros(h.total, dtype=torch.float64, device="cuda")
        assert _noalloc(plan, pb, ab, mb2) == 0
        torch.cuda.synchronize()
        assert torch.equal(mb2, ref)
        lev = h.levelmin + 1
        plan.solve(m * 1.01, level=lev, icount=2)
        ref_l = plan.solve_adjoint(pb, ab, level=lev)
        mb3 = torch.zeros(h.total, dtype=torch.float64, device="cuda")
        assert _noalloc(plan, pb, ab, mb3, level=lev) == 0
        torch.cuda.synchronize()
        assert torch.equal(mb3, ref_l)
        plan.close()


def test_noalloc_adjoint_refuses_oversized_plans():
    h = unigrid(7)
    m = torch.from_numpy(cell_masses(h, plummer(1.0, 0.1), 0.01, 9)).cuda()
    plan = A.Plan(h, p=4, precision="fp64")
    plan.solve(m)
    z = torch.zeros(h.total, dtype=torch.float64, device="cuda")
    z3 = torch.zeros(h.total, 3, dtype=torch.float64, device="cuda")
    assert _noalloc(plan, z, z3, z) == -5
    assert b"static maximum" in _lib.lib().afmm_last_error()
    # nothing ran: the output is untouched, and the plan still works
    torch.cuda.synchronize()
    assert bool((z == 0).all())
    plan.solve(m)
    torch.cuda.synchronize()
