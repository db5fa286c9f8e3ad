"""Drifted stale trees in adaptive time steps (afmm_solve_drift).

Alg. 1 keeps the trees it does not rebuild (those of the inactive coarser
levels, and at a sub-step without a rebuild all of them) as they were at
their last rebuild; the drifted solve advances their masses to the solve's
time with the mass rates recorded at that rebuild (first order in time).  Pins:

- a mass field that changes linearly in time is solved exactly at every
  sub-step of an adaptive-time-step cycle (equal to a synchronous solve of the
  current masses), while the undrifted solve is not;
- on a non-linear evolution the drifted solve equals the oracle evaluated on
  the drifted masses (snapshot + elapsed time x rate per stale level, rebuilt
  levels current), FP64 to 1e-10 and the FP32 form to its gate;
- trees last rebuilt by a plain solve carry no rates and stay undrifted.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_util import check_errors, rel_l2  # noqa: E402

import oracle  # noqa: E402
import paper_2607_19489_amd as A  # noqa: E402
from synth import cell_masses, plummer  # noqa: E402
from synth.hierarchy import build_graded, refine_sphere  # noqa: E402

H = build_graded(3, 6, refine_sphere((0.5, 0.5, 0.5), {3: 0.3, 4: 0.2, 5: 0.1}))
LEV = H.level_of()
LEAF = H.leaf_mask()


def _cycle(lmin, lmax):
    """(level, icount) of one coarse step of Alg. 1: level l sub-cycles twice
    per step of level l - 1, the second sub-step rebuilding its trees."""
    out = []

    def rec(l, icount):
        out.append((l, icount))
        if l < lmax:
            rec(l + 1, 1)
            rec(l + 1, 2)
    rec(lmin, 1)
    return out


SEQ = _cycle(3, 6)
TIMES = [0.1 * k for k in range(len(SEQ))]


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _solve(plan, fn, *args, **kw):
    phi, acc = fn(*args, **kw)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), acc.cpu().numpy()


def test_linear_mass_evolution_is_solved_exactly():
    m0 = cell_masses(H, plummer(1.0, 0.08), 0.01, 5)
    rate = m0 * np.random.default_rng(6).uniform(-0.5, 0.5, H.total)
    plan = A.Plan(H, p=4, precision="fp64")
    plain = A.Plan(H, p=4, precision="fp64")
    sync = A.Plan(H, p=4, precision="fp64")
    worst_drift = worst_plain = 0.0
    for (l, ic), t in zip(SEQ, TIMES):
        m = m0 + t * rate
        sel = (LEV == l) & LEAF
        pd, ad = _solve(plan, plan.solve_drift, _cuda(m), _cuda(rate), t, level=l, icount=ic)
        pp, ap = _solve(plain, plain.solve, _cuda(m), level=l, icount=ic)
        ps, as_ = _solve(sync, sync.solve, _cuda(m))
        worst_drift = max(worst_drift, rel_l2(ad[sel], as_[sel]), rel_l2(pd[sel], ps[sel]))
        worst_plain = max(worst_plain, rel_l2(ap[sel], as_[sel]))
    print(f"linear evolution over {len(SEQ)} sub-steps: drifted vs synchronous {worst_drift:.2e}, "
          f"undrifted {worst_plain:.2e}", flush=True)
    assert worst_drift < 1e-12
    assert worst_plain > 1e-4
    for pl in (plan, plain, sync):
        pl.close()


def _expected(seq_times, mass_fn, rate_fn, plain_at=()):
    """Host bookkeeping of Alg. 1 with drift: per level, the masses, rates and
    time of its last rebuild (no rates after a plain rebuild); the steps in
    plain_at are plain solves, which drift nothing."""
    snap_m = np.zeros(H.total)
    snap_r = np.zeros(H.total)
    t_snap = {}
    has_rate = {}
    out = []
    for k, ((l, ic), t) in enumerate(seq_times):
        m, r = mass_fn(t), rate_fn(t)
        if l == 3 or ic > 1:
            for j in range(l, 7):
                s = LEV == j
                snap_m[s] = m[s]
                snap_r[s] = r[s]
                t_snap[j] = t
                has_rate[j] = k not in plain_at
        # every tree not rebuilt now is stale, whatever its level (the trees of
        # levels >= l too when Alg. 1 rebuilds none): advanced if it has rates
        eff = snap_m.copy()
        for j in range(3, 7):
            s = LEV == j
            if k not in plain_at and has_rate.get(j) and t_snap[j] != t:
                eff[s] = snap_m[s] + (t - t_snap[j]) * snap_r[s]
        out.append(eff)
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nonlinear_evolution_matches_oracle_on_drifted_masses(precision):
    m0 = cell_masses(H, plummer(1.0, 0.08), 0.01, 7)
    ph = np.random.default_rng(8).uniform(0, 2 * np.pi, H.total)

    def mass(t):
        return m0 * (1.0 + 0.3 * np.sin(2.0 * t + ph))

    def rate(t):
        return m0 * 0.6 * np.cos(2.0 * t + ph)
    seq = list(zip(SEQ, TIMES))
    effs = _expected(seq, mass, rate)
    plan = A.Plan(H, p=4, precision=precision)
    o = oracle.Oracle(H, 4)
    tol = 1e-10 if precision == "fp64" else 1e-4
    for ((l, ic), t), eff in zip(seq, effs):
        pd, ad = _solve(plan, plan.solve_drift, _cuda(mass(t)), _cuda(rate(t)), t, level=l, icount=ic)
        o.rebuild(3, eff)
        tg = np.nonzero((LEV == l) & LEAF)[0]
        po, ao = o.eval(l, tg)
        check_errors(pd[tg], ad[tg], po, ao, precision, tol, what=f"drift l={l} icount={ic} t={t:.1f}")
    plan.close()


def test_plain_rebuilds_carry_no_rates():
    m0 = cell_masses(H, plummer(1.0, 0.08), 0.01, 9)
    ph = np.random.default_rng(10).uniform(0, 2 * np.pi, H.total)

    def mass(t):
        return m0 * (1.0 + 0.3 * np.sin(2.0 * t + ph))

    def rate(t):
        return m0 * 0.6 * np.cos(2.0 * t + ph)
    # drift rebuild of every tree, a plain rebuild of levels >= 5, then drifted solves
    seq = [((3, 1), 0.0), ((5, 2), 0.4), ((6, 1), 0.7), ((4, 1), 0.9)]
    effs = _expected(seq, mass, rate, plain_at=(1,))
    plan = A.Plan(H, p=4, precision="fp64")
    o = oracle.Oracle(H, 4)
    for k, (((l, ic), t), eff) in enumerate(zip(seq, effs)):
        if k == 1:
            pd, ad = _solve(plan, plan.solve, _cuda(mass(t)), level=l, icount=ic)
        else:
            pd, ad = _solve(plan, plan.solve_drift, _cuda(mass(t)), _cuda(rate(t)), t, level=l, icount=ic)
        o.rebuild(3, eff)
        tg = np.nonzero((LEV == l) & LEAF)[0]
        po, ao = o.eval(l, tg)
        assert rel_l2(ad[tg], ao) < 1e-10 and rel_l2(pd[tg], po) < 1e-10, (l, ic, t)
    plan.close()


def test_drift_errors_and_input_check():
    m = _cuda(cell_masses(H, plummer(1.0, 0.08), 0.01, 11))
    r = torch.zeros_like(m)
    plan = A.Plan(H, p=4, precision="fp64", check_input=True)
    with pytest.raises(A.AfmmError, match="ATS_ORDER"):
        plan.solve_drift(m, r, 0.0, level=5, icount=1)
    with pytest.raises(A.AfmmError, match="INVALID_ARG"):
        plan.solve_drift(m, r, float("nan"), level=3, icount=1)
    bad = r.clone()
    bad[int(np.nonzero((LEV == 4) & LEAF)[0][0])] = float("inf")
    with pytest.raises(A.AfmmError, match="NONFINITE"):
        plan.solve_drift(m, bad, 0.0, level=3, icount=1)
    plan.solve_drift(m, r, 0.0, level=3, icount=1)
    # level 6 without a rebuild reads no rates: a bad rate of level 4 is not read
    plan.solve_drift(m, bad, 0.5, level=6, icount=1)
    torch.cuda.synchronize()
    plan.close()
