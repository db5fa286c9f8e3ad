#!/usr/bin/env python3
"""Throughput of one full adaptive-FMM solve (potential + acceleration of every
leaf) on one MI355X, FP32-mixed form vs FP64 form.

Default workload: the deep AMR hierarchy -- level 7 (128^3) base, up to four
more levels refined where the cell mass exceeds 1.25x the mean level-7 cell
mass (8,083,818 leaves over levels 7..11), Plummer a=0.05 + 32 Gaussian clumps
+ 1% noise (seed 3), expansion order p=6.  Inputs (plan and masses) are
resident in HBM before the timed region; a "step" is one full solve (upward
pass, M2L/L2L over every FMM level, far/intermediate/near/nearest fields at
every leaf).  Plan creation (host topology + uploads) is timed separately.

Prints one JSON line.  The roofline object describes the kernel family with
the largest share of the timed region: its algorithmic flops divided by its
summed launch time, both measured live with hipEvents on the solve stream.
The cpu_baseline object times the FP64 CPU oracle (test infrastructure) on a
bounded, spatially clustered sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cells/sec full FMM solve (φ+accel) at rel. force err ≤1e-4, FP32 vs FP64"
PEAK = {"fp32_mfma": 157.3, "fp64_mfma": 78.6, "fp32_vector": 157.3, "fp64_vector": 78.6, "hbm": 8000.0}
KERNEL_NAMES = {"near_f32": "k_near<float, P>", "near_f64": "k_near<double, P>",
                "m2l_f32": "k_m2l_mfma<float, P>", "m2l_f64": "k_m2l_mfma<double, P>",
                "m2p_f32": "k_m2p<float, P, XB>", "m2p_f64": "k_m2p<double, P, XB>",
                "l2l": "k_l2l<T, TL, P>", "upward": "k_upward<P>", "gather": "k_gather_mass",
                "adj_near": "k_adj_near_leaf + k_adj_near_m2p<P>", "adj_m2p": "k_adj_m2p<P>",
                "adj_m2l": "k_adj_m2l<P>", "adj_tree": "k_adj_l2l/k_adj_down/k_adj_out"}
MFMA_FAMILIES = ("m2l_f32", "m2l_f64", "m2p_f32", "m2p_f64")


def make_workload(name: str):
    from synth import configs
    if name == "cfg1":
        return configs.cfg1(), "unigrid 32^3 (32,768 leaves), Plummer a=0.1, p=4"
    if name == "cfg2":
        return configs.cfg2(), ("level 6 + level 7 within r<=0.15 (287,680 leaves, 3,648 refined), "
                                "Plummer a=0.05 + 1% noise, p=6")
    if name == "cfg3":
        return configs.cfg3(), ("level 7 (128^3) base + up to 4 levels refined where the cell mass exceeds "
                                f"{configs.CFG3_K}x the mean level-7 cell mass (8,083,818 leaves on levels 7..11; "
                                "this threshold is calibrated to about 8M leaves, the 8x threshold gives 2.94M "
                                "leaves on levels 7..10), Plummer a=0.05 + 32 Gaussian clumps + 1% noise, seed 3, p=6")
    if name == "cfg5":
        return configs.cfg5(), "level 7 + r<0.2 + r<0.1 (3,081,632 leaves), Plummer a=0.05, p=6"
    raise ValueError(name)


def ats_sequence(lmin, lmax):
    """Adaptive-time-step solve order (Alg. 1): a level-l step solves l, then runs two
    steps of level l+1 (icount 1 and 2): 1 + 2 + 4 + ... solves."""
    seq = []

    def rec(l, icount):
        seq.append((l, icount))
        if l < lmax:
            rec(l + 1, 1)
            rec(l + 1, 2)

    rec(lmin, 1)
    return seq


def time_ats(h, mass_t, p, precision, reps=2, graph=False, drift=False):
    """One coarse step of the adaptive-time-step sequence, masses of the active
    levels perturbed by 1e-3 seeded noise before every solve.  With `graph` the
    plan replays captured graphs (AFMM_GRAPH); the masses of each substep are
    then copied into one buffer first (a device copy inside the timed region),
    as an integrator updating them in place would.  With `drift` every solve
    is a drifted one (afmm_solve_drift, substep k at time 0.01 k, seeded mass
    rates of the same magnitude as the perturbations)."""
    import torch
    import paper_2607_19489_amd as A
    plan = A.Plan(h, p=p, precision=precision, graph=graph)
    plan.autotune(mass_t)
    seq = ats_sequence(h.levelmin, h.levelmax)
    lev = torch.from_numpy(h.level_of()).cuda()
    gen = torch.Generator(device="cuda").manual_seed(3)
    noise = [1.0 + 1e-3 * (2 * torch.rand(h.total, dtype=torch.float64, device="cuda", generator=gen) - 1)
             for _ in range(len(seq))]
    masses = []
    m = mass_t.clone()
    for (l, _), u in zip(seq, noise):
        m = torch.where(lev >= l, m * u, m)
        masses.append(m)
    phi = torch.zeros(h.total, dtype=torch.float64, device="cuda")
    acc = torch.zeros(h.total, 3, dtype=torch.float64, device="cuda")
    mbuf = mass_t.clone()
    rate = mass_t * 0.1 * (2 * torch.rand(h.total, dtype=torch.float64, device="cuda", generator=gen) - 1)
    per_level = {}
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in seq]
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, ((l, ic), mm, (a, b)) in enumerate(zip(seq, masses, ev)):
            a.record()
            if graph:
                mbuf.copy_(mm)
                mm = mbuf
            if drift:
                plan.solve_drift(mm, rate, 0.01 * k, level=l, icount=ic, phi=phi, acc=acc)
            else:
                plan.solve(mm, level=l, icount=ic, phi=phi, acc=acc)
            b.record()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if best is None or dt < best:
            best = dt
            per_level = {}
            for (l, ic), (a, b) in zip(seq, ev):
                per_level.setdefault(str(l), []).append(a.elapsed_time(b))
    info = plan.info()
    leaf_updates = sum(info["leaves_per_level"][l] for l, _ in seq)
    plan.close()
    return {"solves": len(seq), "sequence_ms": 1e3 * best, "leaf_updates": leaf_updates,
            "leaf_updates_per_s": leaf_updates / best,
            "mean_ms_per_solve_by_level": {k: sum(v) / len(v) for k, v in per_level.items()},
            "solves_by_level": {k: len(v) for k, v in per_level.items()}}


def time_adjoint(h, mass_t, p, precision, steps):
    """Forward + adjoint of the full solve (the backward of AFMMSolve)."""
    import torch
    import paper_2607_19489_amd as A
    plan = A.Plan(h, p=p, precision=precision)
    gen = torch.Generator(device="cuda").manual_seed(5)
    pb = torch.randn(h.total, dtype=torch.float64, device="cuda", generator=gen)
    ab = torch.randn(h.total, 3, dtype=torch.float64, device="cuda", generator=gen)
    mb = torch.zeros(h.total, dtype=torch.float64, device="cuda")
    phi, acc = plan.solve(mass_t)
    plan.solve_adjoint(pb, ab, mass_bar=mb)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    plan.get_profile()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(mass_t, phi=phi, acc=acc)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / steps
    fwd_prof = plan.get_profile()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve_adjoint(pb, ab, mass_bar=mb)
    torch.cuda.synchronize()
    t_adj = (time.perf_counter() - t0) / steps
    prof = plan.get_profile()
    plan.close()
    adj = {k: v for k, v in prof.items() if k.startswith("adj_")}
    return {"forward_ms": 1e3 * t_fwd, "adjoint_ms": 1e3 * t_adj, "adjoint_over_forward": t_adj / t_fwd,
            "adjoint_precision": "per level as the forward (fp32 form)" if precision == "fp32" else "f64", "kernels": kernel_table({"kernels": adj, "steps": steps}),
            "forward_kernels": kernel_table({"kernels": fwd_prof, "steps": steps})}


def run_binary(levelmax, dt=0.01, tend=8.0):
    """The binary-orbit time loop (two masses G m = 0.01, separation 0.15,
    levelmin 6, two cells of mesh expansion, fixed-step leapfrog to t = 8): wall
    time per step, plans built, and the orbit's deviations from the analytic
    circular orbit."""
    import torch
    from paper_2607_19489_amd import pm
    pos, vel, m, omega = pm.binary_initial(gm=0.01, sep=0.15)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = pm.ParticleMesh(pos, vel, m, 6, levelmax, nexpand=2, p=6, precision="fp64")
    n = int(round(tend / dt))
    for _ in range(n):
        sim.step(dt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    x, v = sim.pos.cpu().numpy(), sim.vel.cpu().numpy()
    d = x[0] - x[1]
    ang = np.arctan2(d[1], d[0])
    out = {"levels": [6, levelmax], "steps": n, "dt": dt, "t": sim.t, "plans": sim.replans,
           "ms_per_step": 1e3 * wall / n, "final_sep_rel_err": float(abs(np.linalg.norm(d) - 0.15) / 0.15),
           "final_phase_rad": float((ang - omega * sim.t + np.pi) % (2 * np.pi) - np.pi),
           "cells": int(sim.h.total)}
    sim.close()
    return out


def run_batch(args):
    """Batched workload: independent hierarchies of uneven size, one graph launch per solve."""
    import torch
    import paper_2607_19489_amd as A
    from synth import configs
    t0 = time.perf_counter()
    ws = configs.cfg4(args.members, p=args.p)
    nleaf = sum(w.hierarchy.nleaves() for w in ws)
    print(f"[bench] batch of {len(ws)} hierarchies, {nleaf} leaves, generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    plans = [A.Plan(w.hierarchy, p=args.p, precision="fp32") for w in ws]
    batch = A.Batch(plans)
    for pl in plans:
        pl.close()
    masses = [torch.from_numpy(w.mass).cuda() for w in ws]
    phis = [torch.zeros(w.hierarchy.total, dtype=torch.float64, device="cuda") for w in ws]
    accs = [torch.zeros(w.hierarchy.total, 3, dtype=torch.float64, device="cuda") for w in ws]
    tune = None if args.no_autotune else batch.autotune(masses)
    for _ in range(args.warmup):
        batch.solve(masses, phis, accs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.solve(masses, phis, accs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # one eager profiled pass for the per-kernel roofline
    batch.set_profiling(True)
    batch.get_profile()
    for _ in range(2):
        batch.solve(masses, phis, accs)
    torch.cuda.synchronize()
    prof = batch.get_profile()
    batch.set_profiling(False)
    res = {"kernels": prof, "steps": 2, "autotune": tune}
    info = batch.info()
    base = None
    if not args.no_cpu:
        import oracle
        t_used, done = 0.0, 0
        for w in ws:
            o = oracle.Oracle(w.hierarchy, args.p)
            t1 = time.perf_counter()
            o.solve_all(w.mass)
            t_used += time.perf_counter() - t1
            done += w.hierarchy.nleaves()
            if t_used > args.cpu_seconds:
                break
        base = {"value": done / t_used, "unit": "cells/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"full oracle solves of the first hierarchies of the batch ({done} leaves, {t_used:.1f} s)"}
    line = {
        "metric": METRIC, "value": nleaf / dt, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"cfg4: batch of {len(ws)} independent hierarchies (base level 4-6, 0-3 mass-refined "
                                f"levels, Plummer or clumps), {nleaf} leaves, one hipGraph launch per solve"),
                   "p": args.p, "precision": "FP32 mixed", "leaves": nleaf, "hierarchies": len(ws)},
        "roofline": roofline(res, "fp32"), "cpu_baseline": base, "autotune": tune,
        "algorithmic_flops_per_step": info["flops_m2l"] + info["flops_m2p"] + info["flops_p2p"] + info["flops_updown"],
        "kernels_fp32": kernel_table(res),
    }
    print(json.dumps(line), flush=True)


def m2p_shape_ok(p, fp32, shape):
    """Tile shapes the library runs for this order and precision (afmm_options.m2p_shape)."""
    return shape == 0 or (shape == 3 and (fp32 or p <= 7)) or (fp32 and (shape == 1 or (shape == 2 and p <= 5)))


def time_form(h, mass_t, p, precision, steps, warmup, overlap=False, autotune=True, graph=False, periodic=False,
              m2p_shape=0):
    """Autotuned plan (tap splits), timed solves (no instrumentation), then the same
    number of profiled solves: the profiled pass runs serially with hipEvents
    around every launch."""
    import torch
    import paper_2607_19489_amd as A
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = A.Plan(h, p=p, precision=precision, overlap=overlap, graph=graph, periodic=periodic, m2p_shape=m2p_shape)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)
    info = plan.info()
    phi = torch.zeros(h.total, dtype=torch.float64, device="cuda")
    acc = torch.zeros(h.total, 3, dtype=torch.float64, device="cuda")
    tune = plan.autotune(mass_t, phi, acc) if autotune else None
    for _ in range(warmup):
        plan.solve(mass_t, phi=phi, acc=acc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(mass_t, phi=phi, acc=acc)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.set_profiling(True)
    plan.get_profile()  # reset
    for _ in range(steps):
        plan.solve(mass_t, phi=phi, acc=acc)
    torch.cuda.synchronize()
    prof = plan.get_profile()
    plan.set_profiling(False)
    # M2P tile shape that ran, [FP64 kernels, FP32 kernels]: the tuner's, or the
    # option where the order and precision support it (else the plan used 0)
    fixed = [m2p_shape if m2p_shape_ok(p, fp32, m2p_shape) else 0 for fp32 in (False, True)]
    out = {"ms_per_step": 1e3 * dt / steps, "value": info["nleaves"] * steps / dt, "info": info,
           "kernels": prof, "steps": steps, "autotune": tune, "plan_create_ms": plan_ms,
           "m2p_shape": tune["m2p_shape"] if tune else fixed}
    phi_np, acc_np = phi.cpu().numpy(), acc.cpu().numpy()
    plan.close()
    return out, phi_np, acc_np


SYMBOLS = {"m2p_f32": "k_m2p<float, {p}, {xb}>", "m2p_f64": "k_m2p<double, {p}, {xb}>",
           "m2l_f32": "k_m2l_mfma<float, {p}>", "m2l_f64": "k_m2l_mfma<double, {p}>",
           "near_f32": "k_near<float, {p}>", "near_f64": "k_near<double, {p}>", "upward": "k_upward<{p}>"}


def m2p_kernel_symbol(family, p, shape):
    """rocprofv3's name of the M2P kernel that the tuned tile shape launches
    (shapes 1 and 2 the row-staged kernel, 0 and 3 the direct one without and
    with crossbar B fragments)."""
    if family == "m2p_f32" and shape in (1, 2):
        return f"k_m2p_s<float, {p}, {shape}>"
    return SYMBOLS.get(family, "").format(p=p, xb="true" if shape == 3 else "false")


def measured_traffic(family, p, workload, shape=0):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary of this
    kernel and workload, or None (none taken, or the kernels changed since)."""
    import glob
    sys.path.insert(0, ROOT)
    from bench_profile import source_hash
    want = m2p_kernel_symbol(family, p, shape)
    for f in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        try:
            t = json.load(open(f))
        except (OSError, ValueError):
            continue
        if t.get("kernel") == want and t.get("workload") == workload and t.get("source_sha256") == source_hash():
            return t["traffic_bytes_per_launch"], os.path.relpath(f, ROOT)
    return None, None


def roofline(res, precision, p=None, workload=None):
    """Roofline of the kernel family with the largest summed time in the timed region."""
    prof = res["kernels"]
    name, k = max(prof.items(), key=lambda kv: kv[1]["ms"])
    total_ms = sum(v["ms"] for v in prof.values())
    shapes = res.get("m2p_shape") or (res.get("autotune") or {}).get("m2p_shape") or [0, 0]
    shape = shapes[1 if name.endswith("f32") else 0]
    traffic, tsrc = measured_traffic(name, p, workload, shape) if p is not None else (None, None)
    kname = KERNEL_NAMES.get(name, name)
    if name.startswith("m2p_"):
        kname = (f"k_m2p_s<float, P, {shape}>" if shape in (1, 2) and name == "m2p_f32"
                 else kname.replace("XB", "true" if shape == 3 else "false"))
    common = {"kernel": kname, "family": name, "launches": k["launches"],
              "traffic_source": tsrc,
              "avg_launch_ms": k["ms"] / max(k["launches"], 1),
              "flops_per_launch": k["flops"] / max(k["launches"], 1),
              "bytes_per_launch": k["bytes"] / max(k["launches"], 1), "share_of_step": k["ms"] / total_ms}
    if name in ("gather", "upward", "l2l"):
        achieved = k["bytes"] / (k["ms"] * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm"], "unit": "GB/s",
                "frac": achieved / PEAK["hbm"], "traffic": traffic, **common}
    tf = k["flops"] / (k["ms"] * 1e-3) / 1e12 if k["ms"] > 0 else 0.0
    fp = "fp32" if name.endswith("f32") else "fp64"
    if name in MFMA_FAMILIES:
        peak = PEAK[f"{fp}_mfma"]
        return {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
                "traffic": traffic, **common}
    peak = PEAK[f"{fp}_vector"]
    return {"bound": "alu", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
            "traffic": traffic, **common}


def kernel_table(res):
    out = {}
    for name, k in res["kernels"].items():
        sec = k["ms"] * 1e-3
        out[name] = {"ms_per_step": k["ms"] / res["steps"], "launches_per_step": k["launches"] / res["steps"],
                     "tflops": k["flops"] / sec / 1e12 if sec > 0 else 0.0,
                     "gbps": k["bytes"] / sec / 1e9 if sec > 0 else 0.0}
    return out


def clustered_sample(h, nclusters, seed=0):
    """All leaves under `nclusters` random cells of level levelmin-2 (targets that share
    their ancestors' local expansions, as in a full solve)."""
    rng = np.random.default_rng(seed)
    cl = max(h.levelmin - 2, 1)
    lev = h.level_of()
    ijk = h.flat_ijk().astype(np.int64)
    anc = ijk >> (lev - cl)[:, None]
    key = (anc[:, 0] << 40) | (anc[:, 1] << 20) | anc[:, 2]
    leaf = h.leaf_mask()
    ukeys = np.unique(key[leaf])
    pick = rng.choice(ukeys, size=min(nclusters, ukeys.size), replace=False)
    return np.nonzero(leaf & np.isin(key, pick))[0]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(h, m, p, budget_s, gpu_outputs, min_s=10.0):
    """The FP64 oracle on the host cores, timed on the same workload.  When a full
    solve (upward pass + every leaf) fits the budget it is repeated until at least
    `min_s` seconds have run; otherwise the upward pass plus the leaves under a
    set of random level-(levelmin-2) cells, grown until the evaluation takes at
    least `min_s`, scaled to all leaves.  Also returns the GPU forms' errors
    against the oracle on the evaluated leaves."""
    import oracle
    o = oracle.Oracle(h, p)
    nleaf = h.nleaves()
    leaves = np.nonzero(h.leaf_mask())[0]
    t0 = time.perf_counter()
    o.rebuild(h.levelmin, m)
    t_up = time.perf_counter() - t0
    pilot = clustered_sample(h, 32, seed=11)
    t0 = time.perf_counter()
    o.eval_sample(pilot)
    t_pilot = max(time.perf_counter() - t0, 1e-3)
    est_full = t_up + t_pilot * nleaf / pilot.size
    if est_full <= budget_s / 2:
        reps, total = 0, 0.0
        while True:
            t0 = time.perf_counter()
            o.rebuild(h.levelmin, m)
            po, ao = o.eval_sample(leaves)
            dt = time.perf_counter() - t0
            reps += 1
            total += dt
            if total >= min_s or total + dt > budget_s:
                break
        sample = leaves
        value = nleaf * reps / total
        desc = f"full oracle solves (upward pass + all {nleaf} leaves), {reps} repetitions, {total:.1f} s"
        seconds = total
    else:
        ncl = max(1, int(32 * (min_s - t_up) / t_pilot))
        while True:
            sample = clustered_sample(h, ncl, seed=1)
            t0 = time.perf_counter()
            po, ao = o.eval_sample(sample)
            t_eval = time.perf_counter() - t0
            if t_eval >= min_s or sample.size >= leaves.size or t_up + 2 * t_eval > budget_s:
                break
            ncl = int(ncl * min(4.0, max(1.5, min_s / max(t_eval, 1e-3))))
        value = nleaf / (t_up + t_eval * nleaf / sample.size)
        desc = (f"oracle upward pass over all {nleaf} leaves ({t_up:.2f} s) + evaluation of {sample.size} leaves "
                f"under random level-{max(h.levelmin - 2, 1)} cells ({t_eval:.2f} s), scaled to all leaves")
        seconds = t_up + t_eval
    errs = {}
    for form, (phi, acc) in gpu_outputs.items():
        da = np.linalg.norm(acc[sample] - ao, axis=1)
        ra = np.linalg.norm(ao, axis=1)
        errs[form] = {
            "rel_l2_acc": float(np.linalg.norm(acc[sample] - ao) / np.linalg.norm(ao)),
            "rel_l2_phi": float(np.linalg.norm(phi[sample] - po) / np.linalg.norm(po)),
            "max_acc_over_max": float(np.abs(acc[sample] - ao).max() / np.abs(ao).max()),
            "p99_cell_rel_acc": float(np.percentile(da[ra > 0] / ra[ra > 0], 99)),
            "leaves": int(sample.size),
        }
    base = {"value": value, "unit": "cells/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": desc, "seconds": seconds, "cpu_model": cpu_model()}
    return base, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg3", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"])
    ap.add_argument("--overlap", action="store_true", help="also time the two-stream schedule (AFMM_OVERLAP)")
    ap.add_argument("--no-ats", action="store_true", help="skip the adaptive-time-step cycle")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timings (AFMM_GRAPH)")
    ap.add_argument("--binary", action="store_true", help="also run the binary-orbit time loop (levelmax 6, 7, 8)")
    ap.add_argument("--p", type=int, default=4, help="expansion order of the batched workload (cfg4)")
    ap.add_argument("--members", type=int, default=256, help="hierarchies in the batched workload (cfg4)")
    ap.add_argument("--adjoint", action="store_true", help="also time the adjoint pass (default for cfg5)")
    ap.add_argument("--ats", action="store_true", help="also time one adaptive-time-step cycle (default for cfg3)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-periodic", action="store_true", help="skip the periodic-box timing")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form run")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tap splits")
    ap.add_argument("--m2p-shape", type=int, default=0,
                    help="M2P tile shape of the plans when the autotuner is off (afmm_options.m2p_shape)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (reference for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on one GPU; sharding over several GPUs is not built, "
              "so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        src = torch.ones(256 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "cfg4":
        run_batch(args)
        return
    w, desc = make_workload(args.workload)
    h, m = w.hierarchy, w.mass
    mass_t = torch.from_numpy(m).cuda()
    print(f"[bench] workload {w.name}: {h.nleaves()} leaves", file=sys.stderr, flush=True)

    r32, phi32, acc32 = time_form(h, mass_t, w.p, "fp32", args.steps, args.warmup, autotune=not args.no_autotune, m2p_shape=args.m2p_shape)
    print(f"[bench] fp32 form: {r32['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    r32s = None
    if args.overlap:
        r32s, _, _ = time_form(h, mass_t, w.p, "fp32", args.steps, 1, overlap=True, autotune=not args.no_autotune, m2p_shape=args.m2p_shape)
        print(f"[bench] fp32 form, two streams: {r32s['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    outputs = {"fp32": (phi32, acc32)}
    r32g = None
    if not args.no_graph:
        r32g, phi32g, acc32g = time_form(h, mass_t, w.p, "fp32", args.steps, args.warmup, graph=True,
                                         autotune=not args.no_autotune, m2p_shape=args.m2p_shape)
        print(f"[bench] fp32 form, graph replay: {r32g['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        # identical bits to the eager solves when the tuner chose the same splits
        same = (r32g["autotune"] or {}).get("m2l_split") == (r32["autotune"] or {}).get("m2l_split") and \
            (r32g["autotune"] or {}).get("m2p_split") == (r32["autotune"] or {}).get("m2p_split")
        graph_equal = bool(np.array_equal(phi32g, phi32) and np.array_equal(acc32g, acc32)) if same else None
    r64 = None
    if not args.no_fp64:
        r64, phi64, acc64 = time_form(h, mass_t, w.p, "fp64", max(args.steps // 2, 1), 1,
                                      autotune=not args.no_autotune, m2p_shape=args.m2p_shape)
        outputs["fp64"] = (phi64, acc64)
        print(f"[bench] fp64 form: {r64['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    ats = None
    if args.ats or (args.workload == "cfg3" and not args.no_ats):
        ats = time_ats(h, mass_t, w.p, "fp32")
        print(f"[bench] ATS step: {ats['solves']} solves in {ats['sequence_ms']:.2f} ms", file=sys.stderr, flush=True)
        if not args.no_graph:
            atsg = time_ats(h, mass_t, w.p, "fp32", graph=True)
            ats["graph_sequence_ms"] = atsg["sequence_ms"]
            ats["graph_leaf_updates_per_s"] = atsg["leaf_updates_per_s"]
            print(f"[bench] ATS step, graph replay: {atsg['sequence_ms']:.2f} ms", file=sys.stderr, flush=True)
        atsd = time_ats(h, mass_t, w.p, "fp32", drift=True)
        ats["drift_sequence_ms"] = atsd["sequence_ms"]
        ats["drift_mean_ms_per_solve_by_level"] = atsd["mean_ms_per_solve_by_level"]
        print(f"[bench] ATS step, drifted stale trees: {atsd['sequence_ms']:.2f} ms", file=sys.stderr, flush=True)

    adj = None
    if args.adjoint or args.workload == "cfg5":
        adj = time_adjoint(h, mass_t, w.p, "fp32", max(args.steps // 4, 2))
        print(f"[bench] adjoint {adj['adjoint_ms']:.3f} ms vs forward {adj['forward_ms']:.3f} ms",
              file=sys.stderr, flush=True)

    periodic = None
    if not args.no_periodic:
        # the same hierarchy and masses on a periodic box (AFMM_PERIODIC), autotuned like
        # the isolated form; its plan creation includes, for the first periodic plan of
        # this order, the host's level-2 far-operator table
        try:
            rp, _, _ = time_form(h, mass_t, w.p, "fp32", max(args.steps // 2, 2), 1,
                                 autotune=not args.no_autotune, m2p_shape=args.m2p_shape, periodic=True)
            periodic = {"ms_per_step": rp["ms_per_step"], "value": rp["value"], "unit": "cells/s",
                        "over_isolated": rp["ms_per_step"] / r32["ms_per_step"],
                        "plan_create_ms": rp["plan_create_ms"], "autotune": rp["autotune"],
                        "kernels": kernel_table(rp)}
            print(f"[bench] periodic box: {rp['ms_per_step']:.3f} ms/step "
                  f"({periodic['over_isolated']:.3f}x isolated), plan {rp['plan_create_ms']:.0f} ms",
                  file=sys.stderr, flush=True)
        except RuntimeError as e:   # AfmmError: a hierarchy graded only inside the box
            periodic = {"skipped": str(e)}

    binary = None
    if args.binary:
        binary = [run_binary(lm) for lm in (6, 7, 8)]
        for b in binary:
            print(f"[bench] binary orbit {b['levels']}: {b['ms_per_step']:.2f} ms/step, {b['plans']} plans",
                  file=sys.stderr, flush=True)

    base, errs = (None, None)
    if not args.no_cpu:
        base, errs = cpu_baseline(h, m, w.p, args.cpu_seconds, outputs)
        print(f"[bench] cpu oracle baseline {base['value']:.3e} cells/s", file=sys.stderr, flush=True)

    info = r32["info"]
    line = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {desc}", "p": w.p, "precision": "FP32 mixed (FP64 P2M/M2M, "
                   "FMM levels <= 3 and outputs)", "leaves": info["nleaves"], "levels": [h.levelmin, h.levelmax]},
        "roofline": roofline(r32, "fp32", w.p, w.name),
        "cpu_baseline": base,
        "fp64_form": None if r64 is None else {"value": r64["value"], "unit": "cells/s",
                                                "ms_per_step": r64["ms_per_step"], "dtype": "f64",
                                                "roofline": roofline(r64, "fp64", w.p, w.name)},
        "fp32_over_fp64": None if r64 is None else r32["value"] / r64["value"],
        "plan_create_ms": {"fp32": r32["plan_create_ms"], "fp64": None if r64 is None else r64["plan_create_ms"]},
        "end_to_end_first_solve_ms": r32["plan_create_ms"] + r32["ms_per_step"],
        "overlap_ms_per_step": None if r32s is None else r32s["ms_per_step"],
        "graph": None if r32g is None else {"ms_per_step": r32g["ms_per_step"], "value": r32g["value"],
                                            "eager_ms_per_step": r32["ms_per_step"],
                                            "bitwise_equal_to_eager": graph_equal,
                                            "autotune": r32g["autotune"]},
        "autotune_fp32": r32["autotune"], "autotune_fp64": None if r64 is None else r64["autotune"],
        "profiled_ms_per_step": sum(v["ms"] for v in r32["kernels"].values()) / r32["steps"],
        "error_vs_oracle_sample": errs,
        "algorithmic_flops_per_step": info["flops_m2l"] + info["flops_m2p"] + info["flops_p2p"]
        + info["flops_updown"],
        "kernels_fp32": kernel_table(r32),
        "kernels_fp64": None if r64 is None else kernel_table(r64),
        "adjoint": adj,
        "periodic": periodic,
        "ats_step": ats,
        "binary_orbit": binary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
