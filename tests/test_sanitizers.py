"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (CPU only).

- The HIP library's host side (plan validation, Morton sort, neighbour rows,
  group lists, work counts, translation-table generation, option checks, the
  max_device_bytes path) is compiled by hipcc with the sanitizers on the host
  pass only (every -fsanitize= right after -Xarch_host: device code is built
  as usual) and driven through the C ABI on valid and invalid hierarchies.
- The oracle is compiled by gcc with the same sanitizers and runs full solves,
  the option pins' code paths and the building blocks.

Each build is loaded in a fresh Python process with the sanitizer runtime
preloaded; any report aborts the process and fails the test.  No GPU is used.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "paper_2607_19489_amd", "_build", "sanitize")
SAN = "-fsanitize=address,undefined"
ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(script, preload):
    env = dict(os.environ, **ENV, LD_PRELOAD=preload, PYTHONPATH=ROOT, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(script)], env=env, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_oracle_under_asan_ubsan():
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", SAN, "-fopenmp", "-shared", "-fPIC",
                           "-std=c11", os.path.join(ROOT, "oracle", "afmm_oracle.c"), "-o", lib, "-lm"])
    preload = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    out = _run(f"""
        import numpy as np, oracle
        oracle.LIB = {lib!r}
        oracle._lib = None
        from synth import cell_masses, plummer, unigrid
        from synth.hierarchy import build_graded, refine_sphere
        h = build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {{3: 0.3, 4: 0.2}}))
        m = cell_masses(h, plummer(1.0, 0.1), 0.01, 1)
        for p in (1, 4, 8):
            for cap, selfp in ((False, False), (True, True)):
                po, ao = oracle.Oracle(h, p, quad_cap=cap, self_potential=selfp).solve_all(m)
                assert np.all(np.isfinite(po[h.leaf_mask()]))
        o = oracle.Oracle(h, 4)
        o.solve(3, 1, m, np.zeros(h.total), np.zeros((h.total, 3)))
        o.solve(4, 2, m, np.zeros(h.total), np.zeros((h.total, 3)))
        o.chain_check(5)
        o.set_merged_all(True)
        o.solve_all(m)
        x = np.random.default_rng(0).uniform(size=(50, 3))
        oracle.direct(x, np.ones(50), x)
        oracle.derivs(9, [0.3, -0.2, 0.7])
        oracle.self_constant()
        try:
            oracle.Oracle(build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {{3: 0.05, 4: 0.3}})), 4)
        except oracle.OracleError:
            pass
        print("ORACLE_SAN_OK")
    """, preload)
    assert "ORACLE_SAN_OK" in out


def test_host_runtime_under_asan_ubsan():
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not installed")
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang ASan runtime not found")
    sys.path.insert(0, ROOT)
    from paper_2607_19489_amd import build as B
    os.makedirs(OUT, exist_ok=True)
    objs, procs = [], []
    for src in B.SOURCES:
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc, *B.flags(), "-O1", "-g", "-fno-omit-frame-pointer", "-Xarch_host", SAN,
               "-c", "-x", "hip", os.path.join(B.CSRC, src), "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode(errors="replace")[-4000:]
    lib = os.path.join(OUT, "libafmm_san.so")
    subprocess.check_call([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-Xarch_host", SAN,
                           "-shared-libsan", *objs, "-o", lib])
    out = _run(f"""
        import ctypes as C
        import numpy as np
        from paper_2607_19489_amd import _lib
        _lib.LIB_PATH = {lib!r}
        _lib._lib = None
        import paper_2607_19489_amd as A
        from synth import configs, unigrid
        from synth.hierarchy import Hierarchy, build_graded, refine_sphere
        h = build_graded(3, 6, refine_sphere((0.3, 0.5, 0.6), {{3: 0.3, 4: 0.2, 5: 0.1}}))
        for p in range(1, 9):
            A.hierarchy_check(h, p=p, precision="fp32")
            A.hierarchy_check(h, p=p, quad_cap=True, self_potential=True)
        A.hierarchy_check(configs.cfg2().hierarchy, p=6)
        A.hierarchy_check(unigrid(1), p=2)
        bad = Hierarchy(h.levelmin, h.levelmax, [a.copy() for a in h.ijk], [r.copy() for r in h.refined])
        bad.ijk[1][3] = bad.ijk[1][4]
        for hh, p in ((bad, 4), (h, 9), (build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {{3: 0.05, 4: 0.3}})), 4)):
            try:
                A.hierarchy_check(hh, p=p)
            except A.AfmmError:
                pass
        o = A.make_options(p=4, max_device_bytes=1)
        arrs = A.afmm._hierarchy_arrays(h)
        hc = A.afmm._hier_struct(*arrs)
        ptr = C.c_void_p()
        assert _lib.lib().afmm_plan_create(C.byref(hc), C.byref(o), None, C.byref(ptr)) == -5
        assert _lib.lib().afmm_status_string(-99) == b"unknown status"
        print("HOST_SAN_OK")
    """, rt[0])
    assert "HOST_SAN_OK" in out
