"""AddressSanitizer + UndefinedBehaviorSanitizer on the host code: the C
oracle and the library's host driver (planner, selector, batched planner,
argument checks), each rebuilt with gcc -fsanitize=address,undefined into a
temporary directory and driven in a child process with the sanitizer runtime
preloaded.  Any report fails the child (halt_on_error).  The device code is
the normal build's objects (no GPU needed: nothing is launched)."""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_10131_amd", "csrc")
OBJS = os.path.join(ROOT, "paper_2010_10131_amd", "_build")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _asan_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("gcc's libasan is not installed")
    return p


def _run_child(code, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = _asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=99"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=98"
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], capture_output=True, text=True,
                       env=env, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", *SAN, "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           os.path.join(ROOT, "oracle", "sthosvd_oracle.c"), "-o", lib, "-lm"])
    out = _run_child("""
        import numpy as np, oracle
        oracle._LIB = %r
        import workloads as wl
        X = wl.lowrank_plus_noise((9, 7, 5), (3, 2, 2), "0.9", 1e-3, 5, "float64")
        L0 = [wl.gaussian_init(d, r, 3, n) for n, (d, r) in enumerate(zip((9, 7, 5), (3, 2, 2)))]
        for meth in ([0, 0, 0], [1, 1, 1], [0, 1, 0]):
            G, U, _ = oracle.sthosvd(X, (3, 2, 2), methods=meth, L0=L0)
            Xh = oracle.reconstruct(G, U)
            assert np.linalg.norm(Xh - X) <= 1e-2 * np.linalg.norm(X)
        S = np.asfortranarray(np.random.default_rng(1).standard_normal((11, 11)))
        lam, V, _ = oracle.jacobi_eig(S + S.T)
        Y = wl.lowrank_plus_noise((6, 5, 4, 3), (2, 2, 2, 2), "2^-k", 1e-4, 6, "float64")
        G, U, _ = oracle.sthosvd(Y, (2, 2, 2, 2), order=[3, 1, 0, 2])
        print("oracle ok")
    """ % lib, {"OMP_NUM_THREADS": "2"})
    assert "oracle ok" in out


def test_host_driver_under_asan_ubsan(tmp_path):
    objs = sorted(glob.glob(os.path.join(OBJS, "*.hip.o")))
    if not objs:
        pytest.skip("the library is not built (paper_2010_10131_amd/build.py)")
    host = []
    for f in ("api.cpp", "selector.cpp"):
        o = str(tmp_path / (f + ".o"))
        subprocess.check_call(["g++", "-std=c++17", *SAN, "-fPIC", "-D__HIP_PLATFORM_AMD__",
                               "-I/opt/rocm/include", "-c", os.path.join(CSRC, f), "-o", o])
        host.append(o)
    lib = str(tmp_path / "libsthosvd_san.so")
    subprocess.check_call(["g++", "-shared", "-fsanitize=address,undefined", "-o", lib, *host, *objs,
                           "-L/opt/rocm/lib", "-lamdhip64"])
    out = _run_child("""
        import ctypes
        from paper_2010_10131_amd import _lib
        _lib.LIB_PATH = "@LIB@"
        L = _lib.load()
        assert L.sth_version().startswith(b"sthosvd")

        def plan(dims, ranks, solver=0, per_mode=None, mode_order=None, cap=0, dtype=1, gp=1, tp=1):
            d = _lib.sth_desc()
            N = len(dims)
            da, ra = (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks)
            d.order, d.dims, d.ranks = N, da, ra
            keep = [da, ra]
            if per_mode:
                pm = (ctypes.c_int32 * N)(*per_mode); keep.append(pm); d.per_mode = pm
            if mode_order:
                mo = (ctypes.c_int32 * N)(*mode_order); keep.append(mo); d.mode_order = mo
            d.dtype, d.gram_prec, d.ttm_prec, d.solver = dtype, gp, tp, solver
            d.als_iters, d.eig_max_sweeps, d.workspace_cap = 5, 0, cap
            h, ws = ctypes.c_void_p(), ctypes.c_size_t()
            st = L.sthosvd_plan(ctypes.byref(d), ctypes.byref(h), ctypes.byref(ws))
            if st == 0:
                out = (ctypes.c_int32 * N)()
                assert L.sthosvd_plan_solvers(h, out) == 0
                L.sthosvd_plan_destroy(h)
                return st, list(out), ws.value
            L.sth_last_error()
            return st, None, 0

        cases = [((16, 12, 10), (4, 3, 2)), ((512, 64, 64), (32, 8, 8)), ((30648, 12, 10), (6, 5, 4)),
                 ((48,) * 5, (8,) * 5), ((160,) * 4, (16,) * 4), ((64, 2, 2), (5, 2, 2)), ((7,), (3,))]
        for dims, ranks in cases:
            for solver in (0, 1, 2, 3):
                plan(dims, ranks, solver)
            plan(dims, ranks, 2, cap=1 << 20)
            plan(dims, ranks, 2, mode_order=list(range(len(dims)))[::-1])
        plan((16, 12, 10), (4, 3, 2), dtype=0, gp=0, tp=0)
        for bad in (((16, 0, 10), (4, 3, 2)), ((16, 12, 10), (4, 13, 2)), ((2,) * 9, (1,) * 9)):
            assert plan(*bad)[0] != 0
        assert plan((16, 12, 10), (4, 3, 2), per_mode=[0, 5, 0])[0] != 0
        assert plan((16, 12, 10), (4, 3, 2), mode_order=[0, 0, 1])[0] != 0
        # selector inference
        f = (ctypes.c_float * 10)()
        y = (ctypes.c_float * 2)()
        c = ctypes.c_int32()
        for I, R, J in ((512, 64, 262144), (48, 8, 5308416), (30648, 6, 120), (3, 1, 2)):
            assert L.sth_selector_features(I, R, J, f) == 0
            assert L.sth_selector_predict(None, I, R, J, y) == 0
            assert L.sth_selector_choose(None, I, R, J, ctypes.byref(c)) == 0
            assert L.sth_selector_tree_choose(I, R, J, ctypes.byref(c)) == 0
        # batched planner (tables for many shapes)
        shapes = [((32 + 7 * k, 40 + 5 * k, 36 + 3 * k), (4 + k % 5, 5, 6)) for k in range(24)]
        descs = (_lib.sth_desc * len(shapes))()
        keep = []
        for k, (dims, ranks) in enumerate(shapes):
            da, ra = (ctypes.c_int64 * 3)(*dims), (ctypes.c_int64 * 3)(*ranks)
            keep += [da, ra]
            descs[k].order, descs[k].dims, descs[k].ranks = 3, da, ra
            descs[k].dtype, descs[k].gram_prec, descs[k].ttm_prec = 1, 3, 2
        h, ws = ctypes.c_void_p(), ctypes.c_size_t()
        st = L.sthosvd_plan_batched(descs, len(shapes), ctypes.byref(h), ctypes.byref(ws))
        if st == 0:
            L.sthosvd_plan_batched_destroy(h)
        # workspace queries
        dims = (ctypes.c_int64 * 3)(64, 48, 40)
        ranks = (ctypes.c_int64 * 3)(8, 6, 5)
        L.tucker_reconstruct_workspace(3, dims, ranks, 1)
        L.tucker_error_workspace(3, dims, ranks, 1)
        L.sth_hooi_workspace(3, dims, ranks, 1, 1)
        L.gram_mode_n_workspace(3, dims, 1, 1)
        L.eig_leading_workspace(512)
        L.ttm_factor_bytes(512, 64, 2)
        L.sthosvd_mode_step_workspace(3, dims, 0, 8, 0, 1, 1, 1, 5)
        print("driver ok")
    """.replace("@LIB@", lib), {})
    assert "driver ok" in out
