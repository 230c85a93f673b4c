"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the oracle (built with g++ -fsanitize=address,undefined) through every
entry point on small grids, and the HIP library's host logic (its host code
built with the same sanitizers by hipcc, device code as usual) through context
creation, options, plan policies and the launch-geometry description, which
make no GPU call.  Each runs in a child process with the sanitizer runtime
preloaded; any report (or a non-zero exit) fails the test.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow

ORACLE_SCRIPT = textwrap.dedent('''
    import sys
    sys.path.insert(0, %(root)r)
    import numpy as np
    import oracle
    from paper_1603_08893_amd import microstructure as ms
    oracle.use_library(%(lib)r)
    x = np.random.default_rng(0).standard_normal(12) + 0j
    assert np.allclose(oracle.fft1d(x), oracle.dft1d_naive(x))
    a = np.random.default_rng(1).standard_normal((4, 6, 5)) + 0j
    assert np.allclose(oracle.fft3d(a), oracle.dft3d_naive(a))
    for shape in ((5, 5, 5), (6, 4, 7)):
        A = ms.random_field(shape, seed=2)
        for nyq in (False, True):
            G = oracle.project(A, nyq_identity=nyq)
            assert np.allclose(oracle.project(G, nyq_identity=nyq), G)
    shape = (6, 5, 7)
    ph = ms.laminate(shape, 0, 0.4)
    table = [(0.833, 0.386), (8.33, 3.86)]
    K, mu = ms.phase_moduli(ph, table)
    F = ms.near_identity_field(shape, seed=3, scale=0.02)
    p = ms.random_field(shape, seed=4)
    oracle.svk_stress(F, K, mu)
    oracle.svk_tangent(F, K, mu, p)
    b = oracle.project(oracle.apply_operator(F, K, mu, p))
    oracle.cg(F, K, mu, b)
    for m, lo, hi in (("chebyshev", 0.3, 30.0), ("richardson", 0.3, 30.0), ("gmres", 5, 0.0)):
        oracle.krylov(F, K, mu, b, m, lo, hi, max_it=200)
    st, Fn, P, Pbar, S = oracle.solve_increment(K, mu, oracle.identity_field(shape), ms.simple_shear(0.05))
    assert st == 0
    oracle.solve_increment(K, mu, oracle.identity_field(shape), ms.simple_shear(0.05), nyq_identity=True)
    oracle.solve_increment_krylov(K, mu, oracle.identity_field(shape), ms.simple_shear(0.05), "gmres", 10, 0.0)
    oracle.macro_tangent(K, mu, Fn)
    mask = np.zeros(9); mask[4] = mask[8] = 1
    oracle.solve_increment_mixed(K, mu, oracle.identity_field(shape), np.eye(3).reshape(9) + 0.01 * np.eye(9)[0],
                                 mask, np.zeros(9))
    oracle.adjoint(K, mu, Fn, np.ones(9))
    w, V = oracle.jacobi_eig3(np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]]))
    t = np.asarray([(0.833, 0.386, 0.003, 0.01), (0.833, 0.386, 0.006, 0.01)])
    Kj, muj, ty, H = (t[ph, k].copy() for k in range(4))
    h = oracle.virgin_history(shape)
    oracle.j2_stress(F, Kj, muj, ty, H, h)
    oracle.j2_tangent(F, Kj, muj, ty, H, h, p)
    Fj = oracle.identity_field(shape)
    for g in (0.004, 0.008):
        st, Fj, _, _, h, _ = oracle.solve_increment_j2(Kj, muj, ty, H, h, Fj, ms.simple_shear(g))
        assert st == 0
    oracle.solve_increment_j2(Kj, muj, ty, H, h, Fj, np.diag([-0.5, 1.0, 1.0]).reshape(9))
    oracle.solve_increment_mixed_j2(Kj, muj, ty, H, h, Fj, np.eye(3).reshape(9), mask, np.zeros(9))
    print("oracle sanitized run ok")
''')

HOST_SCRIPT = textwrap.dedent('''
    import ctypes, sys
    sys.path.insert(0, %(root)r)
    from paper_1603_08893_amd import fftnk
    fftnk._LIB_PATH = %(lib)r
    L = fftnk.lib()
    cells = [[(128, 128, 128)], [(31, 31, 31)], [(451, 451, 2)], [(452, 7, 113)], [(96, 48, 192)], [(2, 2, 2)],
             [(32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 96, 96), (7, 9, 11)], [(509, 3, 5)], [(12, 6, 8)]]
    for dims in cells:
        for prec in ("fp64", "fp32"):
            for pol in (0, 1, 7, 9, 17, 32, 55):
                fftnk.describe(dims, precision=prec, gmres_restart=(8 if pol == 9 else 0), policy=pol)
    ctx = ctypes.c_void_p()
    assert L.fftnk_create(ctypes.byref(ctx), 1, 8, 8, 0, None) == fftnk.EINVAL
    assert L.fftnk_create(ctypes.byref(ctx), 513, 8, 8, 0, None) == fftnk.EUNSUPPORTED
    assert L.fftnk_create(ctypes.byref(ctx), 24, 20, 16, 0, None) == fftnk.OK
    for opt, val in ((fftnk.OPT_GMRES_RESTART, 12), (fftnk.OPT_J2_TANGENT, 1), (fftnk.OPT_NYQUIST, 1),
                     (fftnk.OPT_CHECK_EVERY, 8), (fftnk.OPT_GRAPHS, 0), (fftnk.OPT_X_WINDOW, 5)):
        assert L.fftnk_set_option(ctx, opt, val) == fftnk.OK
    assert L.fftnk_set_option(ctx, fftnk.OPT_J2_TANGENT, 2) == fftnk.EINVAL
    assert L.fftnk_workspace_bytes(ctx) > 0
    assert L.fftnk_set_plan(ctx, 5) == fftnk.OK
    assert L.fftnk_solve_increment(ctx, None, 1e-5, 1e-8, 50, 100, None, None, None, None) != fftnk.OK
    L.fftnk_destroy(ctx)
    for s in range(12):
        L.fftnk_status_string(s)
    print("host logic sanitized run ok")
''')


def _run(script, preload, env_extra):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=900, env=env)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    return report


SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no libasan for g++")
    lib = str(tmp_path / "liboracle_san.so")
    oracle.build(force=True, path=lib, flags=["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                              "-fno-sanitize-recover=all"])
    out = _run(ORACLE_SCRIPT % {"root": ROOT, "lib": lib}, asan, SAN_ENV)
    assert "oracle sanitized run ok" in out


def test_host_logic_under_sanitizers(tmp_path):
    from paper_1603_08893_amd import build as b
    rts = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("no clang ASan runtime in the ROCm toolchain")
    lib = b.build(out=str(tmp_path / "libfftnk_san.so"), sanitize=True)
    out = _run(HOST_SCRIPT % {"root": ROOT, "lib": lib}, rts[0], SAN_ENV)
    assert "host logic sanitized run ok" in out
