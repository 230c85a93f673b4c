"""ctypes binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

The oracle (``fftnk_oracle.cpp``) is a plain single-threaded implementation of
the finite-strain FFT Newton-Krylov method of de Geus et al. (CMAME 2017).  It is
the parity reference for the HIP library and shares no code with it.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this
module; the library itself never does.

Arrays are numpy float64, tensor fields shaped ``(9, n0, n1, n2)`` (component
``c = 3*i + j``, axis a2 fastest).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fftnk_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_SOLVES = 64

STATUS = {0: "ok", 1: "cg_maxit", 2: "cg_breakdown", 3: "newton_maxit", 4: "nonfinite", 5: "einval",
          6: "return_map_fail"}


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("n_solves", ctypes.c_int),
        ("cg_iters", ctypes.c_int * MAX_SOLVES),
        ("newton_res", ctypes.c_double * MAX_SOLVES),
        ("cg_relres", ctypes.c_double * MAX_SOLVES),
    ]

    def as_dict(self):
        k = self.n_solves
        return {
            "status": self.status,
            "n_solves": k,
            "cg_iters": list(self.cg_iters[:k]),
            "newton_res": list(self.newton_res[:k]),
            "cg_relres": list(self.cg_relres[:k]),
        }


FLAGS = ["-O2", "-fcx-limited-range"]
TIMED_FLAGS = ["-O3", "-march=native", "-fcx-limited-range"]  # the build the CPU baseline is timed with


def build(force=False, path=None, flags=None):
    """Compile the oracle with g++ (no GPU code, no shared sources): the test
    build in-tree, or with `flags` to `path` (e.g. the timed build)."""
    out = path or _LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++"] + (flags or FLAGS) + ["-std=c++17", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, out)
    return out


_lib = None
_lib_path = _LIB


def use_library(path):
    """Load the oracle from another build of the same source (before any call)."""
    global _lib, _lib_path
    _lib_path = path
    _lib = None


def lib():
    global _lib
    if _lib is None:
        if _lib_path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_lib_path)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        L.orc_fft1d.argtypes = [dp, i, i]
        L.orc_dft1d_naive.argtypes = [dp, dp, i, i]
        L.orc_fft3d.argtypes = [dp, i, i, i, i]
        L.orc_dft3d_naive.argtypes = [dp, dp, i, i, i, i]
        L.orc_project.argtypes = [i, i, i, dp, dp]
        L.orc_project_nyq.argtypes = [i, i, i, dp, dp, i]
        L.orc_svk_stress.argtypes = [ctypes.c_long, dp, dp, dp, dp]
        L.orc_svk_tangent.argtypes = [ctypes.c_long, dp, dp, dp, dp, dp]
        L.orc_apply_operator.argtypes = [i, i, i, dp, dp, dp, dp, dp]
        L.orc_cg.argtypes = [i, i, i, dp, dp, dp, dp, dp, ctypes.c_double, i,
                             ctypes.POINTER(i), dp]
        L.orc_cg.restype = i
        L.orc_krylov.argtypes = [i, i, i, dp, dp, dp, dp, dp, ctypes.c_double, i, i, ctypes.c_double,
                                 ctypes.c_double, ctypes.POINTER(i), dp]
        L.orc_krylov.restype = i
        L.orc_solve_increment_krylov.argtypes = [i, i, i, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                                 i, i, dp, dp, ctypes.POINTER(Stats), i, ctypes.c_double,
                                                 ctypes.c_double]
        L.orc_solve_increment_krylov.restype = i
        L.orc_solve_increment_krylov_nyq.argtypes = L.orc_solve_increment_krylov.argtypes + [i]
        L.orc_solve_increment_krylov_nyq.restype = i
        L.orc_solve_increment.argtypes = [i, i, i, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                          i, i, dp, dp, ctypes.POINTER(Stats)]
        L.orc_solve_increment.restype = i
        L.orc_solve_increment_nyq.argtypes = [i, i, i, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                              i, i, dp, dp, ctypes.POINTER(Stats), i]
        L.orc_solve_increment_nyq.restype = i
        ip = ctypes.POINTER(i)
        L.orc_macro_tangent.argtypes = [i, i, i, dp, dp, dp, ip, ctypes.c_double, i, dp]
        L.orc_macro_tangent.restype = i
        L.orc_solve_increment_mixed.argtypes = [i, i, i, dp, dp, dp, dp, ip, dp, ctypes.c_double, i,
                                                ctypes.c_double, ctypes.c_double, i, i, dp, dp,
                                                ctypes.POINTER(Stats), ip]
        L.orc_solve_increment_mixed.restype = i
        L.orc_solve_increment_mixed_j2.argtypes = [i, i, i, dp, dp, dp, dp, dp, dp, dp, ip, dp, ctypes.c_double,
                                                   i, ctypes.c_double, ctypes.c_double, i, i, dp, dp,
                                                   ctypes.POINTER(Stats), ip]
        L.orc_solve_increment_mixed_j2.restype = i
        L.orc_adjoint.argtypes = [i, i, i, dp, dp, dp, dp, ctypes.c_double, i, dp, dp, ctypes.POINTER(i)]
        L.orc_adjoint.restype = i
        L.orc_jacobi_eig3.argtypes = [dp, dp, dp]
        L.orc_j2_stress.argtypes = [ctypes.c_long, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_j2_stress.restype = i
        L.orc_j2_tangent.argtypes = [ctypes.c_long, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_j2_tangent.restype = i
        L.orc_solve_increment_j2.argtypes = [i, i, i, dp, dp, dp, dp, dp, dp, dp, ctypes.c_double,
                                             ctypes.c_double, i, i, dp, dp, ctypes.POINTER(Stats)]
        L.orc_solve_increment_j2.restype = i
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- transforms
def fft1d(x, sign=-1):
    x = np.array(x, dtype=np.complex128, copy=True)
    buf = x.view(np.float64)
    lib().orc_fft1d(_p(buf), x.size, sign)
    return x


def dft1d_naive(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    lib().orc_dft1d_naive(_p(x.view(np.float64)), _p(out.view(np.float64)), x.size, sign)
    return out


def fft3d(x, sign=-1):
    x = np.array(x, dtype=np.complex128, copy=True)
    n0, n1, n2 = x.shape
    lib().orc_fft3d(_p(x.view(np.float64).reshape(-1)), n0, n1, n2, sign)
    return x


def dft3d_naive(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    n0, n1, n2 = x.shape
    lib().orc_dft3d_naive(_p(x.view(np.float64).reshape(-1)), _p(out.view(np.float64).reshape(-1)),
                          n0, n1, n2, sign)
    return out


# ---------------------------------------------------------------- projection
def project(A, nyq_identity=False):
    """G(A) for a tensor field A of shape (9, n0, n1, n2) (or (3, 3, n0, n1, n2)).

    nyq_identity selects the even-grid choice of App. C: False, G-hat = 0 at
    Nyquist frequencies (compatible F); True, G-hat = identity there
    (equilibrated stress)."""
    shp = A.shape
    A = _c(A).reshape(9, *shp[-3:])
    out = np.empty_like(A)
    n0, n1, n2 = A.shape[1:]
    if nyq_identity:
        lib().orc_project_nyq(n0, n1, n2, _p(A), _p(out), 1)
    else:
        lib().orc_project(n0, n1, n2, _p(A), _p(out))
    return out.reshape(shp)


# ---------------------------------------------------------------- material
def _fields(F, K, mu):
    F = _c(F)
    grid = F.shape[-3:] if F.ndim >= 4 else F.shape[1:]
    n = int(np.prod(F.shape)) // 9
    K = _c(np.broadcast_to(K, grid) if np.ndim(K) else np.full(grid, float(K)))
    mu = _c(np.broadcast_to(mu, grid) if np.ndim(mu) else np.full(grid, float(mu)))
    return F, K, mu, n


def svk_stress(F, K, mu):
    """First Piola-Kirchhoff stress of St. Venant-Kirchhoff, per voxel."""
    F, K, mu, n = _fields(F, K, mu)
    P = np.empty_like(F)
    lib().orc_svk_stress(n, _p(F), _p(K), _p(mu), _p(P))
    return P


def svk_tangent(F, K, mu, dF):
    """Consistent tangent of St. Venant-Kirchhoff applied to dF."""
    F, K, mu, n = _fields(F, K, mu)
    dF = _c(np.broadcast_to(dF, F.shape))
    out = np.empty_like(F)
    lib().orc_svk_tangent(n, _p(F), _p(K), _p(mu), _p(dF), _p(out))
    return out


def apply_operator(F, K, mu, p):
    """A p = G(K(F) : p), the projected-tangent operator."""
    F, K, mu, n = _fields(F, K, mu)
    p = _c(p).reshape(F.shape)
    out = np.empty_like(F)
    n0, n1, n2 = F.shape[-3:]
    lib().orc_apply_operator(n0, n1, n2, _p(K), _p(mu), _p(F), _p(p), _p(out))
    return out


def cg(F, K, mu, b, eta=1e-8, max_cg=10000):
    F, K, mu, n = _fields(F, K, mu)
    b = _c(b).reshape(F.shape)
    x = np.empty_like(F)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    n0, n1, n2 = F.shape[-3:]
    st = lib().orc_cg(n0, n1, n2, _p(K), _p(mu), _p(F), _p(b), _p(x), eta, max_cg, ctypes.byref(it),
                      ctypes.byref(rel))
    return x, st, it.value, rel.value


METHODS = {"cg": 0, "chebyshev": 1, "richardson": 2, "gmres": 3}


def krylov(F, K, mu, b, method="chebyshev", lo=0.0, hi=0.0, eta=1e-8, max_it=10000):
    """One linear solve A x = b, x0 = 0, with CG, Chebyshev, Richardson
    (spectral bounds [lo, hi] of A on range(G)) or GMRES (lo = restart length).
    Returns (x, status, iterations, final ||r|| / ||b||)."""
    F, K, mu, n = _fields(F, K, mu)
    b = _c(b).reshape(F.shape)
    x = np.empty_like(F)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    n0, n1, n2 = F.shape[-3:]
    st = lib().orc_krylov(n0, n1, n2, _p(K), _p(mu), _p(F), _p(b), _p(x), eta, max_it, METHODS[method], lo, hi,
                          ctypes.byref(it), ctypes.byref(rel))
    return x, st, it.value, rel.value


def solve_increment_krylov(K, mu, F, Fbar, method, lo, hi, eta_nw=1e-5, eta_cg=1e-8, max_newton=50,
                           max_cg=10000, nyq_identity=False):
    """One increment whose linear solves use `method` (GMRES: lo = restart length).
    Returns (status, F_new, P, Pbar, stats)."""
    F = np.array(F, dtype=np.float64, copy=True, order="C")
    grid = F.shape[1:]
    K = _c(np.broadcast_to(K, grid))
    mu = _c(np.broadcast_to(mu, grid))
    Fbar = _c(np.asarray(Fbar, dtype=np.float64).reshape(9))
    P = np.zeros_like(F)
    Pbar = np.zeros(9)
    st = Stats()
    status = lib().orc_solve_increment_krylov_nyq(grid[0], grid[1], grid[2], _p(K), _p(mu), _p(F), _p(Fbar),
                                                  eta_nw, eta_cg, max_newton, max_cg, _p(P), _p(Pbar),
                                                  ctypes.byref(st), METHODS[method], lo, hi,
                                                  1 if nyq_identity else 0)
    return status, F, P, Pbar, st.as_dict()


def identity_field(shape):
    F = np.zeros((9,) + tuple(shape))
    F[0] = F[4] = F[8] = 1.0
    return F


def adjoint(K, mu, F, g, eta_cg=1e-8, max_cg=10000):
    """dL/dmu(x), dL/dK(x) for the cotangent g = dL/dPbar at the converged F.

    Returns (status, dLdmu, dLdK, cg_iterations), fields shaped like the grid."""
    F = _c(F)
    grid = F.shape[1:]
    K = _c(np.broadcast_to(K, grid))
    mu = _c(np.broadcast_to(mu, grid))
    g = _c(np.asarray(g, dtype=np.float64).reshape(9))
    dmu = np.zeros(grid)
    dK = np.zeros(grid)
    it = ctypes.c_int(0)
    st = lib().orc_adjoint(grid[0], grid[1], grid[2], _p(K), _p(mu), _p(F), _p(g), eta_cg, max_cg, _p(dmu),
                           _p(dK), ctypes.byref(it))
    return st, dmu, dK, it.value


def solve_increment(K, mu, F, Fbar, eta_nw=1e-5, eta_cg=1e-8, max_newton=50, max_cg=10000, nyq_identity=False):
    """One increment of Algorithm 1.  Returns (status, F_new, P, Pbar, stats).

    nyq_identity: the projection's Nyquist choice (see project)."""
    F = np.array(F, dtype=np.float64, copy=True, order="C")
    grid = F.shape[1:]
    K = _c(np.broadcast_to(K, grid))
    mu = _c(np.broadcast_to(mu, grid))
    Fbar = _c(np.asarray(Fbar, dtype=np.float64).reshape(9))
    P = np.zeros_like(F)
    Pbar = np.zeros(9)
    st = Stats()
    status = lib().orc_solve_increment_nyq(grid[0], grid[1], grid[2], _p(K), _p(mu), _p(F), _p(Fbar),
                                           eta_nw, eta_cg, max_newton, max_cg, _p(P), _p(Pbar),
                                           ctypes.byref(st), 1 if nyq_identity else 0)
    return status, F, P, Pbar, st.as_dict()


# ---------------------------------------------------------------- mixed control
def _mask(mask):
    m = np.ascontiguousarray(np.asarray(mask).reshape(9) != 0, dtype=np.int32)
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def macro_tangent(K, mu, F, want=None, eta_cg=1e-10, max_cg=10000):
    """C[i, m] = dPbar_i / dFbar_m at the equilibrium F (columns with want[m]).

    Returns (status, C) with C a 9 x 9 array (unrequested columns zero)."""
    F = _c(F)
    grid = F.shape[1:]
    K = _c(np.broadcast_to(K, grid))
    mu = _c(np.broadcast_to(mu, grid))
    w, wp = _mask(np.ones(9) if want is None else want)
    C = np.zeros(81)
    st = lib().orc_macro_tangent(grid[0], grid[1], grid[2], _p(K), _p(mu), _p(F), wp, eta_cg, max_cg, _p(C))
    return st, C.reshape(9, 9)


def solve_increment_mixed(K, mu, F, Fbar, mask, Ptarget, tol_stress=1e-10, max_outer=20, eta_nw=1e-5,
                          eta_cg=1e-8, max_newton=50, max_cg=10000):
    """One increment under mixed control: Pbar_m = Ptarget_m where mask[m], Fbar_m
    elsewhere (Fbar's masked entries: the starting guess).

    Returns (status, F_new, P, Pbar, Fbar_solution, stats, outer_iterations)."""
    F = np.array(F, dtype=np.float64, copy=True, order="C")
    grid = F.shape[1:]
    K = _c(np.broadcast_to(K, grid))
    mu = _c(np.broadcast_to(mu, grid))
    Fb = np.array(np.asarray(Fbar, dtype=np.float64).reshape(9), copy=True)
    Pt = _c(np.asarray(Ptarget, dtype=np.float64).reshape(9))
    m, mp = _mask(mask)
    P = np.zeros_like(F)
    Pbar = np.zeros(9)
    st = Stats()
    outer = ctypes.c_int(0)
    status = lib().orc_solve_increment_mixed(grid[0], grid[1], grid[2], _p(K), _p(mu), _p(F), _p(Fb), mp, _p(Pt),
                                             tol_stress, max_outer, eta_nw, eta_cg, max_newton, max_cg, _p(P),
                                             _p(Pbar), ctypes.byref(st), ctypes.byref(outer))
    return status, F, P, Pbar, Fb, st.as_dict(), outer.value


def solve_increment_mixed_j2(K, mu, ty0, H, hist, F, Fbar, mask, Ptarget, tol_stress=1e-10, max_outer=20,
                             eta_nw=1e-5, eta_cg=1e-8, max_newton=50, max_cg=10000):
    """Mixed control with the J2 law.  Returns (status, F, P, Pbar, Fbar, hist_new, stats, outer)."""
    F = np.array(F, dtype=np.float64, copy=True, order="C")
    grid = F.shape[1:]
    b = lambda a: _c(np.broadcast_to(a, grid))
    K, mu, ty0, H = b(K), b(mu), b(ty0), b(H)
    hist = np.array(hist, dtype=np.float64, copy=True, order="C")
    Fb = np.array(np.asarray(Fbar, dtype=np.float64).reshape(9), copy=True)
    Pt = _c(np.asarray(Ptarget, dtype=np.float64).reshape(9))
    m, mp = _mask(mask)
    P = np.zeros_like(F)
    Pbar = np.zeros(9)
    st = Stats()
    outer = ctypes.c_int(0)
    status = lib().orc_solve_increment_mixed_j2(grid[0], grid[1], grid[2], _p(K), _p(mu), _p(ty0), _p(H),
                                                _p(hist), _p(F), _p(Fb), mp, _p(Pt), tol_stress, max_outer, eta_nw,
                                                eta_cg, max_newton, max_cg, _p(P), _p(Pbar), ctypes.byref(st),
                                                ctypes.byref(outer))
    return status, F, P, Pbar, Fb, hist, st.as_dict(), outer.value


# ---------------------------------------------------------------- J2 plasticity
def virgin_history(shape):
    """C_p^-1 = I (xx yy zz xy yz xz) and eps_p = 0, shape (7, *grid)."""
    h = np.zeros((7,) + tuple(shape))
    h[0] = h[1] = h[2] = 1.0
    return h


def jacobi_eig3(A):
    A = _c(np.asarray(A).reshape(9))
    w = np.zeros(3)
    V = np.zeros(9)
    lib().orc_jacobi_eig3(_p(A), _p(w), _p(V))
    return w, V.reshape(3, 3)


def _j2_fields(F, K, mu, ty0, H):
    F = _c(F)
    grid = F.shape[1:]
    b = lambda a: _c(np.broadcast_to(a, grid))
    return F, b(K), b(mu), b(ty0), b(H), int(np.prod(grid))


def j2_stress(F, K, mu, ty0, H, hist):
    """(status, P, hist_new) of the return mapping at every voxel."""
    F, K, mu, ty0, H, n = _j2_fields(F, K, mu, ty0, H)
    hist = _c(hist)
    P = np.zeros_like(F)
    hn = np.zeros_like(hist)
    st = lib().orc_j2_stress(n, _p(F), _p(K), _p(mu), _p(ty0), _p(H), _p(hist), _p(P), _p(hn))
    return st, P, hn


def j2_tangent(F, K, mu, ty0, H, hist, dF):
    F, K, mu, ty0, H, n = _j2_fields(F, K, mu, ty0, H)
    dF = _c(np.broadcast_to(dF, F.shape))
    out = np.zeros_like(F)
    st = lib().orc_j2_tangent(n, _p(F), _p(K), _p(mu), _p(ty0), _p(H), _c(hist).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), _p(dF), _p(out))
    return st, out


def solve_increment_j2(K, mu, ty0, H, hist, F, Fbar, eta_nw=1e-5, eta_cg=1e-8, max_newton=50, max_cg=10000):
    """One J2 increment.  Returns (status, F_new, P, Pbar, hist_new, stats)."""
    F = np.array(F, dtype=np.float64, copy=True, order="C")
    grid = F.shape[1:]
    b = lambda a: _c(np.broadcast_to(a, grid))
    K, mu, ty0, H = b(K), b(mu), b(ty0), b(H)
    hist = np.array(hist, dtype=np.float64, copy=True, order="C")
    Fbar = _c(np.asarray(Fbar, dtype=np.float64).reshape(9))
    P = np.zeros_like(F)
    Pbar = np.zeros(9)
    st = Stats()
    status = lib().orc_solve_increment_j2(grid[0], grid[1], grid[2], _p(K), _p(mu), _p(ty0), _p(H), _p(hist),
                                          _p(F), _p(Fbar), eta_nw, eta_cg, max_newton, max_cg, _p(P), _p(Pbar),
                                          ctypes.byref(st))
    return status, F, P, Pbar, hist, st.as_dict()
