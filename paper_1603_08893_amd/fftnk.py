"""Thin ctypes binding of libfftnk (include/fftnk.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of
the library.  PyTorch supplies device memory (the workspace and all fields are
torch tensors on ``cuda``) and the stream.  Importing works without a GPU; any
call that needs the library raises ``FftnkError`` if it has not been built
(``python -m paper_1603_08893_amd.build``) -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libfftnk.so")

OK, EINVAL, ESTATE, ENOMEM, EHIP, ECG_MAXIT, ECG_BREAKDOWN, ENEWTON_MAXIT, ENONFINITE, EMATERIAL, EUNSUPPORTED = range(11)
FP64, FP32_MIXED = 0, 1
SVK, J2 = 0, 1
OPT_GRAPHS, OPT_CHECK_EVERY, OPT_NYQUIST, OPT_GMRES_RESTART, OPT_J2_TANGENT, OPT_X_WINDOW = 1, 2, 3, 4, 5, 6
KRYLOV = {"cg": 0, "chebyshev": 1, "richardson": 2, "gmres": 3}
MAX_SOLVES = 64

# every symbol include/fftnk.h declares
EXPORTS = [
    "fftnk_create", "fftnk_create_batched", "fftnk_workspace_bytes", "fftnk_bind_workspace", "fftnk_set_phases",
    "fftnk_set_material", "fftnk_set_modulus_field", "fftnk_set_option", "fftnk_reset_state", "fftnk_solve_increment",
    "fftnk_solve_increment_mixed", "fftnk_macro_tangent", "fftnk_set_krylov",
    "fftnk_solve_linear", "fftnk_describe", "fftnk_set_plan", "fftnk_autotune",
    "fftnk_set_linearization", "fftnk_apply_operator", "fftnk_project", "fftnk_constitutive", "fftnk_adjoint",
    "fftnk_launch_pass", "fftnk_profile_cg", "fftnk_get_history", "fftnk_set_history", "fftnk_get_state",
    "fftnk_set_state", "fftnk_status_string", "fftnk_destroy", "fftnk_stream",
    "fftnk_project_noalloc",
]


class FftnkError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, status_string(status), status))


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("n_solves", ctypes.c_int),
        ("cg_iters", ctypes.c_int * MAX_SOLVES),
        ("newton_res", ctypes.c_double * MAX_SOLVES),
        ("cg_relres", ctypes.c_double * MAX_SOLVES),
        ("t_ms", ctypes.c_double),
    ]

    def as_dict(self):
        k = self.n_solves
        return {"status": self.status, "n_solves": k, "cg_iters": list(self.cg_iters[:k]),
                "newton_res": list(self.newton_res[:k]), "cg_relres": list(self.cg_relres[:k]), "t_ms": self.t_ms}


_lib = None


def lib():
    """Load libfftnk.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise FftnkError(EHIP, "libfftnk.so not built (run python -m paper_1603_08893_amd.build)")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    L.fftnk_create.argtypes = [ctypes.POINTER(vp), i, i, i, i, vp]
    L.fftnk_create_batched.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(i), i, vp]
    L.fftnk_workspace_bytes.argtypes = [vp]
    L.fftnk_workspace_bytes.restype = sz
    L.fftnk_bind_workspace.argtypes = [vp, vp, sz]
    L.fftnk_set_phases.argtypes = [vp, vp]
    L.fftnk_set_material.argtypes = [vp, i, i, dp]
    L.fftnk_set_modulus_field.argtypes = [vp, vp]
    L.fftnk_set_option.argtypes = [vp, i, i]
    L.fftnk_reset_state.argtypes = [vp]
    L.fftnk_set_krylov.argtypes = [vp, i, d, d]
    L.fftnk_solve_linear.argtypes = [vp, vp, vp, d, i, ctypes.POINTER(Stats)]
    L.fftnk_describe.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
    L.fftnk_set_plan.argtypes = [vp, ctypes.c_uint]
    L.fftnk_autotune.argtypes = [vp, i, i, ctypes.POINTER(ctypes.c_uint), ctypes.POINTER(d)]
    L.fftnk_solve_increment.argtypes = [vp, dp, d, d, i, i, vp, vp, dp, ctypes.POINTER(Stats)]
    ip = ctypes.POINTER(i)
    L.fftnk_solve_increment_mixed.argtypes = [vp, dp, ip, dp, d, i, d, d, i, i, vp, vp, dp, ctypes.POINTER(Stats), ip]
    L.fftnk_macro_tangent.argtypes = [vp, ip, d, i, dp, ctypes.POINTER(Stats)]
    L.fftnk_set_linearization.argtypes = [vp, vp]
    L.fftnk_apply_operator.argtypes = [vp, vp, vp]
    L.fftnk_project.argtypes = [vp, vp, vp]
    L.fftnk_constitutive.argtypes = [vp, vp, vp, dp]
    L.fftnk_adjoint.argtypes = [vp, dp, d, i, vp, vp, ctypes.POINTER(Stats)]
    L.fftnk_launch_pass.argtypes = [vp, i]
    L.fftnk_profile_cg.argtypes = [vp, i, vp]
    L.fftnk_get_history.argtypes = [vp, vp]
    L.fftnk_set_history.argtypes = [vp, vp]
    L.fftnk_get_state.argtypes = [vp, vp]
    L.fftnk_set_state.argtypes = [vp, vp]
    L.fftnk_status_string.argtypes = [i]
    L.fftnk_status_string.restype = ctypes.c_char_p
    L.fftnk_destroy.argtypes = [vp]
    L.fftnk_destroy.restype = None
    L.fftnk_stream.argtypes = [i, i, vp, vp, vp, sz, i, vp, dp]
    L.fftnk_project_noalloc.argtypes = [i, i, i, i, vp, vp, vp]
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def status_string(s):
    try:
        return lib().fftnk_status_string(int(s)).decode()
    except FftnkError:
        return "status %d" % s


def describe(dims, precision="fp64", gmres_restart=0, policy=0):
    """The launch geometry the library plans for a cell (or a batch of cells)
    under a plan policy (fftnk_set_plan), as a dict; needs no GPU (a context is
    created and described, never bound)."""
    import json
    L = lib()
    if isinstance(dims[0], (int, np.integer)):
        dims = [dims]
    arr = (ctypes.c_int * (3 * len(dims)))(*[int(v) for d in dims for v in d])
    ctx = ctypes.c_void_p()
    _check(L.fftnk_create_batched(ctypes.byref(ctx), len(dims), arr, FP64 if precision == "fp64" else FP32_MIXED,
                                  None), "fftnk_create_batched")
    try:
        if gmres_restart:
            _check(L.fftnk_set_option(ctx, OPT_GMRES_RESTART, int(gmres_restart)), "fftnk_set_option")
        if policy:
            _check(L.fftnk_set_plan(ctx, int(policy)), "fftnk_set_plan")
        return _describe_ctx(ctx)
    finally:
        L.fftnk_destroy(ctx)


def _describe_ctx(ctx):
    import json
    L = lib()
    need = ctypes.c_size_t(0)
    L.fftnk_describe(ctx, None, 0, ctypes.byref(need))
    buf = ctypes.create_string_buffer(need.value)
    _check(L.fftnk_describe(ctx, buf, need.value, None), "fftnk_describe")
    return json.loads(buf.value.decode())


def project_noalloc(a, dims, out=None, stream=None):
    """G(a) through fftnk_project_noalloc (no context, no allocation inside the
    library): a, out torch CUDA tensors of 9 n0 n1 n2 doubles or floats."""
    import torch
    prec = FP64 if a.dtype == torch.float64 else FP32_MIXED
    out = torch.empty_like(a) if out is None else out
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    _check(lib().fftnk_project_noalloc(int(dims[0]), int(dims[1]), int(dims[2]), prec, ctypes.c_void_p(a.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream)),
           "fftnk_project_noalloc")
    return out


STREAM_KINDS = {"read": 0, "write": 1, "copy": 2, "triad": 3}
STREAM_MOVES = {"read": 1, "write": 1, "copy": 2, "triad": 3}  # arrays of `bytes` moved per launch


def stream(kind, lane_bytes, dst, src1=None, src2=None, reps=20, stream=None, nontemporal=False):
    """Mean ms per launch of a streaming kernel (fftnk_stream) over torch CUDA
    buffers of equal size; returns (ms, GB/s)."""
    import torch
    nbytes = dst.numel() * dst.element_size()
    st = stream if stream is not None else torch.cuda.current_stream(dst.device)
    ms = ctypes.c_double(0.0)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    _check(lib().fftnk_stream(STREAM_KINDS[kind] | (16 if nontemporal else 0), int(lane_bytes), ptr(dst), ptr(src1), ptr(src2), nbytes, int(reps),
                              ctypes.c_void_p(st.cuda_stream), ctypes.byref(ms)), "fftnk_stream")
    return ms.value, STREAM_MOVES[kind] * nbytes / (ms.value * 1e-3) / 1e9


def _check(status, what):
    if status != OK:
        raise FftnkError(status, what)


def _dptr(a):
    return ctypes.cast(ctypes.c_void_p(a.ctypes.data), ctypes.POINTER(ctypes.c_double))


class Solver:
    """One fftnk context: a periodic cell (or a batch of cells) on one GPU.

    dims: (n0, n1, n2) or a list of them (batched).  precision: "fp64" or
    "fp32" (FP32 Krylov solve, FP64 Newton residual).  gmres_restart: reserve
    the basis of restarted GMRES with this restart length (0: none).
    j2_stored_tangent: reserve and use the compact J2 tangent stored per
    linearisation point (FFTNK_OPT_J2_TANGENT; J2 law, FP64).  x_window: CG
    directions kept for the windowed update of the iterate (FFTNK_OPT_X_WINDOW,
    1..8; None: the library's default).
    """

    def __init__(self, dims, precision="fp64", device="cuda", stream=None, gmres_restart=0,
                 j2_stored_tangent=False, x_window=None):
        import torch
        self.torch = torch
        if isinstance(dims[0], (int, np.integer)):
            dims = [tuple(int(v) for v in dims)]
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.nrve = len(self.dims)
        self.n = [d[0] * d[1] * d[2] for d in self.dims]
        self.ntot = sum(self.n)
        self.precision = precision
        self.prec = FP64 if precision == "fp64" else FP32_MIXED
        self.vdtype = torch.float64 if self.prec == FP64 else torch.float32
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lib()
        ctx = ctypes.c_void_p()
        arr = (ctypes.c_int * (3 * self.nrve))(*[v for d in self.dims for v in d])
        _check(L.fftnk_create_batched(ctypes.byref(ctx), self.nrve, arr, self.prec,
                                      ctypes.c_void_p(self.stream.cuda_stream)), "fftnk_create_batched")
        self.ctx = ctx
        if gmres_restart:
            _check(L.fftnk_set_option(ctx, OPT_GMRES_RESTART, int(gmres_restart)), "fftnk_set_option")
        if j2_stored_tangent:
            _check(L.fftnk_set_option(ctx, OPT_J2_TANGENT, 1), "fftnk_set_option")
        if x_window is not None:
            _check(L.fftnk_set_option(ctx, OPT_X_WINDOW, int(x_window)), "fftnk_set_option")
        self.x_window = int(_describe_ctx(ctx)["x_window"])
        nbytes = L.fftnk_workspace_bytes(ctx)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        _check(L.fftnk_bind_workspace(ctx, ctypes.c_void_p(aligned), nbytes), "fftnk_bind_workspace")
        self.workspace_bytes = nbytes
        # bumped by every call that changes the committed state, the phases or
        # the moduli (what fftnk_adjoint differentiates at)
        self.generation = 0

    def __del__(self):
        if getattr(self, "ctx", None) is not None and _lib is not None:
            _lib.fftnk_destroy(self.ctx)
            self.ctx = None

    # ------------------------------------------------------------ set-up
    def field(self, dtype=None):
        return self.torch.empty(9 * self.ntot, dtype=dtype or self.vdtype, device=self.device)

    def set_phases(self, phase):
        self.generation += 1
        ph = np.ascontiguousarray(phase, dtype=np.uint8).reshape(-1)
        if ph.size != self.ntot:
            raise FftnkError(EINVAL, "set_phases: %d values for %d voxels" % (ph.size, self.ntot))
        self._max_phase = int(ph.max())
        if getattr(self, "_nphase", None) is not None and self._max_phase >= self._nphase:
            raise FftnkError(EINVAL, "set_phases: phase index beyond the material table")
        t = self.torch.as_tensor(ph).to(self.device)
        self._phase = t
        _check(lib().fftnk_set_phases(self.ctx, ctypes.c_void_p(t.data_ptr())), "fftnk_set_phases")

    def set_material(self, table, model=SVK):
        self.generation += 1
        tab = np.ascontiguousarray(table, dtype=np.float64)
        if getattr(self, "_max_phase", None) is not None and self._max_phase >= tab.shape[0]:
            raise FftnkError(EINVAL, "set_material: fewer phases than the phase map uses")
        self._nphase = tab.shape[0]
        _check(lib().fftnk_set_material(self.ctx, model, tab.shape[0], _dptr(tab)), "fftnk_set_material")

    def set_modulus_field(self, mu):
        self.generation += 1
        if mu is None:
            _check(lib().fftnk_set_modulus_field(self.ctx, None), "fftnk_set_modulus_field")
            return
        if isinstance(mu, self.torch.Tensor):
            t = mu.detach().reshape(-1).to(self.device, self.torch.float64).contiguous()
        else:
            t = self.torch.as_tensor(np.ascontiguousarray(mu, dtype=np.float64).reshape(-1)).to(self.device)
        if t.numel() != self.ntot:
            raise FftnkError(EINVAL, "set_modulus_field: %d values for %d voxels" % (t.numel(), self.ntot))
        _check(lib().fftnk_set_modulus_field(self.ctx, ctypes.c_void_p(t.data_ptr())), "fftnk_set_modulus_field")

    def set_option(self, option, value):
        """OPT_GRAPHS (replay CG iterations from HIP graphs), OPT_CHECK_EVERY, or
        OPT_NYQUIST (0: G-hat zero at Nyquist frequencies, 1: identity there)."""
        _check(lib().fftnk_set_option(self.ctx, int(option), int(value)), "fftnk_set_option")

    def set_plan(self, policy):
        """FFT plan policy (engines and tile sizes; see fftnk_set_plan)."""
        _check(lib().fftnk_set_plan(self.ctx, int(policy)), "fftnk_set_plan")

    def autotune(self, reps=5, use_cache=True):
        """Time the operator under every distinct plan policy and keep the
        fastest; returns (policy, ms per application), ms = -1 when the choice
        came from this process's cache."""
        pol = ctypes.c_uint(0)
        ms = ctypes.c_double(0.0)
        _check(lib().fftnk_autotune(self.ctx, int(reps), 1 if use_cache else 0, ctypes.byref(pol), ctypes.byref(ms)),
               "fftnk_autotune")
        return int(pol.value), float(ms.value)

    def set_krylov(self, method="cg", lo=None, hi=None, table=None):
        """Krylov method of later linear solves: "cg", "chebyshev", "richardson"
        or "gmres" (needs gmres_restart at construction).  Chebyshev and
        Richardson need spectral bounds [lo, hi] of A on range(G); if omitted
        they are taken from a St. Venant-Kirchhoff table [(K, mu), ...] as
        [0.9 min mu, 1.1 max 3K] (near F = I)."""
        if method in ("chebyshev", "richardson") and (lo is None or hi is None):
            tab = np.asarray(table, dtype=np.float64)
            lo = 0.9 * float(tab[:, 1].min()) if lo is None else lo
            hi = 1.1 * 3.0 * float(tab[:, 0].max()) if hi is None else hi
        _check(lib().fftnk_set_krylov(self.ctx, KRYLOV[method], float(lo or 0.0), float(hi or 0.0)),
               "fftnk_set_krylov")

    def reset_state(self):
        self.generation += 1
        _check(lib().fftnk_reset_state(self.ctx), "fftnk_reset_state")

    # ------------------------------------------------------------ solve
    def solve_increment(self, Fbar, eta_nw=1e-5, eta_cg=1e-8, max_newton=50, max_cg=10000, fields=True,
                        raise_on_error=True):
        """One load increment.  Returns (status, F, P, Pbar[nrve, 9], stats list)."""
        self.generation += 1
        Fb = np.ascontiguousarray(np.asarray(Fbar, dtype=np.float64).reshape(self.nrve, 9))
        Pbar = np.zeros((self.nrve, 9))
        stats = (Stats * self.nrve)()
        F = self.field(self.torch.float64) if fields else None
        P = self.field(self.torch.float64) if fields else None
        st = lib().fftnk_solve_increment(self.ctx, _dptr(Fb), eta_nw, eta_cg, max_newton, max_cg,
                                         ctypes.c_void_p(F.data_ptr()) if fields else None,
                                         ctypes.c_void_p(P.data_ptr()) if fields else None,
                                         _dptr(Pbar), stats)
        if raise_on_error:
            _check(st, "fftnk_solve_increment")
        return st, F, P, Pbar, [s.as_dict() for s in stats]

    def solve_increment_mixed(self, Fbar, mask, Ptarget, tol_stress=1e-10, max_outer=20, eta_nw=1e-5, eta_cg=1e-8,
                              max_newton=50, max_cg=10000, fields=True, raise_on_error=True):
        """One increment under mixed control: Pbar_k = Ptarget_k where mask_k != 0,
        Fbar_k elsewhere (Fbar's masked entries: the starting guess).  mask,
        Ptarget, Fbar: [9] or [nrve, 9].

        Returns (status, F, P, Pbar[nrve, 9], Fbar[nrve, 9], stats list, outer[nrve])."""
        self.generation += 1
        Fb = np.array(np.broadcast_to(np.asarray(Fbar, dtype=np.float64).reshape(-1, 9), (self.nrve, 9)),
                      dtype=np.float64, order="C")
        Pt = np.ascontiguousarray(np.broadcast_to(np.asarray(Ptarget, dtype=np.float64).reshape(-1, 9),
                                                  (self.nrve, 9)))
        mk = np.ascontiguousarray(np.broadcast_to(np.asarray(mask).reshape(-1, 9) != 0, (self.nrve, 9)),
                                  dtype=np.int32)
        Pbar = np.zeros((self.nrve, 9))
        stats = (Stats * self.nrve)()
        outer = np.zeros(self.nrve, dtype=np.int32)
        F = self.field(self.torch.float64) if fields else None
        P = self.field(self.torch.float64) if fields else None
        ip = ctypes.POINTER(ctypes.c_int)
        st = lib().fftnk_solve_increment_mixed(self.ctx, _dptr(Fb), mk.ctypes.data_as(ip), _dptr(Pt), tol_stress,
                                               max_outer, eta_nw, eta_cg, max_newton, max_cg,
                                               ctypes.c_void_p(F.data_ptr()) if fields else None,
                                               ctypes.c_void_p(P.data_ptr()) if fields else None,
                                               _dptr(Pbar), stats, outer.ctypes.data_as(ip))
        if raise_on_error:
            _check(st, "fftnk_solve_increment_mixed")
        return st, F, P, Pbar, Fb, [s.as_dict() for s in stats], outer

    def macro_tangent(self, want=None, eta_cg=1e-10, max_cg=10000):
        """dPbar/dFbar at the committed state: array [nrve, 9, 9] (columns with want)."""
        C = np.zeros((self.nrve, 9, 9))
        stats = (Stats * self.nrve)()
        ip = ctypes.POINTER(ctypes.c_int)
        if want is None:
            wp = None
        else:
            w = np.ascontiguousarray(np.broadcast_to(np.asarray(want).reshape(-1, 9) != 0, (self.nrve, 9)),
                                     dtype=np.int32)
            wp = w.ctypes.data_as(ip)
        _check(lib().fftnk_macro_tangent(self.ctx, wp, eta_cg, max_cg, _dptr(C), stats), "fftnk_macro_tangent")
        return C

    def set_linearization(self, F):
        F = F.to(self.device, self.torch.float64).contiguous()
        _check(lib().fftnk_set_linearization(self.ctx, ctypes.c_void_p(F.data_ptr())), "fftnk_set_linearization")

    def apply_operator(self, p, out=None):
        p = p.to(self.device, self.vdtype).contiguous()
        out = self.field() if out is None else out
        _check(lib().fftnk_apply_operator(self.ctx, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(out.data_ptr())),
               "fftnk_apply_operator")
        return out

    def solve_linear(self, b, eta=1e-8, max_it=10000, raise_on_error=True):
        """x with A x = G(b) at the linearisation point (FP64 in and out).
        Returns (status, x, stats list)."""
        b = b.to(self.device, self.torch.float64).contiguous()
        x = self.field(self.torch.float64)
        stats = (Stats * self.nrve)()
        st = lib().fftnk_solve_linear(self.ctx, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), eta,
                                      max_it, stats)
        if raise_on_error and st not in (OK, ECG_MAXIT):
            _check(st, "fftnk_solve_linear")
        return st, x, [s.as_dict() for s in stats]

    def project(self, a, out=None):
        a = a.to(self.device, self.vdtype).contiguous()
        out = self.field() if out is None else out
        _check(lib().fftnk_project(self.ctx, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(out.data_ptr())),
               "fftnk_project")
        return out

    def constitutive(self, F):
        F = F.to(self.device, self.torch.float64).contiguous()
        P = self.field(self.torch.float64)
        Pbar = np.zeros((self.nrve, 9))
        _check(lib().fftnk_constitutive(self.ctx, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(P.data_ptr()),
                                        _dptr(Pbar)), "fftnk_constitutive")
        return P, Pbar

    def adjoint(self, gbar, eta_cg=1e-8, max_cg=10000, want_K=False):
        """dL/dmu (and dL/dK) per voxel, [ntot] device doubles, for cotangents gbar [nrve, 9]."""
        g = np.ascontiguousarray(np.asarray(gbar, dtype=np.float64).reshape(self.nrve, 9))
        dmu = self.torch.empty(self.ntot, dtype=self.torch.float64, device=self.device)
        dK = self.torch.empty(self.ntot, dtype=self.torch.float64, device=self.device) if want_K else None
        stats = (Stats * self.nrve)()
        _check(lib().fftnk_adjoint(self.ctx, _dptr(g), eta_cg, max_cg, ctypes.c_void_p(dmu.data_ptr()),
                                   ctypes.c_void_p(dK.data_ptr()) if want_K else None, stats), "fftnk_adjoint")
        return dmu, dK, [s.as_dict() for s in stats]

    def launch_pass(self, k):
        """Enqueue pass k (1..5) of the operator alone (timing instrumentation)."""
        _check(lib().fftnk_launch_pass(self.ctx, int(k)), "fftnk_launch_pass")

    CG_KERNELS = ("pass1", "alpha", "pass2", "pass3", "pass4", "pass5", "beta")

    def profile_cg(self, iters=20, detail=False):
        """Mean ms per launch of each kernel of a CG iteration at the current iterate
        (timing instrumentation; call after a solve, clobbers the Krylov vectors).
        pass1 is its mean over a window of x_window iterations (one of which
        applies the window's x updates); detail=True also returns both times."""
        ms = np.zeros(8, dtype=np.float64)
        _check(lib().fftnk_profile_cg(self.ctx, int(iters), ms.ctypes.data), "fftnk_profile_cg")
        W = self.x_window
        k = dict(zip(self.CG_KERNELS, ms[:7].tolist()))
        if W > 1:
            k["pass1"] = ((W - 1) * ms[0] + ms[7]) / W
        if detail:
            return k, {"x_window": W, "pass1_within_window": float(ms[0]), "pass1_xupdate": float(ms[7])}
        return k

    def get_history(self):
        """J2 history, [7 * ntot] device doubles (C_p^-1 xx yy zz xy yz xz, eps_p)."""
        h = self.torch.empty(7 * self.ntot, dtype=self.torch.float64, device=self.device)
        _check(lib().fftnk_get_history(self.ctx, ctypes.c_void_p(h.data_ptr())), "fftnk_get_history")
        return h

    def set_history(self, h):
        self.generation += 1
        h = h.to(self.device, self.torch.float64).contiguous()
        _check(lib().fftnk_set_history(self.ctx, ctypes.c_void_p(h.data_ptr())), "fftnk_set_history")

    def get_state(self):
        F = self.field(self.torch.float64)
        _check(lib().fftnk_get_state(self.ctx, ctypes.c_void_p(F.data_ptr())), "fftnk_get_state")
        return F

    def set_state(self, F):
        self.generation += 1
        F = F.to(self.device, self.torch.float64).contiguous()
        _check(lib().fftnk_set_state(self.ctx, ctypes.c_void_p(F.data_ptr())), "fftnk_set_state")


def _autograd_function():
    import torch

    class HomogenizedStress(torch.autograd.Function):
        """P-bar of one load increment from the stress-free state, for each load
        case, as a differentiable function of the per-voxel shear modulus.

        forward(mu [N0, N1, N2] float64 cuda, solver, Fbars [nrve, 9]) -> Pbar [nrve, 9]
        The solver's RVEs share the modulus field (one load case per RVE, same
        grid).  backward runs fftnk_adjoint (one CG per load case at the
        converged states) and sums the per-case gradients; it raises if the
        solver's state changed after this forward (Solver.generation).
        """

        @staticmethod
        def forward(ctx, mu, solver, Fbars, eta_nw=1e-5, eta_cg=1e-8):
            m = mu.detach().reshape(-1).to(solver.device, torch.float64)
            solver.set_modulus_field(m.repeat(solver.nrve))
            solver.reset_state()
            _, _, _, Pbar, stats = solver.solve_increment(Fbars, eta_nw, eta_cg, fields=False)
            ctx.solver = solver
            ctx.generation = solver.generation
            ctx.eta_cg = eta_cg
            ctx.shape = mu.shape
            ctx.forward_stats = stats
            return torch.from_numpy(Pbar).to(mu.device)

        @staticmethod
        def backward(ctx, grad_Pbar):
            s = ctx.solver
            if s.generation != ctx.generation:
                raise RuntimeError("HomogenizedStress.backward: the solver's state changed after this forward "
                                   "(another solve, reset or set_* call); the adjoint would be taken at the "
                                   "wrong equilibrium -- run forward again before backward")
            dmu, _, _ = s.adjoint(grad_Pbar.detach().cpu().numpy(), eta_cg=ctx.eta_cg)
            g = dmu.view(s.nrve, -1).sum(dim=0).reshape(ctx.shape)
            return g, None, None, None, None

    return HomogenizedStress


_HS = None


def homogenized_stress(mu, solver, Fbars, eta_nw=1e-5, eta_cg=1e-8):
    """Differentiable P-bar [nrve, 9] (see HomogenizedStress)."""
    global _HS
    if _HS is None:
        _HS = _autograd_function()
    return _HS.apply(mu, solver, Fbars, eta_nw, eta_cg)
