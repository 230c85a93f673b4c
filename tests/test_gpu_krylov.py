"""Chebyshev and Richardson iterations on the GPU (fftnk_set_krylov) against the
oracle's, through the C-ABI.

* Homogeneous cell at F = I with the exact bounds [mu, lambda + 2 mu]: the
  residual of a linear solve (fftnk_solve_linear) after k iterations equals
  the closed forms ||r0|| / T_k(sigma) (Chebyshev) and
  ||r0|| ((kappa - 1)/(kappa + 1))^k (Richardson), independent of both
  implementations; CG ends after two iterations (two eigenvalues).
* Heterogeneous linear solves: the oracle's iteration count (+-1) and
  solution (1e-9 relative), for CG too.
* Heterogeneous increments with each method: the same Newton and iteration
  counts as the oracle (within +-1 per solve), F within 1e-10 relative (FP64);
  FP32-mixed P-bar within 1e-5; the state matches the CG increment's.
* Bad bounds are rejected.
* GMRES: two iterations on the two-eigenvalue operator; linear solves
  (restart lengths 5, 20, 60) and increments (FP64, FP32-mixed, a batch of two
  cells) with the oracle's GMRES iteration counts (+-1) and solutions; the
  basis must be reserved before the workspace is bound.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms

pytestmark = pytest.mark.gpu

TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(dims, prec, phase, table=TABLE):
    from paper_1603_08893_amd.fftnk import Solver
    s = Solver(dims, precision=prec)
    s.set_phases(phase)
    s.set_material(table)
    return s


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.mark.parametrize("method", ["chebyshev", "richardson", "cg"])
def test_closed_form_residuals(torch_cuda, orc, method):
    torch = torch_cuda
    shape = (9, 8, 10)
    print("krylov closed form", method, flush=True)
    K0, mu0 = ms.K_HARD, ms.MU_HARD
    L = K0 - 2 * mu0 / 3
    lo, hi = mu0, L + 2 * mu0
    s = _solver(shape, "fp64", np.zeros(shape, dtype=np.uint8), table=[(K0, mu0)])
    s.set_krylov(method, lo, hi)
    s.set_linearization(torch.from_numpy(orc.identity_field(shape).reshape(-1)))
    b = torch.from_numpy(ms.random_field(shape, seed=3).reshape(-1))
    sigma = (hi + lo) / (hi - lo)
    q = (hi / lo - 1) / (hi / lo + 1)
    if method == "cg":  # two eigenvalues: two iterations
        st, x, S = s.solve_linear(b, 1e-12, 100)
        assert st == 0 and S[0]["cg_iters"][0] == 2
        return
    for k in (1, 2, 4, 7):
        st, x, S = s.solve_linear(b, 1e-30, k)
        ref = 1.0 / np.cosh(k * np.arccosh(sigma)) if method == "chebyshev" else q ** k
        assert S[0]["cg_iters"][0] == k
        assert abs(S[0]["cg_relres"][0] - ref) <= 1e-9 * ref, k


@pytest.mark.parametrize("method", ["chebyshev", "richardson", "cg"])
@pytest.mark.parametrize("shape", [(9, 7, 8), (16, 16, 16)])
def test_linear_solve_vs_oracle(torch_cuda, orc, method, shape):
    torch = torch_cuda
    print("krylov linear", method, shape, flush=True)
    rng = np.random.default_rng(5)
    ph = (rng.random(shape) < 0.3).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    F = ms.near_identity_field(shape, seed=6, scale=0.01)
    lo = 0.95 * min(m for _, m in TABLE)
    hi = 1.05 * 3 * max(k for k, _ in TABLE)
    braw = ms.random_field(shape, seed=7)
    b = orc.project(braw)
    xo, st, it, rel = orc.krylov(F, K, mu, b, method, lo, hi, 1e-10, 20000)
    assert st == 0
    s = _solver(shape, "fp64", ph)
    s.set_krylov(method, lo, hi)
    s.set_linearization(torch.from_numpy(F.reshape(-1)))
    stg, x, S = s.solve_linear(torch.from_numpy(braw.reshape(-1)), 1e-10, 20000)
    print("oracle", it, "gpu", S[0]["cg_iters"][0], flush=True)
    assert stg == 0 and abs(S[0]["cg_iters"][0] - it) <= 1
    assert _rel(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.parametrize("method", ["chebyshev", "richardson", "cg"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_increment_vs_oracle(torch_cuda, orc, method, prec):
    shape = (12, 10, 14)
    print("krylov increment", method, prec, flush=True)
    rng = np.random.default_rng(4)
    ph = (rng.random(shape) < 0.3).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    lo = 0.9 * min(m for _, m in TABLE)
    hi = 1.1 * 3 * max(k for k, _ in TABLE)
    Fbar = ms.simple_shear(0.05)
    st, Fo, Po, Pbo, So = orc.solve_increment_krylov(K, mu, orc.identity_field(shape), Fbar, method, lo, hi, 1e-8,
                                                     1e-10)
    assert st == 0
    s = _solver(shape, prec, ph)
    s.set_krylov(method, lo, hi)
    stg, F, P, Pb, S = s.solve_increment(Fbar, 1e-8, 1e-10)
    print("oracle", So["cg_iters"], "gpu", S[0]["cg_iters"], flush=True)
    if prec == "fp64":
        assert S[0]["n_solves"] == So["n_solves"]
        assert all(abs(a - b) <= 1 for a, b in zip(S[0]["cg_iters"], So["cg_iters"]))
        assert _rel(F.cpu().numpy(), Fo) <= 1e-10
        assert np.max(np.abs(Pb[0] - Pbo)) <= 1e-10 * np.max(np.abs(Pbo))
    else:
        assert np.max(np.abs(Pb[0] - Pbo)) <= 1e-5 * np.max(np.abs(Pbo))
    # the same state as the CG increment
    s.reset_state()
    s.set_krylov("cg")
    _, Fc, _, Pbc, _ = s.solve_increment(Fbar, 1e-8, 1e-10)
    assert np.max(np.abs(Pb[0] - Pbc[0])) <= (1e-9 if prec == "fp64" else 1e-5) * np.max(np.abs(Pbc[0]))


def test_bad_bounds_rejected(torch_cuda):
    from paper_1603_08893_amd import fftnk
    s = _solver((4, 4, 4), "fp64", np.zeros((4, 4, 4), dtype=np.uint8))
    for m, lo, hi in (("chebyshev", 0.0, 1.0), ("chebyshev", 2.0, 1.0), ("richardson", -1.0, 1.0),
                      ("chebyshev", 1.0, float("inf"))):
        with pytest.raises(fftnk.FftnkError):
            s.set_krylov(m, lo, hi)


# ---------------------------------------------------------------- GMRES
def _gm_solver(dims, prec, phase, m, table=TABLE):
    from paper_1603_08893_amd.fftnk import Solver
    s = Solver(dims, precision=prec, gmres_restart=m)
    s.set_phases(phase)
    s.set_material(table)
    s.set_krylov("gmres")
    return s


def test_gmres_two_eigenvalues(torch_cuda, orc):
    torch = torch_cuda
    shape = (9, 8, 10)
    print("gmres closed form", flush=True)
    K0, mu0 = ms.K_HARD, ms.MU_HARD
    s = _gm_solver(shape, "fp64", np.zeros(shape, dtype=np.uint8), 30, table=[(K0, mu0)])
    s.set_linearization(torch.from_numpy(orc.identity_field(shape).reshape(-1)))
    st, x, S = s.solve_linear(torch.from_numpy(ms.random_field(shape, seed=3).reshape(-1)), 1e-12, 100)
    assert st == 0 and S[0]["cg_iters"][0] == 2 and S[0]["cg_relres"][0] < 1e-12


@pytest.mark.parametrize("m", [5, 20, 60])
@pytest.mark.parametrize("shape", [(9, 7, 8), (16, 16, 16)])
def test_gmres_linear_solve_vs_oracle(torch_cuda, orc, m, shape):
    torch = torch_cuda
    print("gmres linear", m, shape, flush=True)
    rng = np.random.default_rng(5)
    ph = (rng.random(shape) < 0.3).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    F = ms.near_identity_field(shape, seed=6, scale=0.01)
    braw = ms.random_field(shape, seed=7)
    xo, st, it, rel = orc.krylov(F, K, mu, orc.project(braw), "gmres", m, 0, 1e-10, 20000)
    assert st == 0
    s = _gm_solver(shape, "fp64", ph, m)
    s.set_linearization(torch.from_numpy(F.reshape(-1)))
    stg, x, S = s.solve_linear(torch.from_numpy(braw.reshape(-1)), 1e-10, 20000)
    print("oracle", it, "gpu", S[0]["cg_iters"][0], flush=True)
    assert stg == 0 and abs(S[0]["cg_iters"][0] - it) <= 1
    assert _rel(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gmres_increment_vs_oracle(torch_cuda, orc, prec):
    shape = (12, 10, 14)
    print("gmres increment", prec, flush=True)
    rng = np.random.default_rng(4)
    ph = (rng.random(shape) < 0.3).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    Fbar = ms.simple_shear(0.05)
    st, Fo, Po, Pbo, So = orc.solve_increment_krylov(K, mu, orc.identity_field(shape), Fbar, "gmres", 20, 0, 1e-8,
                                                     1e-10)
    assert st == 0
    s = _gm_solver(shape, prec, ph, 20)
    stg, F, P, Pb, S = s.solve_increment(Fbar, 1e-8, 1e-10)
    print("oracle", So["cg_iters"], "gpu", S[0]["cg_iters"], flush=True)
    if prec == "fp64":
        assert S[0]["n_solves"] == So["n_solves"]
        assert all(abs(a - b) <= 1 for a, b in zip(S[0]["cg_iters"], So["cg_iters"]))
        assert _rel(F.cpu().numpy(), Fo) <= 1e-10
        assert np.max(np.abs(Pb[0] - Pbo)) <= 1e-10 * np.max(np.abs(Pbo))
    else:
        assert np.max(np.abs(Pb[0] - Pbo)) <= 1e-5 * np.max(np.abs(Pbo))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gmres_batched_matches_single(torch_cuda, orc, prec):
    """Three cells whose 9 n values start at even, odd and odd offsets and
    have odd, even and odd lengths: the element-pair kernels' lone first and
    last elements on every combination."""
    from paper_1603_08893_amd.fftnk import Solver
    dims = [(9, 9, 9), (8, 10, 6), (7, 5, 3)]
    print("gmres batched", dims, prec, flush=True)
    phs = [(np.random.default_rng(11 + r).random(d) < 0.3).astype(np.uint8) for r, d in enumerate(dims)]
    Fbars = [ms.simple_shear(0.04), ms.isochoric_stretch(1.03), ms.simple_shear(0.02)]
    s = Solver(dims, precision=prec, gmres_restart=15)
    s.set_phases(np.concatenate([(ph.reshape(-1) + 2 * r).astype(np.uint8) for r, ph in enumerate(phs)]))
    s.set_material(TABLE * 3)
    s.set_krylov("gmres")
    st, F, P, Pb, S = s.solve_increment(np.stack(Fbars), 1e-8, 1e-10)
    assert st == 0
    for r, (d, ph, Fb) in enumerate(zip(dims, phs, Fbars)):
        K, mu = ms.phase_moduli(ph, TABLE)
        sto, Fo, Po, Pbo, So = orc.solve_increment_krylov(K, mu, orc.identity_field(d), Fb, "gmres", 15, 0, 1e-8,
                                                          1e-10)
        assert sto == 0
        if prec == "fp64":
            assert S[r]["n_solves"] == So["n_solves"]
            assert all(abs(a - b) <= 1 for a, b in zip(S[r]["cg_iters"], So["cg_iters"]))
            assert np.max(np.abs(Pb[r] - Pbo)) <= 1e-10 * np.max(np.abs(Pbo))
        else:
            assert np.max(np.abs(Pb[r] - Pbo)) <= 1e-5 * np.max(np.abs(Pbo))


def test_gmres_option_order(torch_cuda):
    from paper_1603_08893_amd import fftnk
    s = _solver((4, 4, 4), "fp64", np.zeros((4, 4, 4), dtype=np.uint8))
    with pytest.raises(fftnk.FftnkError):
        s.set_krylov("gmres")  # no basis reserved
    with pytest.raises(fftnk.FftnkError):
        s.set_option(fftnk.OPT_GMRES_RESTART, 10)  # after the workspace was bound
