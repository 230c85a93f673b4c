"""Pins of the oracle's other Krylov methods on the same operator: Chebyshev and
Richardson iterations (fixed coefficients from spectral bounds [lo, hi] of A
on range(G)) and restarted GMRES, next to CG.

What fixes the answer independently of the oracle's arithmetic:
* a homogeneous cell linearised at F = I (S = 0): on range(G) the operator has
  exactly two eigenvalues, mu for transverse and lambda + 2 mu for longitudinal
  compatible modes (the acoustic tensor of linear elasticity); with [lo, hi] =
  [mu, lambda + 2 mu] the Chebyshev residual is exactly ||r0|| / T_k(sigma),
  sigma = (hi + lo)/(hi - lo), the Richardson residual exactly
  ||r0|| ((kappa - 1)/(kappa + 1))^k, and CG ends after two iterations;
* a heterogeneous cell near F = I with bounds from the moduli (periodic Korn:
  <p, K p> >= mu_min ||p||^2 on gradients at F = I; Rayleigh: <= 3 K_max ||p||^2):
  the residual bounds ||r_k|| <= ||r0|| / T_k(sigma) and ((kappa-1)/(kappa+1))^k
  hold at every k (A symmetric on range(G)), and all three methods reach the
  same solution, checked with the operator itself;
* a full increment solved with Chebyshev reaches the CG increment's state;
* GMRES: see the pins at the end of the file.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms

TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]


def _cheb_bound(k, lo, hi):
    return 1.0 / np.cosh(k * np.arccosh((hi + lo) / (hi - lo)))


def _homogeneous(orc, shape):
    K0, mu0 = ms.K_HARD, ms.MU_HARD
    L = K0 - 2 * mu0 / 3
    b = orc.project(ms.random_field(shape, seed=3))
    return K0, mu0, mu0, L + 2 * mu0, b


@pytest.mark.parametrize("shape", [(7, 9, 5), (6, 8, 4)])
def test_chebyshev_residual_closed_form(orc, shape):
    K0, mu0, lo, hi, b = _homogeneous(orc, shape)
    I = orc.identity_field(shape)
    for k in range(1, 9):
        x, st, it, rel = orc.krylov(I, K0, mu0, b, "chebyshev", lo, hi, 1e-30, k)
        assert st == 1 and it == k
        assert abs(rel - _cheb_bound(k, lo, hi)) <= 1e-10 * _cheb_bound(k, lo, hi), k


@pytest.mark.parametrize("shape", [(7, 9, 5), (6, 8, 4)])
def test_richardson_residual_closed_form(orc, shape):
    K0, mu0, lo, hi, b = _homogeneous(orc, shape)
    I = orc.identity_field(shape)
    q = (hi / lo - 1) / (hi / lo + 1)
    for k in range(1, 7):
        x, st, it, rel = orc.krylov(I, K0, mu0, b, "richardson", lo, hi, 1e-30, k)
        assert st == 1 and abs(rel - q ** k) <= 1e-10 * q ** k, k


def test_cg_two_eigenvalues_two_iterations(orc):
    shape = (7, 9, 5)
    K0, mu0, lo, hi, b = _homogeneous(orc, shape)
    x, st, it, rel = orc.krylov(orc.identity_field(shape), K0, mu0, b, "cg", eta=1e-12)
    assert st == 0 and it == 2 and rel < 1e-12


def _hetero(orc, shape, seed):
    rng = np.random.default_rng(seed)
    ph = (rng.random(shape) < 0.3).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    F = ms.near_identity_field(shape, seed=seed + 1, scale=0.01)
    lo = 0.95 * min(m for _, m in TABLE)
    hi = 1.05 * 3 * max(k for k, _ in TABLE)
    b = orc.project(ms.random_field(shape, seed=seed + 2))
    return K, mu, F, lo, hi, b


@pytest.mark.parametrize("shape", [(9, 7, 8), (8, 8, 8)])
def test_residual_bounds_and_common_solution(orc, shape):
    K, mu, F, lo, hi, b = _hetero(orc, shape, 5)
    q = (hi / lo - 1) / (hi / lo + 1)
    for k in (1, 3, 10, 30):
        _, _, _, rel = orc.krylov(F, K, mu, b, "chebyshev", lo, hi, 1e-30, k)
        assert rel <= _cheb_bound(k, lo, hi) * (1 + 1e-9), k
        _, _, _, rel = orc.krylov(F, K, mu, b, "richardson", lo, hi, 1e-30, k)
        assert rel <= q ** k * (1 + 1e-9), k
    sols = {}
    for m in ("cg", "chebyshev", "richardson"):
        x, st, it, rel = orc.krylov(F, K, mu, b, m, lo, hi, 1e-11, 20000)
        assert st == 0, m
        res = orc.apply_operator(F, K, mu, x) - b
        assert np.linalg.norm(res) <= 2e-11 * np.linalg.norm(b), m
        sols[m] = (x, it)
    ref = sols["cg"][0]
    for m in ("chebyshev", "richardson"):
        assert np.linalg.norm(sols[m][0] - ref) <= 1e-9 * np.linalg.norm(ref), m
    # iterations: CG < Chebyshev < Richardson, Chebyshev within its a-priori count
    kc = next(k for k in range(1, 10000) if _cheb_bound(k, lo, hi) <= 1e-11)
    assert sols["cg"][1] < sols["chebyshev"][1] <= kc < sols["richardson"][1]


def test_increment_with_chebyshev_matches_cg(orc):
    shape = (7, 7, 7)
    ph = ms.cubic_inclusion(7, 3)
    K, mu = ms.phase_moduli(ph, TABLE)
    lo = 0.9 * min(m for _, m in TABLE)
    hi = 1.1 * 3 * max(k for k, _ in TABLE)
    Fbar = ms.simple_shear(0.05)
    st0, F0, P0, Pb0, S0 = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-10, 1e-12)
    st1, F1, P1, Pb1, S1 = orc.solve_increment_krylov(K, mu, orc.identity_field(shape), Fbar, "chebyshev", lo, hi,
                                                      1e-10, 1e-12)
    assert st0 == st1 == 0 and S0["n_solves"] == S1["n_solves"]
    assert np.max(np.abs(F1 - F0)) < 1e-9 and np.max(np.abs(Pb1 - Pb0)) < 1e-11
    assert sum(S1["cg_iters"]) > sum(S0["cg_iters"])


def test_invalid_bounds(orc):
    shape = (5, 5, 5)
    K, mu, F, lo, hi, b = _hetero(orc, shape, 2)
    for m, l, h in (("chebyshev", 0.0, 1.0), ("chebyshev", 2.0, 1.0), ("richardson", -1.0, 1.0)):
        _, st, it, _ = orc.krylov(F, K, mu, b, m, l, h)
        assert st == 5 and it == 0


# ---------------------------------------------------------------- GMRES
# Pins: a two-eigenvalue operator (homogeneous cell at F = I) is solved in two
# iterations (degree of its minimal polynomial); the residual norm never grows
# within a cycle (least-squares over nested Krylov spaces); unrestarted GMRES
# needs no more iterations than CG (it minimises the residual over the same
# space); restarted or not, it reaches CG's solution, checked with the operator.

def test_gmres_two_eigenvalues(orc):
    shape = (7, 9, 5)
    K0, mu0, lo, hi, b = _homogeneous(orc, shape)
    x, st, it, rel = orc.krylov(orc.identity_field(shape), K0, mu0, b, "gmres", 30, 0, 1e-12, 100)
    assert st == 0 and it == 2 and rel < 1e-12


def test_gmres_monotone_and_minimal(orc):
    shape = (9, 7, 8)
    K, mu, F, lo, hi, b = _hetero(orc, shape, 5)
    prev = 1.0
    for k in range(1, 25):
        _, _, it, rel = orc.krylov(F, K, mu, b, "gmres", 100, 0, 1e-30, k)
        assert it == k and rel <= prev * (1 + 1e-12), k
        prev = rel
    _, st_g, it_g, _ = orc.krylov(F, K, mu, b, "gmres", 500, 0, 1e-10, 5000)
    _, st_c, it_c, _ = orc.krylov(F, K, mu, b, "cg", 0, 0, 1e-10, 5000)
    assert st_g == st_c == 0 and it_g <= it_c


@pytest.mark.parametrize("m", [5, 20])
def test_gmres_restarted_solution(orc, m):
    shape = (8, 8, 8)
    K, mu, F, lo, hi, b = _hetero(orc, shape, 5)
    x, st, it, rel = orc.krylov(F, K, mu, b, "gmres", m, 0, 1e-11, 20000)
    xc, stc, itc, _ = orc.krylov(F, K, mu, b, "cg", 0, 0, 1e-11, 20000)
    assert st == stc == 0
    res = orc.apply_operator(F, K, mu, x) - b
    assert np.linalg.norm(res) <= 2e-11 * np.linalg.norm(b)
    assert np.linalg.norm(x - xc) <= 1e-9 * np.linalg.norm(xc)


def test_increment_with_gmres_matches_cg(orc):
    shape = (7, 7, 7)
    ph = ms.cubic_inclusion(7, 3)
    K, mu = ms.phase_moduli(ph, TABLE)
    Fbar = ms.simple_shear(0.05)
    st0, F0, P0, Pb0, S0 = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-10, 1e-12)
    st1, F1, P1, Pb1, S1 = orc.solve_increment_krylov(K, mu, orc.identity_field(shape), Fbar, "gmres", 20, 0,
                                                      1e-10, 1e-12)
    assert st0 == st1 == 0 and S0["n_solves"] == S1["n_solves"]
    assert np.max(np.abs(F1 - F0)) < 1e-9 and np.max(np.abs(Pb1 - Pb0)) < 1e-11
