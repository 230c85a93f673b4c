"""Pins of the oracle's St. Venant-Kirchhoff law and its consistent tangent (Sec. 4).

* Closed-form states: P(I) = 0, P(R) = 0 for a rotation, objectivity
  P(QF) = Q P(F), and the homogeneous uniaxial stretch worked out by hand.
* The tangent against central finite differences of the stress.
* The tangent against the paper's fourth-order form of the consistent tangent
  (Sec. 4.3): K = S.I + I^RT : (F.C.F^T) : I^RT with dP^T = K : dF^T, assembled
  here from the nomenclature appendix (I_ijkl = d_il d_jk, I^RT_ijkl = d_ik d_jl,
  A:B = A_ijkl B_lk).  This is a different route to the same linearisation.
* Major symmetry <q, dP(p)> = <p, dP(q)>, and the small-strain limit at F = I.
"""
import numpy as np
import pytest

K0, MU0 = 0.833, 0.386


def _rot(axis, ang):
    a = np.asarray(axis, dtype=float)
    a /= np.linalg.norm(a)
    W = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * W + (1 - np.cos(ang)) * W @ W


def _one(F33):
    return np.asarray(F33, dtype=float).reshape(9, 1, 1, 1)


def test_stress_free_states(orc):
    assert np.max(np.abs(orc.svk_stress(_one(np.eye(3)), K0, MU0))) == 0.0
    for ax, ang in [((1, 2, 3), 0.7), ((0, 0, 1), 1.3), ((1, -1, 0.5), 2.9)]:
        P = orc.svk_stress(_one(_rot(ax, ang)), K0, MU0)
        assert np.max(np.abs(P)) < 1e-15


def test_objectivity(orc):
    rng = np.random.default_rng(3)
    F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
    Q = _rot((0.3, 1, -2), 0.9)
    P = orc.svk_stress(_one(F), K0, MU0).reshape(3, 3)
    PQ = orc.svk_stress(_one(Q @ F), K0, MU0).reshape(3, 3)
    assert np.max(np.abs(PQ - Q @ P)) < 1e-14


@pytest.mark.parametrize("lam", [0.9, 1.05, 1.3])
def test_uniaxial_closed_form(orc, lam):
    # F = diag(lam, 1, 1): E11 = (lam^2 - 1)/2, S11 = (lam_L + 2 mu) E11,
    # S22 = S33 = lam_L E11, P = F S.
    lamL = K0 - 2 * MU0 / 3
    E11 = 0.5 * (lam ** 2 - 1)
    ref = np.diag([lam * (lamL + 2 * MU0) * E11, lamL * E11, lamL * E11])
    P = orc.svk_stress(_one(np.diag([lam, 1, 1])), K0, MU0).reshape(3, 3)
    assert np.max(np.abs(P - ref)) < 1e-15


def _paper_tangent(F, S, K, mu):
    """Fourth-order tangent of the paper's Sec. 4.3, nomenclature conventions."""
    d = np.eye(3)
    I4 = np.einsum("il,jk->ijkl", d, d)
    I4rt = np.einsum("ik,jl->ijkl", d, d)
    II = np.einsum("ij,kl->ijkl", d, d)
    I4s = 0.5 * (I4 + I4rt)
    C = K * II + 2 * mu * (I4s - II / 3.0)          # isotropic stiffness, (K, mu) split
    dd44 = lambda A, B: np.einsum("ijkl,lkmn->ijmn", A, B)   # A : B
    SI = np.einsum("ij,jkmn->ikmn", S, I4)              # S . I
    FCFt = np.einsum("ij,jkmn,pn->ikmp", F, C, F)       # F . C . F^T
    return SI + dd44(dd44(I4rt, FCFt), I4rt)


def test_tangent_vs_paper_fourth_order_form(orc):
    rng = np.random.default_rng(8)
    for _ in range(5):
        F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
        dF = rng.standard_normal((3, 3))
        K = rng.uniform(0.5, 9)
        mu = rng.uniform(0.3, 4)
        lamL = K - 2 * mu / 3
        E = 0.5 * (F.T @ F - np.eye(3))
        S = lamL * np.trace(E) * np.eye(3) + 2 * mu * E
        K4 = _paper_tangent(F, S, K, mu)
        dPT = np.einsum("ijkl,lk->ij", K4, dF.T)   # dP^T = K : dF^T
        got = orc.svk_tangent(_one(F), K, mu, _one(dF)).reshape(3, 3)
        assert np.max(np.abs(got - dPT.T)) < 1e-13 * np.max(np.abs(dPT))


def test_tangent_vs_finite_differences(orc):
    rng = np.random.default_rng(9)
    shape = (3, 4, 5)
    F = np.eye(3).reshape(9, 1, 1, 1) + 0.2 * rng.standard_normal((9,) + shape)
    p = rng.standard_normal((9,) + shape)
    K = rng.uniform(0.5, 9, size=shape)
    mu = rng.uniform(0.3, 4, size=shape)
    h = 1e-6
    fd = (orc.svk_stress(F + h * p, K, mu) - orc.svk_stress(F - h * p, K, mu)) / (2 * h)
    got = orc.svk_tangent(F, K, mu, p)
    assert np.max(np.abs(got - fd)) < 1e-8 * np.max(np.abs(got))


def test_tangent_major_symmetry_and_small_strain_limit(orc):
    rng = np.random.default_rng(10)
    F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    p, q = rng.standard_normal((2, 3, 3))
    a = np.sum(q * orc.svk_tangent(_one(F), K0, MU0, _one(p)).reshape(3, 3))
    b = np.sum(p * orc.svk_tangent(_one(F), K0, MU0, _one(q)).reshape(3, 3))
    assert abs(a - b) < 1e-14 * abs(a)
    # at F = I the tangent is linear elasticity acting on sym(p)
    lamL = K0 - 2 * MU0 / 3
    ref = lamL * np.trace(p) * np.eye(3) + MU0 * (p + p.T)
    got = orc.svk_tangent(_one(np.eye(3)), K0, MU0, _one(p)).reshape(3, 3)
    assert np.max(np.abs(got - ref)) < 1e-15
