"""Pins of the oracle's CG, Newton driver and full increments (Sec. 2.6, 3; Alg. 1).

What fixes the answer, independently of the oracle's own arithmetic:
* CG against a dense solve restricted to range(G) (basis from the eigenvectors
  of the assembled G matrix, operator assembled column by column).
* A homogeneous cell: F = Fbar everywhere, two solves with zero right-hand side.
* A one-dimensional laminate on an odd grid: the exact discrete solution is
  piecewise constant, F = Fbar + a_alpha (x) e_d, with the mean and traction
  continuity fixing the 3 unknowns; solved here by a separate small Newton.
  (Stands in for the analytical laminate comparison the paper mentions in Sec. 4.1.)
* Small-strain limit of the laminate: the harmonic / arithmetic shear-modulus
  averages of linear elasticity.
* A dense displacement-form Newton solve (unknowns u, F = Fbar + grad u,
  residual B^T P) on 3^3 and 5^3 grids: the same discrete problem written
  without G (App. D shows range(G) is exactly the set of gradients).
* The paper's cubic-inclusion example needs five Newton iterations (Sec. 4.4).
"""
import json
import os

import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms
from tests.test_oracle_projection import _grad_matrix

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]


def _assemble(fn, m):
    cols = []
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        cols.append(fn(e).reshape(-1))
    return np.array(cols).T


def test_cg_vs_dense_solve_on_range_of_G(orc):
    shape = (3, 3, 3)
    m = 9 * 27
    rng = np.random.default_rng(1)
    ph = rng.integers(0, 2, size=shape).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    F = ms.near_identity_field(shape, 2, 0.05)
    Gm = _assemble(lambda e: orc.project(e.reshape((9,) + shape)), m)
    w, V = np.linalg.eigh(0.5 * (Gm + Gm.T))
    Q = V[:, w > 0.5]  # orthonormal basis of range(G)
    Am = _assemble(lambda e: orc.apply_operator(F, K, mu, e.reshape((9,) + shape)), m)
    Ar = Q.T @ Am @ Q
    assert np.max(np.abs(Ar - Ar.T)) < 1e-12 * np.max(np.abs(Ar))  # symmetric on range(G)
    assert np.min(np.linalg.eigvalsh(0.5 * (Ar + Ar.T))) > 0          # positive definite
    b = orc.project(rng.standard_normal((9,) + shape))
    y = np.linalg.solve(Ar, Q.T @ b.reshape(-1))
    ref = Q @ y
    x, st, it, rel = orc.cg(F, K, mu, b, eta=1e-14)
    assert st == 0 and rel <= 1e-14
    assert np.max(np.abs(x.reshape(-1) - ref)) < 1e-11 * np.max(np.abs(ref))


def test_homogeneous_cell(orc):
    shape = (7, 7, 7)
    F0 = orc.identity_field(shape)
    Fbar = np.array([[1.02, 0.03, 0.0], [0.01, 0.99, 0.02], [0.0, -0.01, 1.01]]).reshape(9)
    st, F, P, Pbar, S = orc.solve_increment(0.833, 0.386, F0, Fbar)
    assert st == 0
    assert S["n_solves"] == 2 and S["cg_iters"] == [0, 0]
    assert np.max(np.abs(F - Fbar[:, None, None, None])) < 1e-15
    Ph = orc.svk_stress(Fbar.reshape(9, 1, 1, 1), 0.833, 0.386).reshape(9)
    assert np.max(np.abs(Pbar - Ph)) < 1e-15


def _laminate_bruteforce(orc, Fbar, f1, d, tab):
    """Piecewise-constant laminate state: 3 unknowns a (phase 1), a2 = -f1 a / f2."""
    f2 = 1.0 - f1
    Fb = Fbar.reshape(3, 3)
    a = np.zeros(3)

    def states(a):
        A1 = np.zeros((3, 3))
        A1[:, d] = a
        return Fb + A1, Fb - (f1 / f2) * A1

    for _ in range(50):
        F1, F2 = states(a)
        P1 = orc.svk_stress(F1.reshape(9, 1, 1, 1), *tab[1]).reshape(3, 3)
        P2 = orc.svk_stress(F2.reshape(9, 1, 1, 1), *tab[0]).reshape(3, 3)
        R = (P1 - P2)[:, d]
        if np.max(np.abs(R)) < 1e-16:
            break
        J = np.zeros((3, 3))
        for k in range(3):
            E = np.zeros((3, 3))
            E[k, d] = 1.0
            dP1 = orc.svk_tangent(F1.reshape(9, 1, 1, 1), *tab[1], E.reshape(9, 1, 1, 1)).reshape(3, 3)
            dP2 = orc.svk_tangent(F2.reshape(9, 1, 1, 1), *tab[0], (-(f1 / f2) * E).reshape(9, 1, 1, 1)).reshape(3, 3)
            J[:, k] = (dP1 - dP2)[:, d]
        a = a - np.linalg.solve(J, R)
    F1, F2 = states(a)
    P1 = orc.svk_stress(F1.reshape(9, 1, 1, 1), *tab[1]).reshape(9)
    P2 = orc.svk_stress(F2.reshape(9, 1, 1, 1), *tab[0]).reshape(9)
    return F1.reshape(9), F2.reshape(9), f1 * P1 + f2 * P2


@pytest.mark.parametrize("d", [0, 1, 2])
def test_laminate_vs_bruteforce(orc, d):
    N = 9
    shape = (N, N, N)
    ph = ms.laminate(shape, axis=d, frac=0.45)
    f1 = ph.mean()
    K, mu = ms.phase_moduli(ph, TABLE)
    Fbar = np.array([[1.05, 0.3, 0.0], [0.0, 1.0, 0.1], [0.05, 0.0, 0.97]]).reshape(9)
    F1, F2, Pbar_ref = _laminate_bruteforce(orc, Fbar, f1, d, TABLE)
    st, F, P, Pbar, S = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, eta_nw=1e-12,
                                            eta_cg=1e-13)
    assert st == 0
    assert np.max(np.abs(Pbar - Pbar_ref)) < 1e-11 * np.max(np.abs(Pbar_ref))
    m1 = ph.astype(bool)
    assert np.max(np.abs(F[:, m1] - F1[:, None])) < 1e-11
    assert np.max(np.abs(F[:, ~m1] - F2[:, None])) < 1e-11


def test_laminate_small_strain_limit(orc):
    # Linear elasticity of a laminate with normal e1 (layers along axis 0):
    # shear in the 1-2 plane sees the harmonic mean of mu, shear in the 2-3
    # plane the arithmetic mean.  P-bar / gamma approaches them with O(gamma) error.
    N = 9
    shape = (N, N, N)
    ph = ms.laminate(shape, axis=0, frac=0.45)
    f1 = ph.mean()
    K, mu = ms.phase_moduli(ph, TABLE)
    mus = np.array([TABLE[0][1], TABLE[1][1]])
    fr = np.array([1 - f1, f1])
    harm = 1.0 / np.sum(fr / mus)
    arith = np.sum(fr * mus)
    errs = []
    for g in [1e-2, 1e-3, 1e-4]:
        Fb = np.eye(3)
        Fb[0, 1] = g
        _, _, _, Pb, _ = orc.solve_increment(K, mu, orc.identity_field(shape), Fb.reshape(9), 1e-12, 1e-13)
        Fc = np.eye(3)
        Fc[1, 2] = g
        _, _, _, Pc, _ = orc.solve_increment(K, mu, orc.identity_field(shape), Fc.reshape(9), 1e-12, 1e-13)
        errs.append((abs(Pb[1] / g - harm) / harm, abs(Pc[5] / g - arith) / arith))
    errs = np.array(errs)
    assert np.all(errs[:, 0] < 5 * np.array([1e-2, 1e-3, 1e-4]))
    assert np.all(errs[:, 1] < 5 * np.array([1e-2, 1e-3, 1e-4]))
    assert errs[2, 0] < errs[0, 0] / 50 and errs[2, 1] < errs[0, 1] / 50


@pytest.mark.parametrize("N,seed", [(3, 0), (5, 1)])
def test_dense_displacement_form_newton(orc, N, seed):
    shape = (N, N, N)
    n = N ** 3
    rng = np.random.default_rng(seed)
    ph = rng.integers(0, 2, size=shape).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    Fbar = np.array([[1.03, 0.08, 0.0], [0.02, 0.98, 0.03], [0.0, -0.04, 1.01]]).reshape(9)
    B = _grad_matrix(shape)  # 9n x 3n spectral gradient
    u = np.zeros(3 * n)
    for _ in range(30):
        F = Fbar[:, None] + (B @ u).reshape(9, n)
        P = orc.svk_stress(F.reshape((9,) + shape), K, mu).reshape(-1)
        R = B.T @ P
        if np.max(np.abs(R)) < 1e-15:
            break
        cols = [orc.svk_tangent(F.reshape((9,) + shape), K, mu, B[:, k].reshape((9,) + shape)).reshape(-1)
                for k in range(3 * n)]
        J = B.T @ np.array(cols).T
        u = u - np.linalg.lstsq(J, R, rcond=None)[0]
    Fref = (Fbar[:, None] + (B @ u).reshape(9, n)).reshape((9,) + shape)
    st, Fo, Po, Pbar, S = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-12, 1e-13)
    assert st == 0
    assert np.max(np.abs(Fo - Fref)) < 1e-10
    # mean of F is prescribed exactly (Sec. 3.1)
    assert np.max(np.abs(Fo.reshape(9, -1).mean(axis=1) - Fbar)) < 1e-14


def test_two_increments_equal_one(orc):
    # hyperelastic equilibrium is path independent: reaching Fbar in two
    # increments gives the state reached in one (unique solution)
    N = 7
    shape = (N, N, N)
    ph = ms.cubic_inclusion(N, 3)
    K, mu = ms.phase_moduli(ph, TABLE)
    Fa = ms.simple_shear(0.05)
    Fb = ms.simple_shear(0.1)
    st, F1, _, _, _ = orc.solve_increment(K, mu, orc.identity_field(shape), Fa, 1e-12, 1e-13)
    st2, F2, P2, Pb2, S2 = orc.solve_increment(K, mu, F1, Fb, 1e-12, 1e-13)
    st3, F3, P3, Pb3, S3 = orc.solve_increment(K, mu, orc.identity_field(shape), Fb, 1e-12, 1e-13)
    assert st == st2 == st3 == 0
    assert np.max(np.abs(Pb2 - Pb3)) < 1e-12
    assert np.max(np.abs(F2 - F3)) < 1e-11
    # equilibrium at convergence: ||G(P)|| small against ||P||
    assert np.linalg.norm(orc.project(P3)) < 1e-9 * np.linalg.norm(P3)


def test_failure_statuses_leave_state_untouched(orc):
    N = 5
    shape = (N, N, N)
    ph = ms.cubic_inclusion(N, 2)
    K, mu = ms.phase_moduli(ph, TABLE)
    F0 = orc.identity_field(shape)
    st, F, _, _, S = orc.solve_increment(K, mu, F0, ms.simple_shear(0.05), max_cg=1)
    assert st == 1 and np.array_equal(F, F0)           # CG iteration limit
    st, F, _, _, S = orc.solve_increment(K, mu, F0, np.full(9, np.nan))
    assert st == 4 and np.array_equal(F, F0)           # non-finite load
    st, F, _, _, S = orc.solve_increment(K, -mu, F0, ms.simple_shear(0.05))
    assert st == 2 and np.array_equal(F, F0)           # indefinite tangent -> breakdown


@pytest.mark.slow
def test_paper_cubic_inclusion_five_iterations(orc):
    g = json.load(open(os.path.join(GOLD, "paper_examples.json")))["cubic_inclusion_shear"]
    N = g["N"]
    ph = ms.cubic_inclusion(N, g["inclusion"])
    K, mu = ms.phase_moduli(ph, TABLE)
    st, F, P, Pbar, S = orc.solve_increment(K, mu, orc.identity_field((N, N, N)), ms.simple_shear(g["gamma"]),
                                            g["eta_newton"], g["eta_cg"])
    assert st == 0
    assert S["n_solves"] == g["newton_iterations"]
    assert np.max(np.abs(F.reshape(9, -1).mean(axis=1) - ms.simple_shear(g["gamma"]))) < 1e-13
