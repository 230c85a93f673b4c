"""Pins of the oracle's second even-grid choice of the projection (App. C).

On an even axis the paper allows two values of G-hat at Nyquist frequencies:
zero (the default, which keeps F compatible) or the identity (which keeps the
stress equilibrated).  What fixes the identity choice here, independently of
the oracle's own transforms:
* brute force: it is the orthogonal projector onto the gradients without
  Nyquist content (B B^+, as in the projection pins) plus the fields whose
  spectrum lies on Nyquist frequencies only (assembled with numpy's FFT);
* the difference of the two choices is exactly the Nyquist content of the
  input (numpy's FFT with a frequency mask);
* pure-Nyquist fields are kept, odd grids see no difference, idempotence and
  self-adjointness hold;
* a dense Newton solve of the same discrete problem written without CG or the
  oracle's FFT (unknowns F = Fbar + Q y with Q an orthonormal basis of the
  brute-force range, residual Q^T P) reproduces the increment; its stress is
  equilibrated at every frequency (zero Nyquist content, rows orthogonal to xi).

With the identity choice every field with Nyquist content is in range(G),
rotations F W (W skew) included, on which the St. Venant-Kirchhoff tangent acts
through its geometric part p S only.  Under tension (S positive) the operator
stays positive definite but poorly conditioned; where S has a compressive
direction (shear) it is indefinite on range(G) and CG breaks down, which the
dense reduced tangent shows independently.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms
from tests.test_oracle_projection import _grad_matrix, _nyquist_mask

TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]


def _nyquist_content(A):
    """The part of A whose spectrum lies on Nyquist frequencies (numpy FFT)."""
    shape = A.shape[-3:]
    H = np.fft.fftn(A.reshape((-1,) + shape), axes=(1, 2, 3))
    H[:, ~_nyquist_mask(shape)] = 0.0
    return np.real(np.fft.ifftn(H, axes=(1, 2, 3))).reshape(A.shape)


def _nyquist_projector(shape):
    n = int(np.prod(shape))
    cols = []
    for k in range(9 * n):
        e = np.zeros(9 * n)
        e[k] = 1.0
        cols.append(_nyquist_content(e.reshape((9,) + shape)).reshape(-1))
    return np.array(cols).T


def _range_basis(shape):
    B = _grad_matrix(shape)
    Q = B @ np.linalg.pinv(B, rcond=1e-10) + _nyquist_projector(shape)
    w, V = np.linalg.eigh(0.5 * (Q + Q.T))
    return Q, V[:, w > 0.5]


@pytest.mark.parametrize("shape", [(4, 4, 4), (3, 4, 4), (4, 3, 2), (2, 5, 4)])
def test_identity_choice_equals_bruteforce_projector(orc, shape):
    Q, _ = _range_basis(shape)
    assert np.max(np.abs(Q @ Q - Q)) < 1e-12  # the two parts are orthogonal projectors
    rng = np.random.default_rng(7)
    for _ in range(3):
        A = rng.standard_normal((9,) + shape)
        got = orc.project(A, nyq_identity=True).reshape(-1)
        ref = Q @ A.reshape(-1)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), shape


@pytest.mark.parametrize("shape", [(6, 4, 8), (8, 5, 6), (5, 7, 4), (4, 4, 9)])
def test_choices_differ_by_the_nyquist_content(orc, shape):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal((9,) + shape)
    d = orc.project(A, nyq_identity=True) - orc.project(A)
    ref = _nyquist_content(A)
    assert np.max(np.abs(ref)) > 0.1
    assert np.max(np.abs(d - ref)) < 1e-13 * np.max(np.abs(A)) * 10


def test_pure_nyquist_fields_are_kept(orc):
    N = 8
    x = np.arange(N)
    rng = np.random.default_rng(3)
    T = rng.standard_normal(9)
    alt = np.cos(np.pi * x)
    wave = np.cos(2 * np.pi * x / N)
    # Nyquist along a0 only; along a1 with a non-Nyquist a2 wave; along a2 with a0 wave
    for prof in (alt[:, None, None] * np.ones((1, N, N)),
                 np.ones((N, 1, 1)) * alt[None, :, None] * wave[None, None, :],
                 wave[:, None, None] * np.ones((1, N, 1)) * alt[None, None, :]):
        A = T[:, None, None, None] * prof[None]
        assert np.max(np.abs(orc.project(A, nyq_identity=True) - A)) < 1e-13
        assert np.max(np.abs(orc.project(A))) < 1e-13


@pytest.mark.parametrize("shape", [(5, 7, 3), (9, 9, 9)])
def test_odd_grids_have_one_choice(orc, shape):
    A = np.random.default_rng(1).standard_normal((9,) + shape)
    assert np.array_equal(orc.project(A, nyq_identity=True), orc.project(A))


@pytest.mark.parametrize("shape", [(6, 6, 6), (8, 4, 6), (4, 6, 5)])
def test_identity_choice_invariants(orc, shape):
    rng = np.random.default_rng(len(shape) + shape[0])
    A = rng.standard_normal((9,) + shape)
    B = rng.standard_normal((9,) + shape)
    GA = orc.project(A, nyq_identity=True)
    GB = orc.project(B, nyq_identity=True)
    s = np.max(np.abs(GA))
    assert np.max(np.abs(orc.project(GA, nyq_identity=True) - GA)) < 1e-13 * s
    assert abs(np.sum(B * GA) - np.sum(GB * A)) < 1e-11 * abs(np.sum(B * GA)) + 1e-12
    assert np.max(np.abs(GA.reshape(9, -1).mean(axis=1))) < 1e-14 * s * 10


@pytest.mark.parametrize("shape,seed", [((4, 4, 4), 2), ((4, 3, 4), 5)])
def test_dense_newton_with_identity_choice(orc, shape, seed):
    n = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    ph = rng.integers(0, 2, size=shape).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    Fbar = np.array([[1.03, 0.004, 0.0], [0.002, 1.02, 0.003], [0.0, -0.002, 1.025]]).reshape(9)  # tension
    _, Q = _range_basis(shape)  # orthonormal basis of range(G) with the identity choice
    y = np.zeros(Q.shape[1])
    for _ in range(30):
        F = (Fbar[:, None] + (Q @ y).reshape(9, n)).reshape((9,) + shape)
        R = Q.T @ orc.svk_stress(F, K, mu).reshape(-1)
        if np.max(np.abs(R)) < 1e-15:
            break
        cols = [orc.svk_tangent(F, K, mu, Q[:, k].reshape((9,) + shape)).reshape(-1) for k in range(Q.shape[1])]
        y = y - np.linalg.solve(Q.T @ np.array(cols).T, R)
    Fref = (Fbar[:, None] + (Q @ y).reshape(9, n)).reshape((9,) + shape)
    st, Fo, Po, Pbar, S = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-12, 1e-13,
                                              nyq_identity=True)
    assert st == 0
    assert np.max(np.abs(Fo - Fref)) < 1e-10
    assert np.max(np.abs(Fo.reshape(9, -1).mean(axis=1) - Fbar)) < 1e-14
    # the default choice reaches a different F on this even grid
    st0, F0, _, _, _ = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-12, 1e-13)
    assert st0 == 0 and np.max(np.abs(F0 - Fo)) > 1e-6


def test_identity_choice_is_singular_then_indefinite(orc):
    # dense reduced tangent Q^T K Q on range(G).  At F = I (S = 0) the identity
    # choice leaves the rotations at the Nyquist frequencies in its null space
    # (3 per Nyquist frequency); after the boundary-condition step of a shear
    # load (its minimum-norm solution, which CG from x = 0 also returns) the
    # geometric part p S makes it indefinite, so the next CG breaks down.  The
    # default choice is positive definite at both states.
    shape = (4, 4, 4)
    n = 64
    rng = np.random.default_rng(2)
    ph = rng.integers(0, 2, size=shape).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    Fbar = ms.simple_shear(0.05)
    Qz = _grad_matrix(shape)
    Qz = np.linalg.svd(Qz, full_matrices=False)[0][:, :np.linalg.matrix_rank(Qz)]
    I = orc.identity_field(shape)
    U = np.broadcast_to((Fbar - I.reshape(9, -1)[:, 0])[:, None, None, None], I.shape)
    eig = {}
    for name, Q in (("zero", Qz), ("identity", _range_basis(shape)[1])):
        def J_at(F):
            cols = [orc.svk_tangent(F, K, mu, Q[:, k].reshape((9,) + shape)).reshape(-1) for k in range(Q.shape[1])]
            J = Q.T @ np.array(cols).T
            assert np.max(np.abs(J - J.T)) < 1e-12 * np.max(np.abs(J))
            return J
        J0 = J_at(I)
        y = np.linalg.lstsq(J0, -Q.T @ orc.svk_tangent(I, K, mu, U).reshape(-1), rcond=1e-12)[0]
        F1 = (Fbar[:, None] + (Q @ y).reshape(9, n)).reshape((9,) + shape)
        eig[name] = (np.linalg.eigvalsh(J0), np.linalg.eigvalsh(J_at(F1)))
    nyq_freqs = n - 3 ** 3
    assert eig["zero"][0].min() > 0.5 and eig["zero"][1].min() > 0.5
    assert np.sum(np.abs(eig["identity"][0]) < 1e-12) == 3 * nyq_freqs
    assert eig["identity"][0].min() > -1e-12
    assert eig["identity"][1].min() < -1e-3
    st, F, _, _, S = orc.solve_increment(K, mu, I, Fbar, 1e-12, 1e-13, nyq_identity=True)
    assert st == 2 and S["n_solves"] == 2 and np.array_equal(F, I)


def test_identity_choice_equilibrates_the_stress(orc):
    # converged stress: no Nyquist content and rows orthogonal to xi elsewhere
    # (numpy spectra); with the default choice the stress keeps Nyquist content
    # while F - Fbar has none
    shape = (8, 6, 8)
    ph = ms.cubic_inclusion(8, 3)[:, 1:7, :]
    K, mu = ms.phase_moduli(np.ascontiguousarray(ph), TABLE)
    Fbar = np.array([[1.03, 0.004, 0.0], [0.002, 1.02, 0.003], [0.0, -0.002, 1.025]]).reshape(9)  # tension
    res = {}
    for nyq in (False, True):
        st, F, P, Pbar, S = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-12, 1e-13,
                                                nyq_identity=nyq)
        assert st == 0
        Ph = np.fft.fftn(P.reshape((3, 3) + shape), axes=(2, 3, 4))
        xi = np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij")
        div = sum(Ph[:, j] * xi[j] for j in range(3))
        ny = _nyquist_mask(shape)
        s = np.max(np.abs(Ph[:, :, ~ny]))
        res[nyq] = (np.max(np.abs(div[:, ~ny])) / s, np.max(np.abs(Ph[:, :, ny])) / s,
                    np.max(np.abs(_nyquist_content(F))), Pbar)
    assert res[True][0] < 1e-10 and res[True][1] < 1e-10
    assert res[False][0] < 1e-10 and res[False][1] > 1e-6 and res[False][2] < 1e-13
    # the homogenised stress barely depends on the choice (App. C)
    assert np.max(np.abs(res[True][3] - res[False][3])) < 0.05 * np.max(np.abs(res[False][3]))
