"""Pins of the oracle's adjoint sensitivity of the homogenised stress.

The adjoint (one extra CG solve with the same symmetric projected-tangent
operator, derived from the boundary-condition system of Sec. 3.1 and the
symmetry of G of Sec. 2.3) must reproduce:
* central finite differences of g : P-bar with respect to the modulus at single
  voxels and along a random field direction (tight forward solves, h = 1e-6);
* a homogeneous cell, where the adjoint field vanishes and the gradient is the
  closed form (1/n) g : Fbar . 2 dev(E-bar) at every voxel;
* linearity in the cotangent g.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms

TIGHT = dict(eta_nw=1e-12, eta_cg=1e-13)


def _pbar(orc, K, mu, Fbar):
    shape = K.shape
    st, F, P, Pbar, S = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, **TIGHT)
    assert st == 0
    return F, Pbar


@pytest.fixture(scope="module")
def problem():
    N = 5
    rng = np.random.default_rng(1605)
    mu = 0.386 * np.exp(0.5 * rng.standard_normal((N, N, N)))
    K = np.full((N, N, N), 0.833)
    Fbar = ms.tensor(np.eye(3) + np.array([[0.04, 0.05, 0.0], [0.0, -0.02, 0.01], [0.02, 0.0, 0.01]]))
    g = np.array([1.0, 0.3, -0.2, 0.5, -1.0, 0.1, 0.0, 0.4, 0.7])
    return K, mu, Fbar, g


def test_adjoint_vs_central_differences_single_voxels(orc, problem):
    K, mu, Fbar, g = problem
    F, Pbar = _pbar(orc, K, mu, Fbar)
    st, dmu, dK, it = orc.adjoint(K, mu, F, g, eta_cg=1e-13)
    assert st == 0 and it > 0
    h = 1e-6
    for v in [(0, 0, 0), (2, 3, 1), (4, 1, 4)]:
        mp, mm = mu.copy(), mu.copy()
        mp[v] += h
        mm[v] -= h
        fd = (g @ _pbar(orc, K, mp, Fbar)[1] - g @ _pbar(orc, K, mm, Fbar)[1]) / (2 * h)
        assert abs(fd - dmu[v]) <= 1e-6 * abs(dmu[v]) + 1e-12, (v, fd, dmu[v])
        kp, km = K.copy(), K.copy()
        kp[v] += h
        km[v] -= h
        fdK = (g @ _pbar(orc, kp, mu, Fbar)[1] - g @ _pbar(orc, km, mu, Fbar)[1]) / (2 * h)
        assert abs(fdK - dK[v]) <= 1e-6 * abs(dK[v]) + 1e-12, (v, fdK, dK[v])


def test_adjoint_vs_directional_difference(orc, problem):
    K, mu, Fbar, g = problem
    F, Pbar = _pbar(orc, K, mu, Fbar)
    st, dmu, dK, it = orc.adjoint(K, mu, F, g, eta_cg=1e-13)
    d = np.random.default_rng(3).standard_normal(mu.shape)
    h = 1e-6
    fd = (g @ _pbar(orc, K, mu + h * d, Fbar)[1] - g @ _pbar(orc, K, mu - h * d, Fbar)[1]) / (2 * h)
    assert abs(fd - np.sum(dmu * d)) <= 1e-6 * abs(fd)


def test_adjoint_homogeneous_closed_form(orc):
    N = 5
    shape = (N, N, N)
    K = np.full(shape, 0.833)
    mu = np.full(shape, 0.386)
    Fb = np.eye(3) + np.array([[0.05, 0.02, 0.0], [0.01, 0.0, 0.03], [0.0, 0.0, -0.02]])
    g = np.arange(9, dtype=float) - 4.0
    F, _ = _pbar(orc, K, mu, Fb.reshape(9))
    st, dmu, dK, it = orc.adjoint(K, mu, F, g)
    assert st == 0 and it == 0  # G of a uniform field is zero: no CG work
    E = 0.5 * (Fb.T @ Fb - np.eye(3))
    dev = E - np.trace(E) / 3 * np.eye(3)
    ref_mu = np.sum(g.reshape(3, 3) * (Fb @ (2 * dev))) / N ** 3
    ref_K = np.sum(g.reshape(3, 3) * (np.trace(E) * Fb)) / N ** 3
    assert np.max(np.abs(dmu - ref_mu)) < 1e-16
    assert np.max(np.abs(dK - ref_K)) < 1e-16


def test_adjoint_linear_in_cotangent(orc, problem):
    K, mu, Fbar, g = problem
    F, _ = _pbar(orc, K, mu, Fbar)
    g2 = np.random.default_rng(5).standard_normal(9)
    _, a, _, _ = orc.adjoint(K, mu, F, g, eta_cg=1e-13)
    _, b, _, _ = orc.adjoint(K, mu, F, g2, eta_cg=1e-13)
    _, c, _, _ = orc.adjoint(K, mu, F, 2 * g - 3 * g2, eta_cg=1e-13)
    assert np.max(np.abs(c - (2 * a - 3 * b))) < 1e-10 * np.max(np.abs(c))
