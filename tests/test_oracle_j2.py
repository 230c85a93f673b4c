"""Pins of the oracle's finite-strain J2 plasticity (Sec. 5).

* The cyclic Jacobi eigen-decomposition against numpy's symmetric eigensolver,
  including coincident and nearly coincident eigenvalues.
* Below yield the law is Hencky hyperelasticity: tau = K tr(e) I + 2 mu dev(e),
  e = ln(F F^T) / 2, P = tau F^-T -- evaluated here independently with numpy.
* After a plastic return the state sits on the yield surface,
  tau_eq = tau_y0 + H eps_p (consistency, linear hardening of Sec. 5.5), and the
  plastic flow is isochoric: det C_p^-1 stays 1.
* The consistent tangent (Sec. 5.3-5.4) against central differences of the
  stress at frozen history, in elastic and plastic states and at coincident
  eigenvalues; its major symmetry.
* A one-dimensional J2 laminate loaded over several increments: the FFT solve
  must reproduce the piecewise-homogeneous solution found by a per-phase
  Newton iteration with the same history.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms

K0, MU0 = 0.833, 0.386


def _one(A):
    return np.asarray(A, dtype=float).reshape(9, 1, 1, 1)


def _virgin():
    return np.array([1, 1, 1, 0, 0, 0, 0.0]).reshape(7, 1, 1, 1)


def test_jacobi_vs_numpy(orc):
    rng = np.random.default_rng(0)
    cases = [np.eye(3), np.diag([2.0, 2.0, 1.0]), np.diag([1.0, 1.0 + 1e-12, 3.0])]
    for _ in range(20):
        A = rng.standard_normal((3, 3))
        cases.append(A @ A.T + 0.1 * np.eye(3))
    Q = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    cases.append(Q @ np.diag([1.5, 1.5, 0.7]) @ Q.T)
    for A in cases:
        w, V = orc.jacobi_eig3(A)
        assert np.allclose(np.sort(w), np.linalg.eigvalsh(A), atol=1e-14 * max(1, np.abs(A).max()))
        assert np.max(np.abs(V @ np.diag(w) @ V.T - A)) < 1e-14 * max(1, np.abs(A).max())
        assert np.max(np.abs(V.T @ V - np.eye(3))) < 1e-14


def _hencky_P(F, K, mu):
    b = F @ F.T
    w, V = np.linalg.eigh(b)
    e = V @ np.diag(0.5 * np.log(w)) @ V.T
    tau = K * np.trace(e) * np.eye(3) + 2 * mu * (e - np.trace(e) / 3 * np.eye(3))
    return tau @ np.linalg.inv(F).T


def test_elastic_states_are_hencky(orc):
    rng = np.random.default_rng(1)
    for _ in range(5):
        F = np.eye(3) + 0.002 * rng.standard_normal((3, 3))
        st, P, hn = orc.j2_stress(_one(F), K0, MU0, 1.0, 0.01, _virgin())
        assert st == 0
        assert np.max(np.abs(P.reshape(3, 3) - _hencky_P(F, K0, MU0))) < 1e-15
        assert hn.ravel()[6] == 0.0  # no plastic flow
        assert np.allclose(hn.ravel(), _virgin().ravel(), rtol=0, atol=1e-14)  # C_p^-1 stays I


def _tau_eq(P, F):
    tau = P @ F.T
    dev = tau - np.trace(tau) / 3 * np.eye(3)
    return np.sqrt(1.5 * np.sum(dev * dev))


@pytest.mark.parametrize("H", [0.01, 0.0, 0.2])
def test_return_map_consistency_and_isochoric_flow(orc, H):
    rng = np.random.default_rng(2)
    ty0 = 0.003
    for _ in range(5):
        F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
        st, P, hn = orc.j2_stress(_one(F), K0, MU0, ty0, H, _virgin())
        assert st == 0
        ep = hn.ravel()[6]
        assert ep > 0  # these strains are far beyond yield
        assert abs(_tau_eq(P.reshape(3, 3), F) - (ty0 + H * ep)) < 1e-12 * ty0 * 10
        h = hn.ravel()
        Cpi = np.array([[h[0], h[3], h[5]], [h[3], h[1], h[4]], [h[5], h[4], h[2]]])
        assert abs(np.linalg.det(Cpi) - 1.0) < 1e-12
        # a second evaluation with the returned history is elastic (on the surface)
        st2, P2, hn2 = orc.j2_stress(_one(F), K0, MU0, ty0, H, hn)
        assert abs(hn2.ravel()[6] - ep) < 1e-12 * max(ep, 1e-3)
        assert np.max(np.abs(P2 - P)) < 1e-11


@pytest.mark.parametrize("kind", ["elastic", "plastic", "identity", "preloaded"])
def test_tangent_vs_central_differences(orc, kind):
    rng = np.random.default_rng(3)
    ty0, H = 0.003, 0.01
    hist = _virgin()
    if kind == "elastic":
        F = np.eye(3) + 0.001 * rng.standard_normal((3, 3))
    elif kind == "plastic":
        F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    elif kind == "identity":
        F = np.eye(3)
    else:  # history from a previous plastic state, then a further step
        F0 = np.eye(3) + 0.04 * rng.standard_normal((3, 3))
        _, _, hist = orc.j2_stress(_one(F0), K0, MU0, ty0, H, _virgin())
        F = F0 + 0.02 * rng.standard_normal((3, 3))
    for _ in range(3):
        d = rng.standard_normal((3, 3))
        st, dP = orc.j2_tangent(_one(F), K0, MU0, ty0, H, hist, _one(d))
        assert st == 0
        h = 1e-7
        Pp = orc.j2_stress(_one(F + h * d), K0, MU0, ty0, H, hist)[1]
        Pm = orc.j2_stress(_one(F - h * d), K0, MU0, ty0, H, hist)[1]
        fd = (Pp - Pm) / (2 * h)
        assert np.max(np.abs(dP - fd)) < 2e-6 * np.max(np.abs(dP)), kind


def test_tangent_major_symmetry_and_identity_limit(orc):
    rng = np.random.default_rng(4)
    ty0, H = 0.003, 0.01
    F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    p, q = rng.standard_normal((2, 3, 3))
    a = np.sum(q * orc.j2_tangent(_one(F), K0, MU0, ty0, H, _virgin(), _one(p))[1].reshape(3, 3))
    b = np.sum(p * orc.j2_tangent(_one(F), K0, MU0, ty0, H, _virgin(), _one(q))[1].reshape(3, 3))
    assert abs(a - b) < 1e-12 * abs(a)
    # at F = I (all eigenvalues coincide) the tangent is linear elasticity on sym(p)
    lam = K0 - 2 * MU0 / 3
    ref = lam * np.trace(p) * np.eye(3) + MU0 * (p + p.T)
    got = orc.j2_tangent(_one(np.eye(3)), K0, MU0, ty0, H, _virgin(), _one(p))[1].reshape(3, 3)
    assert np.max(np.abs(got - ref)) < 1e-15


def _laminate_j2_bruteforce(orc, Fbars, f1, d, mats):
    """Piecewise-homogeneous J2 laminate over increments: per phase F_a =
    Fbar + a_a (x) e_d, f1 a_1 + f2 a_2 = 0, traction continuity, each phase
    with its own history.  Returns the P-bar after every increment."""
    f2 = 1 - f1
    hists = [_virgin(), _virgin()]
    a = np.zeros(3)
    out = []
    for Fb in Fbars:
        Fb = Fb.reshape(3, 3)

        def states(a):
            A = np.zeros((3, 3))
            A[:, d] = a
            return [Fb - (f1 / f2) * A, Fb + A]  # phase 0, phase 1

        for _ in range(60):
            Fs = states(a)
            Ps = [orc.j2_stress(_one(Fs[k]), *mats[k], hists[k])[1].reshape(3, 3) for k in range(2)]
            R = (Ps[1] - Ps[0])[:, d]
            if np.max(np.abs(R)) < 1e-15:
                break
            J = np.zeros((3, 3))
            for k in range(3):
                E = np.zeros((3, 3))
                E[k, d] = 1.0
                d1 = orc.j2_tangent(_one(Fs[1]), *mats[1], hists[1], _one(E))[1].reshape(3, 3)
                d0 = orc.j2_tangent(_one(Fs[0]), *mats[0], hists[0], _one(-(f1 / f2) * E))[1].reshape(3, 3)
                J[:, k] = (d1 - d0)[:, d]
            a = a - np.linalg.solve(J, R)
        Fs = states(a)
        res = [orc.j2_stress(_one(Fs[k]), *mats[k], hists[k]) for k in range(2)]
        hists = [res[0][2], res[1][2]]
        out.append(f2 * res[0][1].ravel() + f1 * res[1][1].ravel())
    return out


def test_j2_laminate_vs_bruteforce(orc):
    N = 9
    shape = (N, N, N)
    d = 1
    ph = ms.laminate(shape, axis=d, frac=0.45)
    f1 = ph.mean()
    mats = [(K0, MU0, 0.003, 0.01), (K0, MU0, 0.006, 0.01)]
    K = np.full(shape, K0)
    mu = np.full(shape, MU0)
    ty0 = np.where(ph == 1, 0.006, 0.003)
    H = np.full(shape, 0.01)
    Fbars = [ms.simple_shear(0.005 * t) for t in range(1, 7)]
    for k in range(len(Fbars)):  # add a stretch so the laminate is not trivially uniform
        Fbars[k] = Fbars[k].copy()
        Fbars[k][0] += 0.002 * (k + 1)
    ref = _laminate_j2_bruteforce(orc, Fbars, f1, d, mats)
    F = orc.identity_field(shape)
    hist = orc.virgin_history(shape)
    for k, Fb in enumerate(Fbars):
        st, F, P, Pbar, hist, S = orc.solve_increment_j2(K, mu, ty0, H, hist, F, Fb, 1e-12, 1e-13)
        assert st == 0, k
        assert np.max(np.abs(Pbar - ref[k])) < 1e-10 * np.max(np.abs(ref[k])), k
    assert hist[6].max() > 0  # plastic flow happened


def test_j2_homogeneous_increments(orc):
    shape = (5, 5, 5)
    F = orc.identity_field(shape)
    hist = orc.virgin_history(shape)
    Fp, hp = np.eye(3), _virgin()
    for t in range(1, 5):
        Fb = ms.simple_shear(0.01 * t)
        st, F, P, Pbar, hist, S = orc.solve_increment_j2(K0, MU0, 0.003, 0.01, hist, F, Fb)
        assert st == 0 and S["cg_iters"] == [0, 0]
        st, Pp, hp = orc.j2_stress(_one(Fb), K0, MU0, 0.003, 0.01, hp)
        assert np.max(np.abs(Pbar - Pp.ravel())) < 1e-15


def test_j2_inverted_deformation_fails(orc):
    """det F <= 0 has no logarithmic strain: the return mapping, and with it
    the increment, fails (status 6) instead of producing a stress."""
    shape = (5, 5, 5)
    ph = ms.laminate(shape, 0, 0.4)
    tab = np.array([(K0, MU0, 0.003, 0.01), (K0, MU0, 0.006, 0.01)])
    K, mu, ty0, H = (tab[ph, k].copy() for k in range(4))
    Fb = np.diag([-0.5, 1.0, 1.0]).reshape(9)
    st, F, P, Pbar, hist, S = orc.solve_increment_j2(K, mu, ty0, H, orc.virgin_history(shape),
                                                     orc.identity_field(shape), Fb)
    assert st == 6 and S["n_solves"] == 1
