"""Pins of the oracle's macroscopic tangent and mixed macroscopic control.

Neither is in the paper (Sec. 3.1 prescribes the whole macroscopic deformation
gradient and points to the literature for stress or mixed control); both reuse
its boundary-condition system.  What fixes the answer independently:
* a homogeneous cell under uniaxial stress (lateral and shear stresses zero,
  F11 and the lower off-diagonal entries prescribed) has the closed-form state
  F = diag(l, t, t), with S22 = 0 giving t^2 = 1 - lambda (l^2 - 1) / (2 (lambda + mu));
* a homogeneous cell's macroscopic tangent is the local tangent itself;
* central finite differences of deformation-controlled solves reproduce the
  macroscopic tangent, which is also major-symmetric (a hyperelastic cell's
  homogenised stress derives from a potential);
* round trips: the stress a deformation-controlled solve reaches, prescribed
  back under any mask (uniaxial, shear, all nine components), returns the same
  Fbar and the same field, for St. Venant-Kirchhoff and for J2.
A mask that leaves a direction of Fbar without stress response (all nine
components prescribed at zero stress: rigid rotations) makes the masked
tangent block singular; the solve stops with an invalid-argument status.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms

TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]
UNIAXIAL = np.array([0, 1, 1, 0, 1, 1, 0, 0, 1])  # P12 P13 P22 P23 P33 prescribed (zero)


def test_homogeneous_uniaxial_stress_closed_form(orc):
    shape = (5, 4, 6)
    K0, mu0 = ms.K_HARD, ms.MU_HARD
    lam = 1.04
    Fbar = np.eye(3).reshape(9).copy()
    Fbar[0] = lam
    st, F, P, Pb, Fb, S, outer = orc.solve_increment_mixed(K0, mu0, orc.identity_field(shape), Fbar, UNIAXIAL,
                                                           np.zeros(9), 1e-13)
    assert st == 0 and outer >= 2
    L = K0 - 2 * mu0 / 3
    E11 = 0.5 * (lam ** 2 - 1)
    E22 = -L * E11 / (2 * (L + mu0))
    t = np.sqrt(1 + 2 * E22)
    ref = np.diag([lam, t, t]).reshape(9)
    assert np.max(np.abs(Fb - ref)) < 1e-12
    assert np.max(np.abs(F - ref[:, None, None, None])) < 1e-12
    S11 = L * (E11 + 2 * E22) + 2 * mu0 * E11
    assert abs(Pb[0] - lam * S11) < 1e-13
    assert np.max(np.abs(Pb[[1, 2, 3, 4, 5, 6, 7, 8]])) < 1e-13


def test_homogeneous_macro_tangent_is_local_tangent(orc):
    shape = (4, 5, 3)
    Fbar = np.array([[1.02, 0.03, -0.01], [0.01, 0.98, 0.02], [0.0, 0.01, 1.01]]).reshape(9)
    F = np.broadcast_to(Fbar[:, None, None, None], (9,) + shape).copy()
    st, C = orc.macro_tangent(ms.K_SOFT, ms.MU_SOFT, F)
    assert st == 0
    for m in range(9):
        E = np.zeros(9)
        E[m] = 1.0
        col = orc.svk_tangent(F[:, :1, :1, :1], ms.K_SOFT, ms.MU_SOFT, E[:, None, None, None]).reshape(9)
        assert np.max(np.abs(C[:, m] - col)) < 1e-14


def _cell(shape, seed):
    rng = np.random.default_rng(seed)
    ph = (rng.random(shape) < 0.35).astype(np.uint8)
    return ms.phase_moduli(ph, TABLE)


@pytest.mark.parametrize("shape", [(7, 7, 7), (6, 8, 5)])
def test_macro_tangent_finite_differences_and_symmetry(orc, shape):
    K, mu = _cell(shape, 11)
    Fbar = np.array([[1.03, 0.02, 0.0], [0.01, 0.99, 0.02], [0.0, -0.01, 1.01]]).reshape(9)
    st, F, _, Pb, _ = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-12, 1e-13)
    assert st == 0
    st, C = orc.macro_tangent(K, mu, F, eta_cg=1e-13)
    assert st == 0
    h = 1e-5
    for m in range(9):
        d = np.zeros(9)
        d[m] = h
        sp, _, _, Pp, _ = orc.solve_increment(K, mu, F, Fbar + d, 1e-13, 1e-13)
        sm, _, _, Pm, _ = orc.solve_increment(K, mu, F, Fbar - d, 1e-13, 1e-13)
        assert sp == sm == 0
        fd = (Pp - Pm) / (2 * h)
        assert np.max(np.abs(C[:, m] - fd)) < 1e-7 * np.max(np.abs(C)), m
    assert np.max(np.abs(C - C.T)) < 1e-10 * np.max(np.abs(C))


@pytest.mark.parametrize("mask", [UNIAXIAL, np.array([0, 1, 0, 1, 0, 0, 0, 0, 0]), np.ones(9, int)])
def test_round_trip_mixed_control(orc, mask):
    shape = (7, 6, 8)
    K, mu = _cell(shape, 5)
    Fstar = np.array([[1.04, 0.02, 0.01], [-0.01, 0.985, 0.015], [0.005, 0.01, 0.99]]).reshape(9)
    st, Fs, Ps, Pbs, _ = orc.solve_increment(K, mu, orc.identity_field(shape), Fstar, 1e-12, 1e-13)
    assert st == 0
    guess = Fstar.copy()
    if mask.all():  # full stress control: start from a stressed guess (see below)
        guess += 0.004 * np.array([1, -1, 0.5, 0.5, 1, -0.5, 0, 1, -1])
    else:
        guess[mask != 0] = np.eye(3).reshape(9)[mask != 0]
    st, F, P, Pb, Fb, S, outer = orc.solve_increment_mixed(K, mu, orc.identity_field(shape), guess, mask, Pbs,
                                                           1e-13, 20, 1e-12, 1e-13)
    assert st == 0 and 2 <= outer <= 8
    assert np.max(np.abs(Fb - Fstar)) < 1e-10
    assert np.max(np.abs(F - Fs)) < 1e-9
    assert np.max(np.abs(Pb[mask != 0] - Pbs[mask != 0])) <= 1e-13


def test_round_trip_mixed_control_j2(orc):
    shape = (6, 6, 6)
    ph = ms.cubic_inclusion(6, 2)
    K = np.full(shape, 0.833)
    mu = np.full(shape, 0.386)
    ty0 = np.where(ph == 1, 0.006, 0.003)
    H = np.full(shape, 0.01)
    h0 = orc.virgin_history(shape)
    Fstar = np.array([[1.012, 0.004, 0.0], [0.0, 0.995, 0.0], [0.0, 0.0, 0.996]]).reshape(9)
    st, Fs, Ps, Pbs, hs, _ = orc.solve_increment_j2(K, mu, ty0, H, h0, orc.identity_field(shape), Fstar,
                                                    1e-12, 1e-13)
    assert st == 0 and np.max(hs[6]) > 0  # yielded somewhere
    guess = Fstar.copy()
    guess[UNIAXIAL != 0] = np.eye(3).reshape(9)[UNIAXIAL != 0]
    st, F, P, Pb, Fb, hn, S, outer = orc.solve_increment_mixed_j2(K, mu, ty0, H, h0, orc.identity_field(shape),
                                                                  guess, UNIAXIAL, Pbs, 1e-13, 20, 1e-12, 1e-13)
    assert st == 0
    assert np.max(np.abs(Fb - Fstar)) < 1e-9
    assert np.max(np.abs(F - Fs)) < 1e-8
    assert np.max(np.abs(hn - hs)) < 1e-8


def test_full_stress_control_from_zero_stress_is_singular(orc):
    # at F = I the stress is zero and rigid rotations of Fbar change no stress:
    # the masked tangent block is singular, reported as an invalid request
    shape = (5, 5, 5)
    K, mu = _cell(shape, 3)
    Pt = np.array([0.02, 0.0, 0.0, 0.0, -0.01, 0.0, 0.0, 0.0, 0.0])
    st, F, *_ = orc.solve_increment_mixed(K, mu, orc.identity_field(shape), np.eye(3).reshape(9),
                                          np.ones(9, int), Pt, 1e-13)
    assert st == 5 and np.array_equal(F, orc.identity_field(shape))


def test_mixed_control_outer_limit_leaves_state(orc):
    shape = (5, 5, 5)
    K, mu = _cell(shape, 3)
    Fbar = np.eye(3).reshape(9).copy()
    Fbar[0] = 1.05
    F0 = orc.identity_field(shape)
    st, F, *_ = orc.solve_increment_mixed(K, mu, F0, Fbar, UNIAXIAL, np.zeros(9), 1e-13, 1)
    assert st == 3 and np.array_equal(F, F0)
