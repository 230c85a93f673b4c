"""Pins of the plane-strain reading of the paper's 2-D example (Sec. 5).

The 2-D plane-strain problem is run as a 3-D cell with a few layers along a2
through which nothing varies.  What fixes that this is the 2-D problem:
* with one layer the oracle's transforms along a2 are the identity and xi_2 = 0,
  i.e. the 2-D method itself; two and three layers (even and odd, so that the
  a2 Nyquist choice plays no part) give the same fields to round-off;
* the out-of-plane components stay F13 = F23 = F31 = F32 = 0, F33 = 1 and every
  field stays constant along a2 (plane strain), while P33 is not zero;
* J2 (Sec. 5) through a yield point, the paper's pure-shear load.
"""
import numpy as np

from paper_1603_08893_amd import microstructure as ms


def _solve(orc, ph2, layers, chi, lams):
    shape = ph2.shape + (layers,)
    ph = np.repeat(ph2[:, :, None], layers, axis=2)
    tab = ms.plane_strain_j2_table(chi)
    K = np.choose(ph, [tab[0][0], tab[1][0]]).astype(float)
    mu = np.choose(ph, [tab[0][1], tab[1][1]]).astype(float)
    ty0 = np.choose(ph, [tab[0][2], tab[1][2]]).astype(float)
    H = np.choose(ph, [tab[0][3], tab[1][3]]).astype(float)
    h = orc.virgin_history(shape)
    F = orc.identity_field(shape)
    out = []
    for lam in lams:
        st, F, P, Pb, h, S = orc.solve_increment_j2(K, mu, ty0, H, h, F, ms.pure_shear(lam), 1e-10, 1e-12)
        assert st == 0
        out.append((F.copy(), P.copy(), Pb.copy(), h.copy(), S["n_solves"]))
    return out


def test_plane_strain_layers_agree(orc):
    ph2 = ms.micrograph_2d(N=9, ell=1.5, frac=0.3, seed=3, layers=1)[:, :7, 0]
    lams = [1.004, 1.008, 1.012, 1.02]  # elastic, around yield, plastic
    runs = {L: _solve(orc, ph2, L, 2.0, lams) for L in (1, 2, 3)}
    ref = runs[1]
    assert np.max(ref[-1][3][6]) > 0  # plastic by the last increment
    for L in (2, 3):
        for (F, P, Pb, h, ns), (F1, P1, Pb1, h1, ns1) in zip(runs[L], ref):
            assert ns == ns1
            assert np.max(np.abs(F - F1[:, :, :, :1])) < 1e-11
            assert np.max(np.abs(h - h1[:, :, :, :1])) < 1e-11
            assert np.max(np.abs(Pb - Pb1)) < 1e-12
    for L in (1, 2, 3):
        F, P, Pb, h, _ = runs[L][-1]
        for c in (2, 5, 6, 7):  # F13 F23 F31 F32
            assert np.max(np.abs(F[c])) < 1e-14
        assert np.max(np.abs(F[8] - 1.0)) < 1e-14
        assert np.max(np.abs(F - F[:, :, :, :1])) < 1e-13  # constant through the layers (to round-off)
        assert np.min(np.abs(P[8])) > 1e-6  # out-of-plane stress of plane strain
