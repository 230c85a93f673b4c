"""Odd against even grids (App. C): the appendix closes by noting that on an
even grid, one pixel larger along each axis than the odd one, the results of the
2-D example were practically identical, with G-hat set to zero at Nyquist
frequencies (compatible F); the other choice, identity there (equilibrated
stress), is the alternative it describes.

Each grid and choice is first checked against the oracle on the same cell
(equal Newton counts, P-bar within 1e-10 relative), then the odd/even
differences are measured:

* the paper's cubic inclusion (Sec. 4.4) on 31^3 and on 32^3 with the same 9^3
  cube, simple shear 0.05: the zero choice converges on both grids; with the
  identity choice the shear step makes the operator indefinite and CG breaks
  down on the GPU and in the oracle alike (a finding of this build, recorded
  here as a pin);
* the same cells under a tensile load, where all three runs converge;
* the 2-D plane-strain example's set-up (J2, chi = 2, pure shear through yield)
  on a 51 x 51 stand-in micrograph and its 52 x 52 extension.

The bounds on the odd/even differences (1 % of |P-bar|) are what "practically
identical" is taken to mean; the measured values are printed.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms

pytestmark = pytest.mark.gpu

TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]
TENSION = np.array([[1.03, 0.004, 0.0], [0.002, 1.02, 0.003], [0.0, -0.002, 1.025]]).reshape(9)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _relmax(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def _svk_pair(orc, N, Fbar, nyq):
    """GPU and oracle solves of the cubic-inclusion cell on N^3."""
    from paper_1603_08893_amd.fftnk import OPT_NYQUIST, Solver
    ph = ms.cubic_inclusion(N, 9)
    K, mu = ms.phase_moduli(ph, TABLE)
    so, _, _, Pbo, So = orc.solve_increment(K, mu, orc.identity_field(ph.shape), Fbar, nyq_identity=bool(nyq))
    s = Solver(ph.shape, precision="fp64")
    s.set_phases(ph)
    s.set_material(TABLE)
    s.set_option(OPT_NYQUIST, nyq)
    sg, _, _, Pb, S = s.solve_increment(Fbar, fields=False, raise_on_error=False)
    return sg, Pb[0], S[0], so, Pbo, So


@pytest.mark.parametrize("load", ["shear", "tension"])
def test_cubic_inclusion_odd_even(torch_cuda, orc, load):
    from paper_1603_08893_amd.fftnk import ECG_BREAKDOWN
    Fbar = ms.simple_shear(0.05) if load == "shear" else TENSION
    res = {}
    for N, nyq in ((31, 0), (32, 0), (32, 1)):
        print("odd/even", load, N, "identity" if nyq else "zero", flush=True)
        sg, Pb, S, so, Pbo, So = _svk_pair(orc, N, Fbar, nyq)
        if load == "shear" and nyq == 1:
            # indefinite operator: both sides stop with a CG breakdown
            assert so == 2 and sg == ECG_BREAKDOWN, (so, sg)
            continue
        assert so == 0 and sg == 0
        assert S["n_solves"] == So["n_solves"]
        if nyq == 0:  # the identity choice's nearly singular operator takes 2-3x the iterations
            assert all(abs(a - b) <= 2 for a, b in zip(S["cg_iters"], So["cg_iters"]))
        assert _relmax(Pb, Pbo) <= 1e-10
        res[(N, nyq)] = Pb
    d_zero = _relmax(res[(32, 0)], res[(31, 0)])
    print("P-bar odd 31^3 vs even 32^3 (zero at Nyquist): %.3e" % d_zero, flush=True)
    assert d_zero <= 1e-2
    if (32, 1) in res:
        d_id = _relmax(res[(32, 1)], res[(31, 0)])
        d_choice = _relmax(res[(32, 1)], res[(32, 0)])
        print("odd vs even identity: %.3e; the two even choices: %.3e" % (d_id, d_choice), flush=True)
        assert d_id <= 1e-2 and d_choice <= 1e-2


def test_plane_strain_odd_even(torch_cuda, orc):
    from paper_1603_08893_amd import fftnk
    odd = ms.micrograph_2d(N=51, ell=3.0, frac=0.3, seed=1701)
    even = ms.extend_by_one_pixel(odd, axes=(0, 1))
    assert even.shape == (52, 52, 2)
    tab = ms.plane_strain_j2_table(2.0)
    sched = ms.pure_shear_schedule(250, 1.2)[:8]  # through yield (lambda 1.0064)
    pbars = {}
    for ph in (odd, even):
        shape = ph.shape
        print("plane strain odd/even", shape, flush=True)
        t = np.asarray(tab)
        K, mu, ty0, H = (t[ph, k].copy() for k in range(4))
        s = fftnk.Solver(shape, precision="fp64")
        s.set_phases(ph)
        s.set_material(tab, model=fftnk.J2)
        F = orc.identity_field(shape)
        h = orc.virgin_history(shape)
        traj = []
        for Fb in sched:
            st, F, _, Pbo, h, So = orc.solve_increment_j2(K, mu, ty0, H, h, F, Fb)
            assert st == 0
            sg, _, _, Pb, S = s.solve_increment(Fb, fields=False)
            assert S[0]["n_solves"] == So["n_solves"]
            assert _relmax(Pb[0], Pbo) <= 1e-10
            traj.append(Pb[0].copy())
        assert np.max(h[6]) > 0  # yielded
        pbars[shape[0]] = np.array(traj)
    d = max(_relmax(a, b) for a, b in zip(pbars[52], pbars[51]))
    print("plane strain P-bar odd 51^2 vs even 52^2, largest over 8 increments: %.3e" % d, flush=True)
    assert d <= 1e-2
