"""The windowed update of the CG iterate (FFTNK_OPT_X_WINDOW): the steps
alpha_j p_j of W iterations are added to x together, in the order of j, by the
first pass of every iteration k with k mod W = 0 and by the finishing kernel.
The same floating-point operations in the same order as the update at every
iteration (W = 1), so every result must be bitwise equal across W: Newton and
CG counts, P-bar, F and P, in FP64 and FP32-mixed, on a single cell, on a batch
whose cells stop at different iterations, with the fixed-coefficient Krylov
methods (Chebyshev, Richardson), through the adjoint solve, and when the CG
breaks down (the iteration's own direction is then not applied).
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


def _solve(dims, prec, W, phase, Fbar, krylov=None, nyq=0):
    from paper_1603_08893_amd.fftnk import OPT_NYQUIST, Solver
    s = Solver(dims, precision=prec, x_window=W)
    assert s.x_window == W
    s.set_phases(phase)
    s.set_material(TABLE)
    if nyq:
        s.set_option(OPT_NYQUIST, 1)
    if krylov:
        s.set_krylov(krylov, table=TABLE)
    st, F, P, Pbar, S = s.solve_increment(Fbar, raise_on_error=False)
    return s, st, F.cpu().numpy(), P.cpu().numpy(), Pbar, S


def _same(a, b, tag):
    sa, sb = a[1:], b[1:]
    assert sa[0] == sb[0], tag
    assert [x["cg_iters"] for x in sa[4]] == [x["cg_iters"] for x in sb[4]], tag
    assert [x["n_solves"] for x in sa[4]] == [x["n_solves"] for x in sb[4]], tag
    for i in (1, 2, 3):
        assert np.array_equal(sa[i], sb[i]), (tag, i)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_cell_bitwise_equal_across_windows(torch_cuda, prec):
    shape = (24, 20, 16)
    ph = ms.grf_threshold(24, ell=4.0, frac=0.3, seed=7)[:, :20, :16].copy()
    print("x window single cell", prec, flush=True)
    ref = _solve(shape, prec, 1, ph, TENSION)
    assert ref[1] == 0 and max(max(x["cg_iters"]) for x in ref[5]) > 16  # several windows of 8
    for W in (2, 3, 8):
        _same(ref, _solve(shape, prec, W, ph, TENSION), (prec, W))


def test_batch_cells_stop_at_different_iterations(torch_cuda):
    dims = [(16, 16, 16), (12, 10, 8), (20, 18, 14)]
    rng = np.random.default_rng(5)
    phases = [rng.integers(0, 2, size=d).astype(np.uint8) for d in dims]
    ph = np.concatenate([p.reshape(-1) for p in phases])
    Fb = np.stack([TENSION, ms.simple_shear(0.04), np.diag([1.02, 0.99, 1.0]).reshape(9)])
    print("x window batch", flush=True)
    ref = _solve(dims, "fp64", 1, ph, Fb)
    iters = [x["cg_iters"] for x in ref[5]]
    assert len({tuple(v) for v in iters}) > 1
    _same(ref, _solve(dims, "fp64", 8, ph, Fb), "batch W=8")
    _same(ref, _solve(dims, "fp64", 5, ph, Fb), "batch W=5")


@pytest.mark.parametrize("method", ["chebyshev", "richardson"])
def test_fixed_coefficient_methods(torch_cuda, method):
    shape = (12, 12, 12)
    ph = np.random.default_rng(3).integers(0, 2, size=shape).astype(np.uint8)
    print("x window", method, flush=True)
    ref = _solve(shape, "fp64", 1, ph, ms.simple_shear(0.03), krylov=method)
    assert ref[1] == 0
    _same(ref, _solve(shape, "fp64", 8, ph, ms.simple_shear(0.03), krylov=method), method)


def test_adjoint_bitwise_equal(torch_cuda):
    shape = (16, 16, 16)
    mu = ms.lognormal_field(16, 0.5, 4.0, seed=11)
    out = []
    print("x window adjoint", flush=True)
    for W in (1, 8):
        torch = torch_cuda
        from paper_1603_08893_amd.fftnk import Solver
        s = Solver(shape, precision="fp64", x_window=W)
        s.set_phases(np.zeros(shape, dtype=np.uint8))
        s.set_material([(ms.K_SOFT, ms.MU_SOFT)])
        s.set_modulus_field(torch.from_numpy(mu.reshape(-1)).cuda())
        s.solve_increment(TENSION, fields=False)
        dmu, _, st = s.adjoint(np.ones(9))
        out.append((dmu.cpu().numpy(), st[0]["cg_iters"]))
    assert out[0][1] == out[1][1] and out[0][1][0] > 8
    assert np.array_equal(out[0][0], out[1][0])


def test_breakdown_leaves_state_and_matches(torch_cuda):
    from paper_1603_08893_amd import fftnk
    shape = (8, 8, 8)
    ph = np.random.default_rng(2).integers(0, 2, size=shape).astype(np.uint8)
    print("x window breakdown", flush=True)
    res = []
    for W in (1, 8):
        s, st, F, P, Pbar, S = _solve(shape, "fp64", W, ph, ms.simple_shear(0.05), nyq=1)
        assert st == fftnk.ECG_BREAKDOWN
        res.append((S[0]["cg_iters"], s.get_state().cpu().numpy()))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])
