"""GPU adjoint sensitivity (dL/dmu of the homogenised stress) through the C-ABI
and the torch.autograd.Function, against the oracle's adjoint and against
central finite differences of the GPU forward solve (tight tolerances).

Inputs follow the adjoint workload: a log-normal shear-modulus field
mu = 0.386 exp(0.5 Z) with Z a standardised Gaussian random field (correlation
length 8 voxels) on 192^3, subsampled at stride 8 to 24^3; K = 0.833 uniform;
load cases of magnitude 0.05.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mu24():
    return np.ascontiguousarray(ms.lognormal_field(192, sigma=0.5, ell=8.0, seed=1605)[::8, ::8, ::8])


def _solver(shape, nrve, prec="fp64"):
    from paper_1603_08893_amd.fftnk import Solver
    s = Solver([shape] * nrve, precision=prec)
    s.set_phases(np.zeros(nrve * int(np.prod(shape)), dtype=np.uint8))
    s.set_material([(0.833, 0.386)])
    return s


def test_adjoint_matches_oracle_24(torch_cuda, orc, mu24):
    torch = torch_cuda
    shape = mu24.shape
    K = np.full(shape, 0.833)
    cases = ms.c5_load_cases()[:3] + ms.c5_load_cases()[5:6]
    rng = np.random.default_rng(1607)
    gs = rng.standard_normal((len(cases), 9))
    s = _solver(shape, len(cases))
    s.set_modulus_field(np.tile(mu24.reshape(-1), len(cases)))
    _, F, _, Pbar, _ = s.solve_increment(np.array(cases), 1e-12, 1e-13)
    dmu, dK, st = s.adjoint(gs, eta_cg=1e-13, want_K=True)
    dmu = dmu.view(len(cases), -1).cpu().numpy()
    dK = dK.view(len(cases), -1).cpu().numpy()
    for c, Fb in enumerate(cases):
        sto, Fo, Po, Pbo, So = orc.solve_increment(K, mu24, orc.identity_field(shape), Fb, 1e-12, 1e-13)
        assert np.max(np.abs(Pbar[c] - Pbo)) <= 1e-11 * np.max(np.abs(Pbo))
        sta, gmu, gK, it = orc.adjoint(K, mu24, Fo, gs[c], eta_cg=1e-13)
        assert sta == 0
        assert abs(st[c]["cg_iters"][0] - it) <= 2
        assert np.linalg.norm(dmu[c] - gmu.reshape(-1)) <= 1e-9 * np.linalg.norm(gmu)
        assert np.linalg.norm(dK[c] - gK.reshape(-1)) <= 1e-9 * np.linalg.norm(gK)


def test_autograd_function_vs_central_differences(torch_cuda, mu24):
    torch = torch_cuda
    from paper_1603_08893_amd.fftnk import homogenized_stress
    shape = mu24.shape
    cases = np.array(ms.c5_load_cases())
    s = _solver(shape, len(cases))
    mu = torch.from_numpy(mu24).cuda().requires_grad_(True)
    target = torch.from_numpy(np.random.default_rng(1606).standard_normal((len(cases), 9)) * 1e-3).cuda()

    def loss_of(m):
        P = homogenized_stress(m, s, cases, 1e-12, 1e-13)
        return ((P - target) ** 2).sum()

    L = loss_of(mu)
    L.backward()
    grad = mu.grad.detach().cpu().numpy()
    h = 1e-6
    rng = np.random.default_rng(1607)
    picks = [tuple(rng.integers(0, n) for n in shape) for _ in range(4)]
    with torch.no_grad():
        for v in picks:
            mp = mu.detach().clone()
            mm = mu.detach().clone()
            mp[v] += h
            mm[v] -= h
            fd = (loss_of(mp).item() - loss_of(mm).item()) / (2 * h)
            assert abs(fd - grad[v]) <= 1e-5 * abs(grad[v]) + 1e-13, (v, fd, grad[v])
        d = torch.from_numpy(rng.standard_normal(shape)).cuda()
        fd = (loss_of(mu.detach() + h * d).item() - loss_of(mu.detach() - h * d).item()) / (2 * h)
        assert abs(fd - float((mu.grad * d).sum())) <= 1e-6 * abs(fd)


def test_adjoint_fp32_mixed_close_to_fp64(torch_cuda, mu24):
    torch = torch_cuda
    shape = mu24.shape
    cases = np.array(ms.c5_load_cases()[:2])
    g = np.ones((2, 9))
    out = {}
    for prec in ["fp64", "fp32"]:
        s = _solver(shape, 2, prec)
        s.set_modulus_field(np.tile(mu24.reshape(-1), 2))
        s.solve_increment(cases, 1e-10, 1e-10)
        out[prec] = s.adjoint(g, eta_cg=1e-10)[0].cpu().numpy()
    assert np.linalg.norm(out["fp32"] - out["fp64"]) <= 1e-4 * np.linalg.norm(out["fp64"])


def test_backward_refuses_a_changed_state(torch_cuda, mu24):
    """A solve on the same Solver between forward and backward would move the
    equilibrium the adjoint is taken at: backward raises instead of returning
    a gradient of another state; a fresh forward works again."""
    torch = torch_cuda
    from paper_1603_08893_amd.fftnk import homogenized_stress
    shape = mu24.shape
    cases = np.array(ms.c5_load_cases()[:2])
    s = _solver(shape, len(cases))
    mu = torch.from_numpy(mu24).cuda().requires_grad_(True)
    L = homogenized_stress(mu, s, cases).sum()
    s.solve_increment(cases * 1.0 + 0.01 * np.eye(3).reshape(9), fields=False)  # another solve in between
    with pytest.raises(RuntimeError, match="state changed"):
        L.backward()
    L2 = homogenized_stress(mu, s, cases).sum()
    L2.backward()
    assert torch.isfinite(mu.grad).all()
