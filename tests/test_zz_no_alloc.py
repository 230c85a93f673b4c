"""The projection entry point that allocates nothing (fftnk_project_noalloc)
against the context's projection (fftnk_project), through the C-ABI.

Two calls in a row on one GPU, the second on a smaller cell (so the shared
scratch buffer is re-planned and holds the previous call's contents), in both
precisions: the results equal the context's bitwise (same kernels, same plan)
and the oracle's projection to the parity bar.  A cell beyond the buffer is
refused with FFTNK_ENOMEM and leaves the next call working.
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


def _context_projection(shape, a, prec):
    from paper_1603_08893_amd.fftnk import Solver
    s = Solver(shape, precision=prec)
    s.set_phases(np.zeros(shape, dtype=np.uint8))
    s.set_material([(1.0, 1.0)])
    return s.project(a)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 5e-6)])
def test_noalloc_matches_context_projection(torch_cuda, orc, prec, tol):
    torch = torch_cuda
    from paper_1603_08893_amd import fftnk
    dt = torch.float64 if prec == "fp64" else torch.float32
    for shape in ((48, 40, 36), (17, 12, 10)):  # the second call on a smaller cell
        print("noalloc project", prec, shape, flush=True)
        A = ms.random_field(shape, seed=sum(shape))
        a = torch.from_numpy(A.reshape(-1)).to("cuda", dt)
        got = fftnk.project_noalloc(a, shape)
        ref = _context_projection(shape, a, prec)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        o = orc.project(A)
        g = got.double().cpu().numpy()
        assert np.linalg.norm(g - o.reshape(-1)) <= tol * np.linalg.norm(o)


def test_noalloc_refuses_oversized_cell(torch_cuda):
    torch = torch_cuda
    from paper_1603_08893_amd import fftnk
    big = (128, 128, 128)  # FP64 spectrum 151 MB > the 64 MiB buffer
    print("noalloc oversized", big, flush=True)
    a = torch.zeros(9 * 128 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(fftnk.FftnkError) as e:
        fftnk.project_noalloc(a, big)
    assert e.value.status == fftnk.ENOMEM
    shape = (9, 8, 12)
    A = ms.random_field(shape, seed=3)
    b = torch.from_numpy(A.reshape(-1)).cuda()
    got = fftnk.project_noalloc(b, shape)
    assert torch.equal(got, _context_projection(shape, b, "fp64"))
