"""Every FFT plan the library builds, one axis at a time: projection parity
with the oracle (FP64, relative L2 <= 1e-13) for each length on each axis,
with small fixed lengths on the other two.

Lengths: all of 2..40 (every radix path and small prime), the 12-point
register engine's 3 * 2^k up to 192, the 8-point engine's powers of two up
to 256, primes and other lengths up to 256 (LDS engine), and on a0 / a1 the
LDS-engine lengths 257..512 (including 451 = 11 x 41 and 512).  Each case
uses one context; the oracle runs its own mixed-radix transforms.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms
from tests.fieldcheck import field_errors

pytestmark = pytest.mark.gpu

SMALL = list(range(2, 41))
REG = [48, 64, 96, 128, 192, 256]
OTHER = [97, 100, 125, 127, 162, 200, 243, 251, 255]
LONG = [257, 300, 384, 451, 509, 512]


def _cases():
    out = []
    for n in SMALL + REG + OTHER:
        out += [(n, 3, 4), (3, n, 4), (3, 4, n)]
    for n in LONG:
        out += [(n, 3, 2), (2, n, 3)]
    return out


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_every_length_on_every_axis(torch_cuda, orc):
    torch = torch_cuda
    from paper_1603_08893_amd.fftnk import Solver
    bad = []
    for shape in _cases():
        A = ms.random_field(shape, seed=sum(shape))
        ref = orc.project(A)
        s = Solver(shape, precision="fp64")
        s.set_phases(np.zeros(shape, dtype=np.uint8))
        s.set_material([(1.0, 1.0)])
        got = s.project(torch.from_numpy(A.reshape(-1))).cpu().numpy()
        l2, mx = field_errors(got, ref)
        if not (l2 <= 1e-13 and mx <= 2e-13):
            bad.append((shape, l2, mx))
        del s
    print("lengths checked:", len(_cases()), flush=True)
    assert not bad, bad
