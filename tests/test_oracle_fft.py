"""Pins of the oracle's discrete Fourier transforms.

The oracle's recursive mixed-radix FFT is checked against the definition of the
DFT (naive O(n^2) sums written independently in C and in numpy), against numpy's
own FFT library routine, and against identities the DFT must satisfy (delta ->
ones, Parseval, Hermitian symmetry of real input, inverse round trip).  The
3-D transform is the separable one of Sec. 3.3 (one 1-D transform per grid line
and axis).
"""
import numpy as np
import pytest


def _naive_numpy(x, sign=-1):
    n = x.size
    j = np.arange(n)
    W = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    return W @ x


@pytest.mark.parametrize("n", list(range(1, 41)) + [48, 64, 96, 128, 192])
def test_fft1d_vs_naive_definition(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = _naive_numpy(x)
    got = orc.fft1d(x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    # the C naive DFT agrees with the numpy one
    assert np.max(np.abs(orc.dft1d_naive(x) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [24, 31, 32, 48, 96, 128, 192, 256])
def test_fft1d_vs_numpy_library(orc, n):
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.allclose(orc.fft1d(x, -1), np.fft.fft(x), rtol=0, atol=1e-12)
    assert np.allclose(orc.fft1d(x, +1), np.fft.ifft(x) * n, rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 3, 3), (4, 5, 6), (5, 5, 5), (6, 4, 3), (7, 7, 7), (8, 8, 8),
                                   (1, 3, 4)])
def test_fft3d_vs_naive_3d_dft(orc, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = orc.dft3d_naive(x)
    got = orc.fft3d(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(ref - np.fft.fftn(x))) <= 1e-11 * np.max(np.abs(ref))


def test_fft3d_identities(orc):
    shape = (9, 8, 7)
    d = np.zeros(shape, dtype=complex)
    d[0, 0, 0] = 1.0
    assert np.max(np.abs(orc.fft3d(d) - 1.0)) < 1e-15  # delta -> all ones
    rng = np.random.default_rng(7)
    x = rng.standard_normal(shape)
    X = orc.fft3d(x)
    n = x.size
    # Parseval
    assert abs(np.sum(np.abs(X) ** 2) / n - np.sum(x ** 2)) < 1e-10 * np.sum(x ** 2)
    # real input -> Hermitian spectrum X(-k) = conj X(k)
    Xm = np.conj(np.roll(np.flip(X, axis=(0, 1, 2)), 1, axis=(0, 1, 2)))
    assert np.max(np.abs(X - Xm)) < 1e-12 * np.max(np.abs(X))
    # round trip (backward transform is unnormalised)
    back = orc.fft3d(X, +1) / n
    assert np.max(np.abs(back - x)) < 1e-13
