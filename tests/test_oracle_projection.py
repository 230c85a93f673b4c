"""Pins of the oracle's compatibility projection G (Sec. 2.3, 2.5; App. C, D).

G must be the orthogonal projector onto the zero-mean compatible fields: every
row of G(A) is a gradient (App. D).  The decisive pin builds that projector by
brute force, without the closed form of G-hat: the spectral gradient operator
B : u -> grad u is assembled column by column on a tiny grid and the projector
onto its range is B B^+ (numpy pseudo-inverse).  On an even axis the fields with
Nyquist content are removed from the domain of B (the App. C choice that keeps F
compatible).  Invariants: idempotence, self-adjointness (Sec. 2.3), the
zero-mean property (Sec. 2.5), curl-free rows (App. D) and preservation of a
one-dimensional laminate field.
"""
import numpy as np
import pytest


def _xi(shape):
    # physical wave numbers (cycles per voxel) of each axis, Nyquist -> 0
    out = []
    for n in shape:
        k = np.fft.fftfreq(n) * n
        if n % 2 == 0:
            k[n // 2] = 0.0
        out.append(k / n)
    return out


def _nyquist_mask(shape):
    m = np.zeros(shape, dtype=bool)
    for ax, n in enumerate(shape):
        if n % 2 == 0:
            sl = [slice(None)] * 3
            sl[ax] = n // 2
            m[tuple(sl)] = True
    return m


def _grad_matrix(shape):
    """Dense B (9n x 3n): (grad u)_ij = d u_i / d X_j, spectral derivatives,
    restricted to u without Nyquist content."""
    n = int(np.prod(shape))
    xi = _xi(shape)
    ny = _nyquist_mask(shape)
    cols = []
    for comp in range(3):
        for v in range(n):
            u = np.zeros((3, n))
            u[comp, v] = 1.0
            U = np.fft.fftn(u.reshape((3,) + shape), axes=(1, 2, 3))
            U[:, ny] = 0.0
            g = np.zeros((3, 3) + shape)
            for i in range(3):
                for j in range(3):
                    kj = np.reshape(xi[j], [-1 if a == j else 1 for a in range(3)])
                    g[i, j] = np.real(np.fft.ifftn(2j * np.pi * kj * U[i]))
            cols.append(g.reshape(-1))
    return np.array(cols).T


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 4, 4), (3, 5, 4), (5, 3, 3)])
def test_projection_equals_bruteforce_projector(orc, shape):
    B = _grad_matrix(shape)
    Q = B @ np.linalg.pinv(B, rcond=1e-10)
    rng = np.random.default_rng(11)
    for _ in range(3):
        A = rng.standard_normal((9,) + shape)
        got = orc.project(A).reshape(-1)
        ref = Q @ A.reshape(-1)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), shape


@pytest.mark.parametrize("shape", [(5, 5, 5), (6, 6, 6), (7, 4, 5), (9, 9, 9), (8, 8, 8)])
def test_projection_invariants(orc, shape):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal((9,) + shape)
    B = rng.standard_normal((9,) + shape)
    GA = orc.project(A)
    GB = orc.project(B)
    scale = np.max(np.abs(GA))
    # idempotent
    assert np.max(np.abs(orc.project(GA) - GA)) < 1e-13 * scale
    # zero mean
    assert np.max(np.abs(GA.reshape(9, -1).mean(axis=1))) < 1e-15 * scale * 10
    # constants are annihilated
    C = np.ones((9,) + shape) * rng.standard_normal((9, 1, 1, 1))
    assert np.max(np.abs(orc.project(C))) < 1e-14
    # self-adjoint: <B, G A> = <G B, A>
    assert abs(np.sum(B * GA) - np.sum(GB * A)) < 1e-11 * abs(np.sum(B * GA)) + 1e-12
    # rows are curl free: xi x hat(row_i) = 0 at every frequency
    xi = np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij")
    H = np.fft.fftn(GA.reshape((3, 3) + shape), axes=(2, 3, 4))
    for i in range(3):
        a = H[i]
        curl = np.stack([xi[1] * a[2] - xi[2] * a[1], xi[2] * a[0] - xi[0] * a[2], xi[0] * a[1] - xi[1] * a[0]])
        assert np.max(np.abs(curl)) < 1e-11 * np.max(np.abs(a))


def test_projection_preserves_gradient_fields(orc):
    # G(grad u) = grad u for u without Nyquist content (odd grid: any u)
    shape = (7, 9, 5)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3,) + shape)
    xi = _xi(shape)
    U = np.fft.fftn(u, axes=(1, 2, 3))
    g = np.zeros((3, 3) + shape)
    for i in range(3):
        for j in range(3):
            kj = np.reshape(xi[j], [-1 if a == j else 1 for a in range(3)])
            g[i, j] = np.real(np.fft.ifftn(2j * np.pi * kj * U[i]))
    g = g.reshape((9,) + shape)
    assert np.max(np.abs(orc.project(g) - g)) < 1e-12 * np.max(np.abs(g))


@pytest.mark.parametrize("N", [9, 11])
def test_projection_laminate_field(orc, N):
    # a(x_d) (x) e_d is compatible: G returns it minus its mean (odd N)
    rng = np.random.default_rng(N)
    for d in range(3):
        a = rng.standard_normal((3, N))
        A = np.zeros((3, 3, N, N, N))
        for i in range(3):
            shp = [1, 1, 1]
            shp[d] = N
            A[i, d] = a[i].reshape(shp)
        A = A.reshape(9, N, N, N)
        ref = A - A.reshape(9, -1).mean(axis=1)[:, None, None, None]
        assert np.max(np.abs(orc.project(A) - ref)) < 1e-13


def test_projection_even_grid_kills_nyquist(orc):
    N = 8
    x = np.arange(N)
    A = np.zeros((9, N, N, N))
    A[3] = np.cos(np.pi * x)[:, None, None] * np.cos(2 * np.pi * x / N)[None, :, None]
    assert np.max(np.abs(orc.project(A))) < 1e-14
