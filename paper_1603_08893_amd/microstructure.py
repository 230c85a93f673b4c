"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the homogenisation method: it only draws
phase maps, modulus fields, load schedules and random test fields.  Both the
HIP library and the CPU oracle consume what it produces.

Recipes (all numpy ``default_rng`` / PCG64 with the stated seeds):

* ``cubic_inclusion`` -- the paper's first example (Sec. 4.4): an N^3 cell with a
  9^3 stiff cube in one corner (a0, a2 in the last 9 planes, a1 in the first 9).
* ``grf_threshold`` -- white noise filtered by a periodic Gaussian
  exp(-2 pi^2 l^2 |k/N|^2) (correlation length l voxels), standardised; phase 1 is
  the top ``frac`` of voxels by rank (ties broken by linear index).
* ``rsa_spheres`` -- random sequential addition of non-overlapping periodic
  spheres, radius uniform in {rmin..rmax}, until a target volume fraction or an
  attempt budget is reached (the achieved fraction is returned).
* ``lognormal_field`` -- mu0 * exp(sigma * Z) with Z the standardised Gaussian
  random field above.
* ``laminate`` -- two phases alternating along one axis.
* ``micrograph_2d`` -- stand-in for the paper's thresholded 451 x 451 dual-phase
  micrograph (Sec. 5, not available): a 2-D Gaussian random field with the same
  periodic filter, thresholded at a hard-phase fraction, as an n x n x 2 plane-
  strain cell (constant through the two a2 layers).
* ``extend_by_one_pixel`` -- an odd grid turned into the next even one by one
  more pixel along the given axes (the periodic image continued by its first
  row), the odd/even comparison of the paper's appendix on even grids.
* ``pure_shear_schedule`` -- the paper's 2-D load, Fbar = l e_x e_x + e_y e_y / l
  (+ e_z e_z), l in equal steps to l_max.
"""
import numpy as np

# Phase moduli of the paper's first example: K = 0.833, mu = 0.386 for the
# matrix and ten times that for the inclusion (listing's parameters).
K_SOFT, MU_SOFT = 0.833, 0.386
K_HARD, MU_HARD = 8.33, 3.86


def cubic_inclusion(N=31, size=9):
    ph = np.zeros((N, N, N), dtype=np.uint8)
    ph[N - size:, :size, N - size:] = 1
    return ph


def gaussian_random_field(N, ell, seed):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N, N))
    k = np.fft.fftfreq(N)  # k / N in cycles per voxel
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    filt = np.exp(-2.0 * np.pi ** 2 * ell ** 2 * k2)
    z = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    z -= z.mean()
    z /= z.std()
    return z


def grf_threshold(N=128, ell=8.0, frac=0.3, seed=1603):
    z = gaussian_random_field(N, ell, seed)
    flat = z.reshape(-1)
    m = int(np.floor(frac * flat.size))
    # rank by value (descending), ties broken by linear index
    order = np.lexsort((np.arange(flat.size), -flat))
    ph = np.zeros(flat.size, dtype=np.uint8)
    ph[order[:m]] = 1
    return ph.reshape(N, N, N)


def micrograph_2d(N=451, ell=6.0, frac=0.3, seed=1701, layers=2):
    """Plane-strain stand-in microstructure: an (N, N, layers) phase map whose
    N x N section is a thresholded periodic 2-D Gaussian random field (phase 1,
    the hard phase, is the top ``frac`` of pixels by rank, ties by index)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N))
    k = np.fft.fftfreq(N)
    filt = np.exp(-2.0 * np.pi ** 2 * ell ** 2 * (k[:, None] ** 2 + k[None, :] ** 2))
    z = np.real(np.fft.ifft2(np.fft.fft2(w) * filt)).reshape(-1)
    m = int(np.floor(frac * z.size))
    order = np.lexsort((np.arange(z.size), -z))
    ph = np.zeros(z.size, dtype=np.uint8)
    ph[order[:m]] = 1
    return np.repeat(ph.reshape(N, N)[:, :, None], layers, axis=2)


def extend_by_one_pixel(ph, axes=(0, 1)):
    """The phase map with one more pixel along each of `axes`: the periodic
    image continued by its first row (index 0 repeated at index N)."""
    out = np.asarray(ph)
    for a in axes:
        out = np.concatenate([out, np.take(out, [0], axis=a)], axis=a)
    return np.ascontiguousarray(out)


def pure_shear(lam):
    """Fbar = lam e_x e_x + e_y e_y / lam + e_z e_z (plane-strain pure shear)."""
    return np.diag([lam, 1.0 / lam, 1.0]).reshape(9)


def pure_shear_schedule(n_incr=250, lam_max=1.2):
    return [pure_shear(1.0 + (lam_max - 1.0) * t / n_incr) for t in range(1, n_incr + 1)]


def plane_strain_j2_table(chi, E=1.0, nu=0.3):
    """J2 table of the 2-D example (Sec. 5): elastically homogeneous phases
    (K, mu from E, nu), soft tau_y0 = 0.003 E, H = 0.01 E, hard = chi x soft."""
    K = E / (3.0 * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return [(K, mu, 0.003 * E, 0.01 * E), (K, mu, 0.003 * E * chi, 0.01 * E * chi)]


def rsa_spheres(N, target_frac, seed, rmin=3, rmax=10, max_attempts=100000):
    """Random sequential addition of periodic spheres.  Returns (phase map,
    achieved volume fraction).

    Each attempt draws a radius U{rmin..rmax} and a centre U[0, N)^3, and is
    rejected if the periodic centre distance to any placed sphere is below the
    sum of the radii; a voxel (centre at index + 1/2) is inside a sphere if
    its periodic distance to the centre is at most the radius.  Stops at the
    target fraction or after max_attempts."""
    rng = np.random.default_rng(seed)
    centres = np.zeros((0, 3))
    radii = np.zeros(0)
    ph = np.zeros((N, N, N), dtype=np.uint8)
    filled = 0
    target = target_frac * N ** 3
    for _ in range(max_attempts):
        if filled >= target:
            break
        r = int(rng.integers(rmin, rmax + 1))
        c = rng.uniform(0.0, N, size=3)
        if len(radii):
            d = np.abs(centres - c)
            d = np.minimum(d, N - d)
            if np.any(np.sqrt((d ** 2).sum(axis=1)) < r + radii):
                continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        # voxels within the sphere's periodic bounding box (the whole axis if
        # the box would wrap onto itself)
        axes = []
        for a in range(3):
            if 2 * r + 3 >= N:
                ix = np.arange(N)
            else:
                ix = np.arange(int(np.floor(c[a] - r - 1)), int(np.ceil(c[a] + r + 1)) + 1) % N
            x = ix + 0.5
            axes.append((ix, np.minimum(np.abs(x - c[a]), N - np.abs(x - c[a]))))
        (i0, d0), (i1, d1), (i2, d2) = axes
        inside = (d0[:, None, None] ** 2 + d1[None, :, None] ** 2 + d2[None, None, :] ** 2) <= r * r
        box = ph[np.ix_(i0, i1, i2)]
        filled += int(np.count_nonzero(inside & (box == 0)))
        box[inside] = 1
        ph[np.ix_(i0, i1, i2)] = box
    return ph, float(ph.mean())


def lognormal_field(N=192, sigma=0.5, ell=8.0, seed=1605, mu0=MU_SOFT):
    return mu0 * np.exp(sigma * gaussian_random_field(N, ell, seed))


def laminate(shape, axis=0, frac=0.5):
    """Phase 1 on the first round(frac * N_axis) planes normal to ``axis``."""
    ph = np.zeros(shape, dtype=np.uint8)
    m = int(round(frac * shape[axis]))
    sl = [slice(None)] * 3
    sl[axis] = slice(0, m)
    ph[tuple(sl)] = 1
    return ph


def phase_moduli(phase, table):
    """Per-voxel (K, mu) arrays from a phase map and a [(K, mu), ...] table."""
    table = np.asarray(table, dtype=np.float64)
    return table[phase, 0].copy(), table[phase, 1].copy()


def random_field(shape, seed, scale=1.0):
    """A 9-component field of iid U(-scale, scale) entries."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(9,) + tuple(shape))


def near_identity_field(shape, seed, scale=0.01):
    """F = I + U(-scale, scale) per entry (not compatible; a linearisation point)."""
    F = random_field(shape, seed, scale)
    F[0] += 1.0
    F[4] += 1.0
    F[8] += 1.0
    return F


def tensor(A):
    return np.asarray(A, dtype=np.float64).reshape(9)


def simple_shear(gamma):
    """I + gamma e1 (x) e2 (Sec. 4.4 load)."""
    F = np.eye(3)
    F[0, 1] = gamma
    return F.reshape(9)


def isochoric_stretch(lam):
    """diag(lam, lam^-1/2, lam^-1/2)."""
    return np.diag([lam, lam ** -0.5, lam ** -0.5]).reshape(9)


def c2_schedule(n_incr=5):
    """Isochoric uniaxial stretch, lambda_t = 1 + 0.01 t, t = 1..n_incr."""
    return [isochoric_stretch(1.0 + 0.01 * t) for t in range(1, n_incr + 1)]


def c4_schedule(n_incr=20, gamma_max=0.1):
    return [simple_shear(gamma_max * t / n_incr) for t in range(1, n_incr + 1)]


def c5_load_cases(mag=0.05):
    """8 load cases: 3 uniaxial, 2 biaxial, 3 shear, magnitude 0.05."""
    out = []
    for i in range(3):
        F = np.eye(3)
        F[i, i] += mag
        out.append(F.reshape(9))
    for (i, j) in [(0, 1), (1, 2)]:
        F = np.eye(3)
        F[i, i] += mag
        F[j, j] += mag
        out.append(F.reshape(9))
    for (i, j) in [(0, 1), (1, 2), (2, 0)]:
        F = np.eye(3)
        F[i, j] += mag
        out.append(F.reshape(9))
    return out


def c3_cell(r, seed0=1603000, sizes=(32, 48, 64, 96), per_size=16):
    """Cell r of the 64-cell batch (see c3_batch)."""
    N = sizes[r // per_size]
    rng = np.random.default_rng(seed0 + r)
    target = rng.uniform(0.20, 0.40)
    chi = rng.uniform(5.0, 20.0)
    H = rng.uniform(-0.05, 0.05, size=(3, 3))
    ph, frac = rsa_spheres(N, target, seed=seed0 + r + 500000)
    return {
        "N": N,
        "phase": ph,
        "frac": frac,
        "table": [(K_SOFT, MU_SOFT), (chi * K_SOFT, chi * MU_SOFT)],
        "Fbar": (np.eye(3) + H).reshape(9),
    }


def c3_batch(seed0=1603000, sizes=(32, 48, 64, 96), per_size=16):
    """64 RVEs: sphere microstructures, per-RVE contrast and load.

    Returns a list of dicts with keys N, phase, frac, table, Fbar.
    """
    return [c3_cell(r, seed0, sizes, per_size) for r in range(len(sizes) * per_size)]
