"""Plan policies and the autotuner on the GPU.

* Every distinct plan policy (engines per axis, pencils per column
  work-group, grid lines per a2 work-group; fftnk_set_plan) computes the same
  projection and operator: parity with the oracle at the usual tolerances
  (FP64 1e-13, FP32 5e-6), switching policies on one bound context.  Shapes
  cover the 8- and 12-point register engines, the LDS engine and a batch.
* The autotuner keeps a valid policy (single cells and a batch of cells on
  different engines), reports its time, caches it per
  process (a second context of the same sizes gets it without timing), and a
  solve under the tuned plan matches the oracle.
"""
import numpy as np
import pytest

from paper_1603_08893_amd import microstructure as ms
from tests.fieldcheck import assert_fields_close

pytestmark = pytest.mark.gpu

TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def distinct_policies(dims, prec):
    """One policy per distinct launch geometry (others launch the same tiles)."""
    from paper_1603_08893_amd import fftnk
    seen, out = set(), []
    for pol in range(64):
        if (pol >> 3) & 3 == 3:
            continue
        try:
            d = fftnk.describe(dims, prec, policy=pol)
        except fftnk.FftnkError:
            continue
        key = tuple((tuple(a["reg"] for a in c["axes"]), c["rt"], c["rt1"],
                     (c["m64"], c["m32"]) if min(c["axes"][0]["reg"], c["axes"][1]["reg"]) == 0 else None)
                    for c in d["cells"])
        if key not in seen:
            seen.add(key)
            out.append(pol)
    return out


CASES = [[(16, 16, 16)], [(24, 20, 12)], [(31, 9, 7)], [(16, 12, 8), (9, 7, 5)]]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 5e-6)])
@pytest.mark.parametrize("dims", CASES, ids=lambda d: "+".join("x".join(map(str, s)) for s in d))
def test_every_policy_matches_oracle(torch_cuda, orc, dims, prec, tol):
    torch = torch_cuda
    from paper_1603_08893_amd.fftnk import Solver
    pols = distinct_policies(dims, prec)
    print("plans", dims, prec, pols, flush=True)
    assert len(pols) >= 2
    rng = np.random.default_rng(3)
    phs = [rng.integers(0, 2, size=d).astype(np.uint8) for d in dims]
    Fs = [ms.near_identity_field(d, seed=5 + r, scale=0.05) for r, d in enumerate(dims)]
    As = [ms.random_field(d, seed=11 + r) for r, d in enumerate(dims)]
    refG = [orc.project(A) for A in As]
    refA = []
    for d, ph, F, A in zip(dims, phs, Fs, As):
        K, mu = ms.phase_moduli(ph, TABLE)
        refA.append(orc.apply_operator(F, K, mu, A))
    s = Solver(dims if len(dims) > 1 else dims[0], precision=prec)
    s.set_phases(np.concatenate([ph.reshape(-1) for ph in phs]))
    s.set_material(TABLE)
    # batched fields: each cell's [9][n] block after the previous cells' blocks
    s.set_linearization(torch.from_numpy(np.concatenate([F.reshape(-1) for F in Fs])))
    A = torch.from_numpy(np.concatenate([a.reshape(-1) for a in As]))
    offs = np.cumsum([0] + [9 * int(np.prod(d)) for d in dims])
    for pol in pols:
        s.set_plan(pol)
        G = s.project(A).double().cpu().numpy()
        Ap = s.apply_operator(A).double().cpu().numpy()
        for r in range(len(dims)):
            assert_fields_close(G[offs[r]:offs[r + 1]], refG[r], tol, (pol, r))
            assert_fields_close(Ap[offs[r]:offs[r + 1]], refA[r], tol, (pol, r))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_cache_and_solve(torch_cuda, orc, prec):
    from paper_1603_08893_amd.fftnk import Solver
    from paper_1603_08893_amd import fftnk
    shape = (24, 24, 16)
    print("autotune", shape, prec, flush=True)
    ph = ms.cubic_inclusion(24, 9)[:, :, :16].copy()
    s = Solver(shape, precision=prec)
    s.set_phases(ph)
    s.set_material(TABLE)
    pol, t = s.autotune(reps=3, use_cache=False)
    print("policy", pol, "ms", t, flush=True)
    assert pol in distinct_policies([shape], prec) or fftnk.describe(shape, prec, policy=pol)["policy"] == pol
    assert 0.0 < t < 1e3
    # a second context of the same sizes takes the cached choice without timing
    s2 = Solver(shape, precision=prec)
    s2.set_phases(ph)
    s2.set_material(TABLE)
    pol2, t2 = s2.autotune(reps=3, use_cache=True)
    assert pol2 == pol and t2 == -1.0
    # a solve under the tuned plan
    K, mu = ms.phase_moduli(ph, TABLE)
    Fbar = ms.simple_shear(0.05)
    st, Fo, Po, Pbo, So = orc.solve_increment(K, mu, orc.identity_field(shape), Fbar, 1e-8, 1e-10)
    stg, F, P, Pb, S = s.solve_increment(Fbar, 1e-8, 1e-10)
    assert st == 0 and stg == 0
    bar = 1e-10 if prec == "fp64" else 1e-5
    assert np.max(np.abs(Pb[0] - Pbo)) <= bar * np.max(np.abs(Pbo))


def test_plan_errors(torch_cuda):
    from paper_1603_08893_amd import fftnk
    s = fftnk.Solver((8, 8, 8), precision="fp64")
    for bad in (24, 64, 1000):  # s = 3 is invalid; codes stop at 63
        with pytest.raises(fftnk.FftnkError):
            s.set_plan(bad)
    with pytest.raises(fftnk.FftnkError):
        s.autotune(reps=3)  # no phases or material yet
    s.set_phases(np.zeros((8, 8, 8), dtype=np.uint8))
    s.set_material([(1.0, 1.0)])
    with pytest.raises(fftnk.FftnkError):
        s.autotune(reps=0)


def test_autotune_batched_cells(torch_cuda, orc):
    """The tuner on a batch of cells with different engines: a valid policy
    for the batch, and each cell's increment under it matches the oracle."""
    from paper_1603_08893_amd.fftnk import Solver
    dims = [(16, 12, 8), (9, 7, 5), (24, 24, 12)]
    print("autotune batched", dims, flush=True)
    rng = np.random.default_rng(21)
    phs = [(rng.random(d) < 0.3).astype(np.uint8) for d in dims]
    s = Solver(dims, precision="fp64")
    s.set_phases(np.concatenate([ph.reshape(-1) for ph in phs]))
    s.set_material(TABLE)
    pol, t = s.autotune(reps=2, use_cache=False)
    assert pol in distinct_policies(dims, "fp64") and t > 0.0
    Fbar = ms.simple_shear(0.03)
    st, F, P, Pb, S = s.solve_increment(np.stack([Fbar] * len(dims)), 1e-8, 1e-10)
    assert st == 0
    for r, (d, ph) in enumerate(zip(dims, phs)):
        K, mu = ms.phase_moduli(ph, TABLE)
        sto, Fo, Po, Pbo, So = orc.solve_increment(K, mu, orc.identity_field(d), Fbar, 1e-8, 1e-10)
        assert sto == 0 and S[r]["n_solves"] == So["n_solves"]
        assert np.max(np.abs(Pb[r] - Pbo)) <= 1e-10 * np.max(np.abs(Pbo))
