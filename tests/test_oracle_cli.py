"""The oracle's .npy command-line front end (python -m oracle) gives what the
in-process oracle gives, and the closed forms hold through it: G is idempotent,
a homogeneous cell's increment leaves F = F-bar everywhere and P-bar equals
the St. Venant-Kirchhoff stress of F-bar (Sec. 4.2)."""
import json
import os
import subprocess
import sys

import numpy as np

from paper_1603_08893_amd import microstructure as ms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]


def _run(*args):
    out = subprocess.run([sys.executable, "-m", "oracle", *args], cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_project_and_operator(orc, tmp_path):
    shape = (7, 6, 5)
    A = ms.random_field(shape, seed=1)
    np.save(tmp_path / "A.npy", A)
    _run("project", "--in", str(tmp_path / "A.npy"), "--out", str(tmp_path / "G.npy"))
    G = np.load(tmp_path / "G.npy")
    assert np.array_equal(G, orc.project(A))
    _run("project", "--in", str(tmp_path / "G.npy"), "--out", str(tmp_path / "GG.npy"))
    assert np.max(np.abs(np.load(tmp_path / "GG.npy") - G)) <= 1e-13 * np.max(np.abs(G))
    ph = (np.random.default_rng(2).random(shape) < 0.3).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    F = ms.near_identity_field(shape, seed=3, scale=0.05)
    for name, a in (("F", F), ("K", K), ("mu", mu)):
        np.save(tmp_path / ("%s.npy" % name), a)
    _run("apply_operator", "--F", str(tmp_path / "F.npy"), "--K", str(tmp_path / "K.npy"), "--mu",
         str(tmp_path / "mu.npy"), "--in", str(tmp_path / "A.npy"), "--out", str(tmp_path / "Ap.npy"))
    assert np.array_equal(np.load(tmp_path / "Ap.npy"), orc.apply_operator(F, K, mu, A))


def test_homogeneous_increment_closed_form(orc, tmp_path):
    shape = (5, 5, 5)
    np.save(tmp_path / "Ft.npy", orc.identity_field(shape))
    Fbar = ms.simple_shear(0.05)
    rec = _run("solve_increment", "--F", str(tmp_path / "Ft.npy"), "--K-value", str(ms.K_SOFT), "--mu-value",
               str(ms.MU_SOFT), "--fbar", ",".join(repr(float(v)) for v in Fbar.reshape(-1)), "--out-F",
               str(tmp_path / "F.npy"))
    assert rec["status"] == 0
    F = np.load(tmp_path / "F.npy")
    assert np.max(np.abs(F.reshape(9, -1) - Fbar.reshape(9, 1))) <= 1e-14
    # P = F S, S = lambda tr(E) I + 2 mu E, E = (F^T F - I) / 2, lambda = K - 2 mu / 3
    Fm = Fbar.reshape(3, 3)
    E = 0.5 * (Fm.T @ Fm - np.eye(3))
    lam = ms.K_SOFT - 2.0 * ms.MU_SOFT / 3.0
    P = Fm @ (lam * np.trace(E) * np.eye(3) + 2.0 * ms.MU_SOFT * E)
    assert np.max(np.abs(np.array(rec["pbar"]) - P.reshape(-1))) <= 1e-14


def test_timing_front_end_small_grid():
    """python -m oracle.timing: pinned, built on the host with the timed flags,
    one JSON line with the per-application times and the host description."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-m", "oracle.timing", "--grid", "12", "--budget", "0.05", "--max-reps", "2"],
                       cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    d = json.loads([l for l in r.stdout.splitlines() if l.startswith("{")][-1])
    assert d["grid"] == 12 and 1 <= d["reps"] <= 2 and d["threads"] == 1
    assert d["sec_per_matvec"] > 0 and "-O3" in d["flags"] and d["cpu_model"]
