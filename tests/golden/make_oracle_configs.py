"""Write the oracle's results for the benchmark configurations at full size.

    python tests/golden/make_oracle_configs.py {e1,c2,c3,c4,c5} [--increments K] [--checkpoint DIR]

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``paper_1603_08893_amd/microstructure.py``); nothing here touches the GPU or
the HIP library.  Each configuration goes to ``tests/golden/oracle_<name>.json``
(rewritten after every increment, ``"complete": true`` once the run finished):

* e1 -- the paper's cubic-inclusion example (Sec. 4.4): 31^3, 9^3 cube ten
  times stiffer, simple shear gamma = 1, one increment, eta_NW 1e-5, eta_CG 1e-8.
* c2 -- 128^3 two-phase Gaussian-random-field cell (30 %, ten-fold moduli),
  isochoric stretch lambda_t = 1 + 0.01 t in five increments.
* c3 -- the first cell of each size class (32, 48, 64, 96) of the 64-cell
  sphere batch (cells 0, 16, 32, 48), one increment each.
* c4 -- finite-strain J2 on 96^3 spheres (25 %), simple shear in steps of
  0.005, the first ``--increments`` increments (default 4: the matrix yields in
  the first, the spheres in the second).
* c5 -- 192^3 log-normal shear-modulus field (sigma 0.5, seed 1605), the first
  load case (uniaxial 0.05 along e1): the forward solve, the target solve on
  the seed-1606 field, and the adjoint for the cotangent 2 (Pbar - Pbar_target).

Per increment the file holds the status, the number of linear solves, the CG
iterations of each, P-bar (17 significant digits), and, after the last one,
F and P at 64 seeded sample voxels and the Frobenius norms of F - I and P over
the whole field; sha256 digests of the generated inputs let a consumer check
it regenerated the same cell.

With --checkpoint DIR the oracle's state (F, and the J2 history) is saved
there after every increment (outside the repository: the 192^3 field is half
a gigabyte), and a run that finds its own state there continues from the last
recorded increment of the existing file instead of starting over; the 64-cell
batch continues from the cells already recorded.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1603_08893_amd import microstructure as ms  # noqa: E402

TABLE = [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)]
ETA_NW, ETA_CG = 1e-5, 1e-8
N_SAMPLES = 64


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def sample_index(n, seed=7):
    return np.sort(np.random.default_rng(seed).choice(n, N_SAMPLES, replace=False))


def fl(a):
    return [float(v) for v in np.asarray(a).reshape(-1)]


def field_summary(F, P, idx):
    n = F.size // 9
    F2 = F.reshape(9, n)
    P2 = P.reshape(9, n)
    Fmi = F2.copy()
    Fmi[0] -= 1.0
    Fmi[4] -= 1.0
    Fmi[8] -= 1.0
    return {"sample_index": [int(i) for i in idx],
            "F_samples": [fl(F2[:, i]) for i in idx],
            "P_samples": [fl(P2[:, i]) for i in idx],
            "norm_F_minus_I": float(np.linalg.norm(Fmi)),
            "norm_P": float(np.linalg.norm(P2))}


def incr_record(status, Pbar, stats, sec):
    return {"status": int(status), "n_solves": int(stats["n_solves"]), "cg_iters": [int(v) for v in stats["cg_iters"]],
            "newton_res": fl(stats["newton_res"]), "Pbar": fl(Pbar), "seconds": round(sec, 2)}


class Out:
    def __init__(self, name, meta, resume=False):
        self.path = os.path.join(HERE, "oracle_%s.json" % name)
        old = None
        if resume and os.path.exists(self.path):
            old = json.load(open(self.path))
            for k in ("config", "phase_sha256", "mu_sha256"):
                if k in meta and old.get(k) != meta[k]:
                    old = None  # another configuration: start over
                    break
        self.doc = old if old is not None else dict(meta)
        self.resumed = old is not None
        self.doc["complete"] = False
        self.doc["oracle_build"] = "oracle.build() (g++ -O2, single thread)"
        self.write()

    def write(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.doc, f, indent=1)
        os.replace(tmp, self.path)

    def log(self, msg):
        print("[%s] %s" % (os.path.basename(self.path), msg), flush=True)


def ckpt_path(args, name):
    return os.path.join(args.checkpoint, "oracle_%s_state.npz" % name) if args.checkpoint else None


def ckpt_save(path, **arrays):
    if path:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp.npz"
        np.savez(tmp, **arrays)
        os.replace(tmp, path)


def ckpt_load(path, done):
    """The saved arrays if they belong to the state after `done` increments."""
    if not path or not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    if int(z["done"]) != done:
        return None
    return {k: z[k] for k in z.files}


def run_svk_schedule(ph, table, schedule, on_increment, recs=None, F=None, ckpt=None):
    """Increments of a St. Venant-Kirchhoff cell from the stress-free state (or
    from F after the increments in `recs`); on_increment(records) after each.
    Returns (F, P, records)."""
    K, mu = ms.phase_moduli(ph, table)
    recs = list(recs or [])
    F = oracle.identity_field(ph.shape) if F is None else F
    P = None
    for Fbar in schedule[len(recs):]:
        t0 = time.time()
        st, F, P, Pbar, S = oracle.solve_increment(K, mu, F, Fbar, ETA_NW, ETA_CG)
        recs.append(dict(incr_record(st, Pbar, S, time.time() - t0), Fbar=fl(Fbar)))
        ckpt_save(ckpt, F=F, P=P, done=len(recs))
        on_increment(recs)
        if st != 0:
            break
    if P is None:  # every increment was already recorded: the stress of the saved state
        P = oracle.svk_stress(F, K, mu)
    return F, P, recs


def _progress(out):
    def cb(recs):
        out.doc["increments"] = recs
        r = recs[-1]
        out.log("increment %d: status %d solves %d cg %s %.0fs" % (len(recs) - 1, r["status"], r["n_solves"],
                                                                    r["cg_iters"], r["seconds"]))
        out.write()
    return cb


def cfg_e1(args):
    N = 31
    ph = ms.cubic_inclusion(N, 9)
    out = Out("e1", {"config": "paper cubic inclusion (Sec. 4.4): 31^3, 9^3 cube x10 moduli, simple shear 1.0",
                     "grid": [N, N, N], "phase_sha256": digest(ph), "table": TABLE,
                     "eta_nw": ETA_NW, "eta_cg": ETA_CG})
    F, P, _ = run_svk_schedule(ph, TABLE, [ms.simple_shear(1.0)], _progress(out))
    out.doc["final"] = field_summary(F, P, sample_index(N ** 3))
    out.doc["complete"] = True
    out.write()


def cfg_c2(args):
    N = 128
    ph = ms.grf_threshold(N, ell=8.0, frac=0.3, seed=1603)
    sched = ms.c2_schedule(args.increments or 5)
    out = Out("c2", {"config": "128^3 two-phase GRF cell (l = 8, 30 %, x10 moduli), isochoric stretch 1.01..1.05",
                     "grid": [N, N, N], "phase_sha256": digest(ph), "table": TABLE,
                     "eta_nw": ETA_NW, "eta_cg": ETA_CG}, resume=bool(args.checkpoint))
    ck = ckpt_path(args, "c2")
    recs = [r for r in out.doc.get("increments", []) if r["status"] == 0]
    state = ckpt_load(ck, len(recs)) if recs else None
    if state is None:
        recs = []
    else:
        out.log("continuing after increment %d" % (len(recs) - 1))
    F, P, _ = run_svk_schedule(ph, TABLE, sched, _progress(out), recs, None if state is None else state["F"], ck)
    out.doc["final"] = field_summary(F, P, sample_index(N ** 3))
    out.doc["complete"] = len(out.doc["increments"]) == len(sched)
    out.write()


def cfg_c3(args):
    items = ms.c3_batch()
    picks = [0, 16, 32, 48]
    out = Out("c3", {"config": "64-cell sphere batch: the first cell of each size class, one increment",
                     "cells": [], "eta_nw": ETA_NW, "eta_cg": ETA_CG}, resume=bool(args.checkpoint))
    done = {c["index"] for c in out.doc["cells"]}
    for r in picks:
        if r in done:
            continue
        it = items[r]
        N = it["N"]
        F, P, recs = run_svk_schedule(it["phase"], it["table"], [it["Fbar"]], lambda recs: None)
        cell = {"index": r, "grid": [N, N, N], "phase_sha256": digest(it["phase"]), "table": it["table"],
                "Fbar": fl(it["Fbar"]), "volume_fraction": it["frac"], "increments": recs,
                "final": field_summary(F, P, sample_index(N ** 3))}
        out.doc["cells"].append(cell)
        out.log("cell %d (%d^3): solves %d cg %s" % (r, N, recs[-1]["n_solves"], recs[-1]["cg_iters"]))
        out.write()
    out.doc["complete"] = True
    out.write()


def cfg_c4(args):
    N = 96
    ph, frac = ms.rsa_spheres(N, 0.25, seed=1604)
    table = [(ms.K_SOFT, ms.MU_SOFT, 0.003, 0.01), (ms.K_SOFT, ms.MU_SOFT, 0.006, 0.01)]
    nin = args.increments or 4
    sched = ms.c4_schedule(20, 0.1)[:nin]
    out = Out("c4", {"config": "J2 96^3, RSA spheres 25 %, tau_y0 0.003 / 0.006, H 0.01, simple shear 0.005 per increment",
                     "grid": [N, N, N], "phase_sha256": digest(ph), "sphere_fraction": frac, "table": table,
                     "eta_nw": ETA_NW, "eta_cg": ETA_CG, "increments": []}, resume=bool(args.checkpoint))
    t = np.asarray(table)
    K, mu, ty0, H = (t[ph, k].copy() for k in range(4))
    F = oracle.identity_field(ph.shape)
    hist = oracle.virgin_history(ph.shape)
    P = None
    ck = ckpt_path(args, "c4")
    recs = [r for r in out.doc.get("increments", []) if r["status"] == 0]
    state = ckpt_load(ck, len(recs)) if recs else None
    if state is None:
        out.doc["increments"] = []
    else:
        out.doc["increments"] = recs
        F, P, hist = state["F"], state["P"], state["hist"]
        out.log("continuing after increment %d" % (len(recs) - 1))
    for k, Fbar in enumerate(sched):
        if k < len(out.doc["increments"]):
            continue
        t0 = time.time()
        st, F, P, Pbar, hist, S = oracle.solve_increment_j2(K, mu, ty0, H, hist, F, Fbar, ETA_NW, ETA_CG)
        sec = time.time() - t0
        rec = dict(incr_record(st, Pbar, S, sec), Fbar=fl(Fbar),
                   plastic_fraction=float(np.mean(hist[6] > 0)), max_eps_p=float(hist[6].max()))
        out.doc["increments"].append(rec)
        ckpt_save(ck, F=F, P=P, hist=hist, done=len(out.doc["increments"]))
        out.log("increment %d: status %d solves %d cg %s %.0fs" % (k, st, S["n_solves"], S["cg_iters"], sec))
        out.write()
        if st != 0:
            break
    fs = field_summary(F, P, sample_index(N ** 3))
    fs["eps_p_samples"] = fl(hist[6].reshape(-1)[fs["sample_index"]])
    out.doc["final"] = fs
    out.doc["complete"] = len(out.doc["increments"]) == len(sched)
    out.write()


def cfg_c5(args):
    N = 192
    mu = ms.lognormal_field(N, 0.5, 8.0, seed=1605)
    mu_t = ms.lognormal_field(N, 0.5, 8.0, seed=1606)
    K = np.full(mu.shape, ms.K_SOFT)
    case = 0
    Fbar = ms.c5_load_cases(0.05)[case]
    out = Out("c5", {"config": "adjoint 192^3, log-normal mu (sigma 0.5, l = 8, seed 1605), load case 0 (uniaxial e1 0.05); "
                               "target Pbar from the seed-1606 field; cotangent 2 (Pbar - Pbar_target)",
                     "grid": [N, N, N], "mu_sha256": digest(mu), "mu_target_sha256": digest(mu_t), "K": ms.K_SOFT,
                     "load_case": case, "Fbar": fl(Fbar), "eta_nw": ETA_NW, "eta_cg": ETA_CG},
              resume=bool(args.checkpoint))
    idx = sample_index(N ** 3)
    ck = ckpt_path(args, "c5")
    state = ckpt_load(ck, 1) if "forward" in out.doc else None
    if state is None:
        out.doc.pop("target", None)
        t0 = time.time()
        st, F, P, Pbar, S = oracle.solve_increment(K, mu, oracle.identity_field(mu.shape), Fbar, ETA_NW, ETA_CG)
        out.doc["forward"] = dict(incr_record(st, Pbar, S, time.time() - t0), final=field_summary(F, P, idx))
        ckpt_save(ck, F=F, done=1)
        out.log("forward: status %d solves %d cg %s" % (st, S["n_solves"], S["cg_iters"]))
        out.write()
        del P
    else:
        F = state["F"]
        st, Pbar = out.doc["forward"]["status"], np.asarray(out.doc["forward"]["Pbar"])
        out.log("continuing after the forward solve")
    if "target" not in out.doc:
        t0 = time.time()
        st_t, _, _, Pbar_t, S_t = oracle.solve_increment(K, mu_t, oracle.identity_field(mu.shape), Fbar, ETA_NW,
                                                         ETA_CG)
        out.doc["target"] = incr_record(st_t, Pbar_t, S_t, time.time() - t0)
        out.log("target: status %d solves %d cg %s" % (st_t, S_t["n_solves"], S_t["cg_iters"]))
        out.write()
    st_t, Pbar_t = out.doc["target"]["status"], np.asarray(out.doc["target"]["Pbar"])
    g = 2.0 * (Pbar - Pbar_t)
    t0 = time.time()
    st_a, dmu, dK, it = oracle.adjoint(K, mu, F, g, ETA_CG)
    out.doc["adjoint"] = {"status": int(st_a), "gbar": fl(g), "cg_iters": int(it), "seconds": round(time.time() - t0, 2),
                          "sample_index": [int(i) for i in idx], "dLdmu_samples": fl(dmu.reshape(-1)[idx]),
                          "dLdmu_norm": float(np.linalg.norm(dmu)), "dLdmu_sum": float(dmu.sum()),
                          "dLdmu_absmax": float(np.abs(dmu).max())}
    out.log("adjoint: status %d cg %d" % (st_a, it))
    out.doc["complete"] = st == 0 and st_t == 0 and st_a == 0
    out.write()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["e1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--increments", type=int, default=0)
    ap.add_argument("--checkpoint", default="", help="directory for the oracle's state between increments")
    args = ap.parse_args()
    oracle.build()
    globals()["cfg_" + args.config](args)


if __name__ == "__main__":
    main()
