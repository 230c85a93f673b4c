"""Command-line front end of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Reads and writes ``.npy`` files (loaded with ``allow_pickle=False``) and
prints one JSON line with the status and statistics.  Tensor fields are
``(9, n0, n1, n2)`` float64; K and mu are ``(n0, n1, n2)`` float64 (or scalars
given with --K-value / --mu-value).

  python -m oracle project         --in A.npy --out GA.npy [--nyq-identity]
  python -m oracle apply_operator  --F F.npy --K K.npy --mu mu.npy --in p.npy --out Ap.npy
  python -m oracle constitutive    --F F.npy --K K.npy --mu mu.npy --out P.npy
  python -m oracle solve_increment --F Ft.npy --K K.npy --mu mu.npy --fbar 1,0.05,0,0,1,0,0,0,1
                                   --out-F F.npy --out-P P.npy [--eta-nw 1e-5] [--eta-cg 1e-8]

project is G of Sec. 2.5 (zero at Nyquist frequencies unless --nyq-identity,
App. C); apply_operator is A p = G(K(F) : p) (Sec. 2.6); constitutive the St.
Venant-Kirchhoff stress (Sec. 4.2); solve_increment one load increment of
Algorithm 1 from the committed state Ft to the macroscopic gradient F-bar.
"""
import argparse
import json
import sys

import numpy as np

from . import apply_operator, project, solve_increment, svk_stress


def _load(path):
    return np.load(path, allow_pickle=False).astype(np.float64)


def _moduli(args, shape):
    K = _load(args.K) if args.K else np.full(shape, float(args.K_value))
    mu = _load(args.mu) if args.mu else np.full(shape, float(args.mu_value))
    return K, mu


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m oracle", description=__doc__.splitlines()[0])
    ap.add_argument("command", choices=["project", "apply_operator", "constitutive", "solve_increment"])
    ap.add_argument("--in", dest="inp")
    ap.add_argument("--out")
    ap.add_argument("--F")
    ap.add_argument("--K")
    ap.add_argument("--mu")
    ap.add_argument("--K-value", type=float)
    ap.add_argument("--mu-value", type=float)
    ap.add_argument("--fbar", help="9 comma-separated components, row-major")
    ap.add_argument("--out-F")
    ap.add_argument("--out-P")
    ap.add_argument("--eta-nw", type=float, default=1e-5)
    ap.add_argument("--eta-cg", type=float, default=1e-8)
    ap.add_argument("--nyq-identity", action="store_true")
    args = ap.parse_args(argv)

    rec = {"command": args.command}
    if args.command == "project":
        A = _load(args.inp)
        np.save(args.out, project(A, nyq_identity=args.nyq_identity))
        rec["status"] = 0
    else:
        F = _load(args.F)
        K, mu = _moduli(args, F.shape[1:])
        if args.command == "apply_operator":
            np.save(args.out, apply_operator(F, K, mu, _load(args.inp)))
            rec["status"] = 0
        elif args.command == "constitutive":
            P = svk_stress(F, K, mu)
            np.save(args.out, P)
            rec["status"] = 0
            rec["pbar"] = P.reshape(9, -1).mean(axis=1).tolist()
        else:
            fbar = np.array([float(v) for v in args.fbar.split(",")], dtype=np.float64)
            if fbar.size != 9:
                ap.error("--fbar needs 9 components")
            st, Fn, P, Pbar, stats = solve_increment(K, mu, F, fbar.reshape(3, 3), args.eta_nw, args.eta_cg)
            if args.out_F:
                np.save(args.out_F, Fn)
            if args.out_P:
                np.save(args.out_P, P)
            rec.update({"status": int(st), "pbar": np.asarray(Pbar).reshape(-1).tolist(),
                        "n_solves": stats["n_solves"], "cg_iters": stats["cg_iters"]})
    print(json.dumps(rec))
    return 0 if rec["status"] == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
