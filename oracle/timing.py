"""CPU-baseline timing of the oracle -- TEST INFRASTRUCTURE ONLY (run by the
benchmark's CPU-baseline leg in a child process of its own).

    python -m oracle.timing --grid 128 --budget 20 [--cpu 0]

Pins the process to one host core, builds the oracle from its source with
-O3 -march=native into a temporary directory (the host it runs on), and times
projected-tangent operator applications (Sec. 2.6) on the 128^3 two-phase
benchmark cell at the linearisation point F = I + U(-0.01, 0.01) (seed 43)
with the direction p = U(-1, 1) (seed 42): at least one, then more until the
time budget is spent (at most `--max-reps`).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--budget", type=float, default=20.0)
    ap.add_argument("--max-reps", type=int, default=5)
    ap.add_argument("--cpu", type=int, default=-1, help="host core to pin to (default: the first allowed)")
    args = ap.parse_args()
    allowed = sorted(os.sched_getaffinity(0))
    core = args.cpu if args.cpu >= 0 else allowed[0]
    os.sched_setaffinity(0, {core})

    import oracle
    from paper_1603_08893_amd import microstructure as ms

    tmp = tempfile.mkdtemp(prefix="oracle_timed_")
    path = os.path.join(tmp, "liboracle_timed.so")
    t0 = time.perf_counter()
    flags = oracle.TIMED_FLAGS
    try:
        oracle.build(force=True, path=path, flags=flags)
    except Exception:  # a compiler without -march=native support: the portable -O3 build
        flags = ["-O3", "-fcx-limited-range"]
        oracle.build(force=True, path=path, flags=flags)
    t_build = time.perf_counter() - t0
    oracle.use_library(path)

    N = args.grid
    ph = ms.grf_threshold(N, ell=8.0, frac=0.3, seed=1603)
    K, mu = ms.phase_moduli(ph, [(ms.K_SOFT, ms.MU_SOFT), (ms.K_HARD, ms.MU_HARD)])
    F = ms.near_identity_field((N, N, N), seed=43, scale=0.01)
    p = ms.random_field((N, N, N), seed=42)
    times = []
    while len(times) < args.max_reps and (not times or sum(times) < args.budget):
        c0 = time.perf_counter()
        oracle.apply_operator(F, K, mu, p)
        times.append(time.perf_counter() - c0)
    for f in os.listdir(tmp):
        os.remove(os.path.join(tmp, f))
    os.rmdir(tmp)
    print(json.dumps({"grid": N, "reps": len(times), "seconds": times, "sec_per_matvec": sum(times) / len(times),
                      "core": core, "threads": 1, "flags": " ".join(flags), "build_seconds": round(t_build, 2),
                      "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "allowed_cpus": len(allowed)}),
          flush=True)


if __name__ == "__main__":
    main()
