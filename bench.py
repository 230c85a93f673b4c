"""Benchmark of the finite-strain FFT Newton-Krylov hot path on one MI355X.

Workload (the paper's method on a 128^3 periodic cell): two phases from a
seeded Gaussian random field (correlation length 8 voxels) thresholded at 30 %
inclusion volume fraction, St. Venant-Kirchhoff with 10x modulus contrast
(K, mu = 0.833, 0.386 and 8.33, 3.86), isochoric stretch Fbar =
diag(l, l^-1/2, l^-1/2) with l = 1.01 ... 1.05 in 5 increments, Newton
tolerance 1e-5, CG tolerance 1e-8, FP64.

A step is one load increment: constitutive update, right-hand sides, every CG
iteration (projected-tangent operator: tangent action, 3-D FFT, projection,
inverse FFT; fused vector updates) and the Newton update.  The timed steps run
the 5-increment schedule from the stress-free state (repeating it if --steps
exceeds 5).  `value` is projected-tangent operator applications per second over
the timed steps.  Besides that line's fields the JSON carries one CG
iteration kernel by kernel (stream events around every launch; `roofline`
is its slowest kernel, with the hardware-counter traffic recorded for these
kernel sources under profiles/ when it matches), the operator alone
(back-to-back applications) pass by pass, the achievable streaming rate of
the device measured with the library's own read / write / copy / triad
kernels (every fraction is also given against it), the operator and CG
iteration at 192^3 (spectra beyond the last-level cache), the FP32-mixed solve
of the same increments, P-bar against the oracle's stored run of the same
cell, and the CPU oracle's rate (one pinned core, -O3 -march=native build).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 128
TABLE = [(0.833, 0.386), (8.33, 3.86)]


def pass_bytes_per_voxel(prec_bytes, n2):
    """Algorithmic HBM bytes per voxel of each operator pass (no re-reads).

    Real fields: 9 components; spectra: 9 complex half-lines of h entries per
    n2 voxels (h = n2/2 for even n2).  Pass 1 reads the direction p and F
    (and one phase byte) and writes the spectrum; passes 2-4 read and write
    the spectrum; pass 5 reads the spectrum and writes the result.
    """
    h = n2 // 2 if n2 % 2 == 0 else (n2 + 1) // 2
    spec = 9 * 2 * prec_bytes * h / n2
    field = 9 * prec_bytes
    return {1: 2 * field + 1 + spec, 2: 2 * spec, 3: 2 * spec, 4: 2 * spec, 5: spec + field}


def cg_bytes_per_voxel(prec_bytes, n2, x_window=8):
    """Algorithmic HBM bytes per voxel of each kernel of one CG iteration (after
    the first), averaged over a window of W = x_window iterations: pass 1 reads
    r, the previous p and the linearisation point F (and one phase byte), writes
    p and the spectrum, and once per window reads x and the W - 1 older
    directions and writes x (the deferred x updates; W = 1: every iteration);
    passes 2-4 read and write the spectrum; pass 5 reads the spectrum and r,
    writes r; alpha and beta touch only per-cell scalars and block partial sums."""
    op = pass_bytes_per_voxel(prec_bytes, n2)
    field = 9 * prec_bytes
    spec = op[2] / 2
    W = x_window
    return {"pass1": 3 * field + 1 + field + spec + (W + 1) * field / W, "alpha": 0.0, "pass2": op[2],
            "pass3": op[3], "pass4": op[4], "pass5": spec + 2 * field, "beta": 0.0}


def pass1_variant_bytes(prec_bytes, n2, x_window):
    """Pass 1 of the CG inside a window (no x update) and at its start (x
    updated with the window's W directions), bytes per voxel."""
    field = 9 * prec_bytes
    plain = 3 * field + 1 + field + pass_bytes_per_voxel(prec_bytes, n2)[2] / 2
    return {"pass1_within_window": plain if x_window > 1 else plain + 2 * field,
            "pass1_xupdate": plain + (x_window + 1) * field}


def three_kernel_bytes_per_voxel(prec_bytes, n2):
    """Lower-bound bytes per voxel of any operator built from three kernels:
    the compulsory reads of p, F and the phase byte and the write of A p, plus
    one write and one read of the 9-field half spectrum (n2/2 + 1 entries per
    line, the Nyquist entry included) per transform direction."""
    field = 9 * prec_bytes
    spec = 9 * 2 * prec_bytes * (n2 // 2 + 1) / n2
    return 3 * field + 1 + 4 * spec


KERNEL_NAMES = {"pass1": "k_fwd_a2<double,FWD_CG>", "pass2": "k_col_a1<double,fwd>", "pass3": "k_col_a0_project<double>",
                "pass4": "k_col_a1<double,inv>", "pass5": "k_inv_a2<double,INV_CGR>", "alpha": "k_col_a1 (step-length groups)",
                "beta": "k_cg_beta"}


def kernel_sources_digest():
    """sha256 over the HIP sources: hardware-counter traffic recorded for other
    sources no longer describes these kernels."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1603_08893_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it was taken on other kernel sources (or is absent)."""
    path = os.path.join(ROOT, "profiles", "traffic_grf128.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != kernel_sources_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cg_kernel_rows(ms_by_kernel, bytes_per_voxel, n, ceiling=None):
    """Per-kernel rows of one CG iteration: ms, algorithmic bytes per voxel,
    GB/s, fraction of the 8 TB/s peak and of the measured streaming ceiling."""
    rows = {}
    for k, t in ms_by_kernel.items():
        row = {"ms": round(t, 5), "bytes_per_voxel": round(bytes_per_voxel[k], 3)}
        if bytes_per_voxel[k] > 0:
            gbs = bytes_per_voxel[k] * n / (t * 1e-3) / 1e9
            row.update({"GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
            if ceiling:
                row["frac_of_ceiling"] = round(gbs / ceiling, 4)
        rows[k] = row
    return rows


def stream_ceiling(torch, dev, gib=2, reps=10):
    """The achievable HBM streaming rate, measured with the library's own
    stream kernels (fftnk_stream, 8-byte lanes) on arrays of `gib` GiB: read,
    write, copy, triad, with normal and with non-temporal accesses; the
    ceiling for kernels that read and write is the best copy or triad."""
    from paper_1603_08893_amd.fftnk import stream
    nb = gib << 30
    a = torch.ones(nb // 8, dtype=torch.float64, device=dev)
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    out = {"bytes_per_array": nb, "lane_bytes": 8, "kernels": "fftnk_stream (k_stream_*<double, nt>)"}
    for nt in (False, True):
        for kind in ("read", "write", "copy", "triad"):
            _, gbs = stream(kind, 8, c if kind == "read" else a, b, c, reps=reps, nontemporal=nt)
            out[kind + ("_nt" if nt else "") + "_GB_s"] = round(gbs, 1)
    out["ceiling_GB_s"] = max(out["copy_GB_s"], out["triad_GB_s"], out["copy_nt_GB_s"], out["triad_nt_GB_s"])
    del a, b, c
    torch.cuda.empty_cache()
    return out


def oracle_pbars(name):
    """P-bar per increment of the oracle's stored run of a configuration
    (tests/golden/oracle_<name>.json), or [] when absent."""
    try:
        d = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_%s.json" % name)))
    except (OSError, ValueError):
        return [], {}
    return [np.asarray(r["Pbar"]) for r in d.get("increments", []) if r.get("status") == 0], d


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def cpu_baseline_leg(budget=20.0):
    """The oracle timed on one pinned host core, built -O3 -march=native on this
    host, in a child process (python -m oracle.timing); with the time of a
    whole increment of the benchmark cell extrapolated from the oracle's own
    operator counts."""
    import subprocess
    res = subprocess.run([sys.executable, "-m", "oracle.timing", "--grid", str(N), "--budget", str(budget),
                          "--max-reps", "5"], cwd=ROOT, capture_output=True, text=True, timeout=600)
    lines = [l for l in res.stdout.splitlines() if l.startswith("{")]
    if res.returncode != 0 or not lines:
        sys.stderr.write(res.stdout[-2000:] + res.stderr[-2000:])
        return None
    t = json.loads(lines[-1])
    spm = t["sec_per_matvec"]
    out = {"value": round(1.0 / spm, 4), "unit": "matvec/s", "cores": t["threads"], "kind": "oracle",
           "sample": "%d projected-tangent operator applications on the 128^3 two-phase cell (FP64, F = I + "
                     "U(-0.01, 0.01)) on one pinned host core, %.1f s; oracle built %s on this host" % (
                         t["reps"], sum(t["seconds"]), t["flags"]),
           "cpu_model": t["cpu_model"], "host_cpus": t["host_cpus"], "pinned_core": t["core"]}
    _, gold = oracle_pbars("c2")
    incs = gold.get("increments", []) if gold else []
    if incs:
        # an increment costs its CG iterations plus one operator-sized right-hand
        # side per linear solve (the boundary-condition one included)
        ops = [sum(r["cg_iters"]) + r["n_solves"] for r in incs]
        out["increment_seconds_extrapolated"] = [round(o * spm, 1) for o in ops]
        out["extrapolation"] = ("timed operator applications x (CG iterations + right-hand sides) of the oracle's "
                                "own run of each increment")
        out["increment_seconds_build_host"] = [r["seconds"] for r in incs]
        out["build_host_note"] = "the same oracle (-O2 build) measured whole on another machine's core"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--matvec-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-192", action="store_true", help="skip the 192^3 operator and CG-iteration rows")
    ap.add_argument("--no-256", action="store_true", help="skip the 256^3 operator rows")
    ap.add_argument("--x-window", type=int, default=None,
                    help="CG directions kept for the windowed x update (1..8; default: the library's)")
    ap.add_argument("--operator-only", action="store_true",
                    help="profiling mode: only the operator passes at a synthetic linearisation point, plus one "
                         "1 GiB device copy (the reference for scaling memory counters); prints per-pass times")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--extra", default="",
                    help="comma list of sizes,c3,c4,c5,nyq,mixed,krylov,c2d,passes2d,j2tangent,oddeven,tune,cpu_baseline,slab: instead of the headline line, one JSON "
                         "line per extra measurement (operator at 96^3..256^3; 64 batched cells; J2 at 96^3; adjoint "
                         "8 x 192^3; the two Nyquist choices at 128^3; mixed control at 128^3; CG / Chebyshev / "
                         "Richardson / GMRES at 128^3; the 2-D plane-strain example at 451^2; the plan autotuner on "
                         "several cells; the CPU oracle at several sizes and on all host cores; one GPU's slab share of "
                         "the 128^3 operator on 8 GPUs)")
    args = ap.parse_args()
    if args.operator_only:
        return operator_only(args)
    if args.extra:
        return extra(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (the per-GPU work is one "
              "periodic cell; independent cells or load cases would be dealt out one per GPU, a single "
              "large cell split into slabs along a0 with an all-to-all around the a0 pass).", flush=True)
        sys.exit(2)

    import torch
    from paper_1603_08893_amd import microstructure as ms
    from paper_1603_08893_amd.fftnk import Solver

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    phase = ms.grf_threshold(N, ell=8.0, frac=0.3, seed=1603)
    sched = ms.c2_schedule(5)
    print("# inputs ready (%.1fs), inclusion fraction %.4f" % (time.time() - t0, phase.mean()), file=sys.stderr,
          flush=True)

    def make(prec):
        s = Solver((N, N, N), precision=prec, x_window=args.x_window)
        s.set_phases(phase)
        s.set_material(TABLE)
        return s

    def run_steps(s, k0, count):
        cg, solves, pbars, stats = 0, 0, [], []
        for k in range(k0, k0 + count):
            if k % len(sched) == 0:
                s.reset_state()
            _, _, _, Pbar, st = s.solve_increment(sched[k % len(sched)], 1e-5, 1e-8, fields=False)
            cg += sum(st[0]["cg_iters"])
            solves += st[0]["n_solves"]
            pbars.append(Pbar[0].copy())
            stats.append(st[0])
        return cg, solves, pbars, stats

    # ------------------------------------------------------------ FP64 solve (the timed steps)
    s64 = make("fp64")
    for k in range(args.warmup):
        run_steps(s64, k, 1)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record()
    cg64, solves64, pbars64, stats64 = run_steps(s64, 0, args.steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = ev0.elapsed_time(ev1)
    sec = ms_total / 1e3
    print("# fp64 steps: %.1f ms, %d CG iterations, %d solves, wall %.2fs" % (ms_total, cg64, solves64, wall),
          file=sys.stderr, flush=True)

    # ------------------------------------------------------------ the CG iteration kernel by kernel
    # (HIP events on the library's stream around every launch, at the converged
    # state of the last timed increment)
    F_lin = s64.get_state()
    n = N ** 3
    cgk, p1var = s64.profile_cg(20, detail=True)
    cgb = cg_bytes_per_voxel(8, N, s64.x_window)
    p1b = pass1_variant_bytes(8, N, s64.x_window)
    for key in ("pass1_within_window", "pass1_xupdate"):
        p1var[key] = {"ms": round(p1var[key], 5), "bytes_per_voxel": p1b[key],
                      "GB_s": round(p1b[key] * n / (p1var[key] * 1e-3) / 1e9, 1)}
    cg_iter_ms = sum(cgk.values())
    dom = max(cgk, key=lambda k: cgk[k])
    achieved = cgb[dom] * n / (cgk[dom] * 1e-3) / 1e9
    print("# CG iteration %.3f ms: %s" % (cg_iter_ms, {k: round(v, 4) for k, v in cgk.items()}), file=sys.stderr,
          flush=True)

    # ------------------------------------------------------------ operator alone + per-pass timing
    res = {}

    def operator_bench(s, reps):
        s.set_linearization(F_lin)
        p = s.project(torch.from_numpy(ms.random_field((N, N, N), seed=42).reshape(-1)).to(dev))
        out = s.field()
        for _ in range(3):
            s.apply_operator(p, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            s.apply_operator(p, out)
        e1.record()
        torch.cuda.synchronize()
        t_mv = e0.elapsed_time(e1) / reps
        # pass by pass, each timed alone over the same number of launches
        # (the internal buffers of the context: pass 1 reads its direction field)
        passes = {}
        for k in range(1, 6):
            for _ in range(2):
                s.launch_pass(k)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                s.launch_pass(k)
            e1.record()
            torch.cuda.synchronize()
            passes[k] = e0.elapsed_time(e1) / reps
        return t_mv, passes

    t_mv64, passes64 = operator_bench(s64, args.matvec_reps)
    bpv64 = pass_bytes_per_voxel(8, N)
    mv_bytes64 = sum(bpv64.values()) * n
    pass_rows = {}
    for k in range(1, 6):
        gbs = bpv64[k] * n / (passes64[k] * 1e-3) / 1e9
        pass_rows["pass%d" % k] = {"ms": round(passes64[k], 5), "bytes_per_voxel": round(bpv64[k], 3),
                                   "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    print("# fp64 operator %.3f ms (%.0f GB/s over the 5-pass bytes); passes %s" %
          (t_mv64, mv_bytes64 / (t_mv64 * 1e-3) / 1e9, {k: round(v, 4) for k, v in passes64.items()}),
          file=sys.stderr, flush=True)

    # ------------------------------------------------------------ FP32-mixed solve of the same increments
    fp32 = None
    if not args.no_fp32:
        s32 = make("fp32")
        run_steps(s32, 0, 1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cg32, solves32, pbars32, stats32 = run_steps(s32, 0, min(args.steps, 5))
        e1.record()
        torch.cuda.synchronize()
        sec32 = e0.elapsed_time(e1) / 1e3
        err = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b))) for a, b in zip(pbars32, pbars64))
        cgk32, p1var32 = s32.profile_cg(20, detail=True)
        x_window32 = s32.x_window
        p1b32 = pass1_variant_bytes(4, N, x_window32)
        for key in ("pass1_within_window", "pass1_xupdate"):
            p1var32[key] = {"ms": round(p1var32[key], 5), "bytes_per_voxel": p1b32[key],
                            "GB_s": round(p1b32[key] * n / (p1var32[key] * 1e-3) / 1e9, 1)}
        t_mv32, passes32 = operator_bench(s32, args.matvec_reps)
        bpv32 = pass_bytes_per_voxel(4, N)
        fp32 = {
            "increments_per_s": round(min(args.steps, 5) / sec32, 3),
            "cg_matvecs_per_s": round(cg32 / sec32, 1),
            "cg_iterations": cg32,
            "operator_ms": round(t_mv32, 4),
            "operator_matvecs_per_s": round(1e3 / t_mv32, 1),
            "operator_GB_s": round(sum(bpv32.values()) * n / (t_mv32 * 1e-3) / 1e9, 1),
            "operator_effective_frac": round(three_kernel_bytes_per_voxel(4, N) * n / (t_mv32 * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4),
            "passes_ms": {k: round(v, 5) for k, v in passes32.items()},
            "pbar_rel_diff_vs_fp64_gpu": err,
            "speedup_vs_fp64": round((min(args.steps, 5) / sec32) / (args.steps / sec), 3),
            "cg_iteration_kernels": cgk32,
        }
        pbars32_all = pbars32
        del s32

    # ------------------------------------------------------------ the achievable streaming rate (own kernels)
    ceil = stream_ceiling(torch, dev)
    ceiling = ceil["ceiling_GB_s"]
    print("# stream ceiling %s" % ceil, file=sys.stderr, flush=True)
    for row in pass_rows.values():
        row["frac_of_ceiling"] = round(row["GB_s"] / ceiling, 4)
    if fp32 is not None:
        cb32 = cg_bytes_per_voxel(4, N, x_window32)
        rows32 = cg_kernel_rows(fp32.pop("cg_iteration_kernels"), cb32, n, ceiling)
        d32 = max((k for k in rows32 if cb32[k] > 0), key=lambda k: rows32[k]["ms"])
        fp32["cg_iteration"] = {"ms": round(sum(r["ms"] for r in rows32.values()), 4),
                                "bytes_per_voxel": round(sum(cb32.values()), 2), "kernels": rows32,
                                "x_window": x_window32, "pass1_variants": p1var32}
        fp32["roofline"] = {"bound": "hbm", "kernel": KERNEL_NAMES[d32].replace("double", "float"),
                            "achieved": rows32[d32]["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": rows32[d32]["frac"], "frac_of_ceiling": rows32[d32]["frac_of_ceiling"],
                            "traffic": recorded_traffic(KERNEL_NAMES[d32].replace("double", "float")),
                            "algorithmic_bytes_per_launch": int(round(cb32[d32] * n)), "launch_ms": rows32[d32]["ms"]}

    # ------------------------------------------------------------ 192^3: spectra beyond the last-level cache
    big = {}
    if not args.no_192:
        N2 = 192
        ph2 = ms.grf_threshold(N2, ell=8.0, frac=0.3, seed=1603)
        for prec, pb in (("fp64", 8), ("fp32", 4)):
            s = Solver((N2,) * 3, precision=prec)
            s.set_phases(ph2)
            s.set_material(TABLE)
            s.solve_increment(sched[0], 1e-5, 1e-8, fields=False)
            k = s.profile_cg(10)
            cb = cg_bytes_per_voxel(pb, N2, s.x_window)
            it_ms = sum(k.values())
            s.set_linearization(s.get_state())
            p = s.project(torch.from_numpy(ms.random_field((N2,) * 3, seed=42).reshape(-1)).to(dev))
            out = s.field()
            for _ in range(3):
                s.apply_operator(p, out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                s.apply_operator(p, out)
            e1.record()
            torch.cuda.synchronize()
            t_op = e0.elapsed_time(e1) / 20
            ob = sum(pass_bytes_per_voxel(pb, N2).values()) * N2 ** 3
            big[prec] = {"operator_ms": round(t_op, 4), "operator_GB_s": round(ob / (t_op * 1e-3) / 1e9, 1),
                         "operator_frac": round(ob / (t_op * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "operator_frac_of_ceiling": round(ob / (t_op * 1e-3) / 1e9 / ceiling, 4),
                         "cg_iteration_ms": round(it_ms, 4),
                         "cg_iteration_GB_s": round(sum(cb.values()) * N2 ** 3 / (it_ms * 1e-3) / 1e9, 1),
                         "cg_kernels": cg_kernel_rows(k, cb, N2 ** 3, ceiling)}
            del s, p, out
            torch.cuda.empty_cache()
        print("# 192^3: %s" % {k: (v["operator_ms"], v["cg_iteration_ms"]) for k, v in big.items()}, file=sys.stderr,
              flush=True)

    # ------------------------------------------------------------ 256^3: operator alone (no solve)
    big256 = {}
    if not args.no_256:
        N3 = 256
        ph3 = ms.grf_threshold(N3, ell=8.0, frac=0.3, seed=1603)
        Flin = torch.from_numpy(ms.near_identity_field((N3,) * 3, seed=43, scale=0.01).reshape(-1)).to(dev)
        for prec, pb in (("fp64", 8), ("fp32", 4)):
            s = Solver((N3,) * 3, precision=prec)
            s.set_phases(ph3)
            s.set_material(TABLE)
            s.set_linearization(Flin)
            p = s.project(torch.from_numpy(ms.random_field((N3,) * 3, seed=42).reshape(-1)).to(dev))
            out = s.field()
            for _ in range(3):
                s.apply_operator(p, out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                s.apply_operator(p, out)
            e1.record()
            torch.cuda.synchronize()
            t_op = e0.elapsed_time(e1) / 20
            ob = sum(pass_bytes_per_voxel(pb, N3).values()) * N3 ** 3
            big256[prec] = {"operator_ms": round(t_op, 4), "operator_GB_s": round(ob / (t_op * 1e-3) / 1e9, 1),
                            "operator_frac": round(ob / (t_op * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "operator_frac_of_ceiling": round(ob / (t_op * 1e-3) / 1e9 / ceiling, 4)}
            del s, p, out
            torch.cuda.empty_cache()
        del Flin
        torch.cuda.empty_cache()
        print("# 256^3 operator: %s" % {k: v["operator_ms"] for k, v in big256.items()}, file=sys.stderr, flush=True)

    # ------------------------------------------------------------ CPU oracle on a bounded sample
    cpu = None if args.no_cpu_baseline else cpu_baseline_leg()

    # ------------------------------------------------------------ P-bar against the oracle's run of the same cell
    gold, _ = oracle_pbars("c2")
    vs_oracle = None
    if gold:
        m = min(len(gold), args.steps, 5)
        vs_oracle = {"increments_compared": m,
                     "fp64": max(rel_err(pbars64[t], gold[t]) for t in range(m))}
        if fp32 is not None:
            vs_oracle["fp32_mixed"] = max(rel_err(pbars32_all[t], gold[t]) for t in range(min(m, len(pbars32_all))))

    line = {
        "metric": "projected-tangent matvecs/s at 128^3 (FP64 Newton-Krylov solve)",
        "value": round(cg64 / sec, 2),
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "128^3 two-phase GRF cell (30%, 10x contrast), St.V-K, isochoric stretch "
                               "1.01..1.05 in 5 increments, eta_NW 1e-5, eta_CG 1e-8", "grid": [N, N, N],
                   "precision": "fp64"},
        "newton_increments_per_s": round(args.steps / sec, 3),
        "linear_solves": solves64,
        "cg_iterations": cg64,
        "cg_per_increment": [s["cg_iters"] for s in stats64],
        "inputs_sha256": {"phase": __import__("hashlib").sha256(np.ascontiguousarray(phase).tobytes()).hexdigest()},
        "pbar_last": [float(v) for v in pbars64[-1]],
        "operator": {"ms": round(t_mv64, 4), "matvecs_per_s": round(1e3 / t_mv64, 1),
                     "bytes_5pass_per_voxel": round(sum(bpv64.values()), 2),
                     "GB_s": round(mv_bytes64 / (t_mv64 * 1e-3) / 1e9, 1),
                     "frac_of_hbm_peak": round(mv_bytes64 / (t_mv64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "frac_of_ceiling": round(mv_bytes64 / (t_mv64 * 1e-3) / 1e9 / ceiling, 4),
                     "cache_note": "at 128^3 the FP64 half spectrum (153 MB) fits the 256 MB last-level cache: "
                                   "passes 2-4 are cache-assisted; grid_192 holds the HBM-bound rates",
                     # the same time over the 3-kernel lower-bound bytes
                     "bytes_3kernel_per_voxel": round(three_kernel_bytes_per_voxel(8, N), 2),
                     "effective_frac": round(three_kernel_bytes_per_voxel(8, N) * n / (t_mv64 * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4)},
        "passes": pass_rows,
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(KERNEL_NAMES[dom]),
                     "algorithmic_bytes_per_launch": int(round(cgb[dom] * n)), "launch_ms": round(cgk[dom], 5),
                     "ceiling_GB_s": ceiling, "frac_of_ceiling": round(achieved / ceiling, 4)},
        "cg_iteration": {"ms": round(cg_iter_ms, 4), "bytes_per_voxel": round(sum(cgb.values()), 2),
                         "GB_s": round(sum(cgb.values()) * n / (cg_iter_ms * 1e-3) / 1e9, 1),
                         "kernels": cg_kernel_rows(cgk, cgb, n, ceiling),
                         "x_window": s64.x_window, "pass1_variants": p1var},
        "stream_ceiling": ceil,
        "grid_192": big,
        "grid_256": big256,
        "pbar_rel_err_vs_oracle": vs_oracle,
        "fp32_mixed": fp32,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def operator_only(args):
    """Operator passes alone at F = I + G(0.01 U(-1,1)) on the 128^3 two-phase cell, then the library's own
    1 GiB copy kernel (the reference that scales memory counters)."""
    import torch
    from paper_1603_08893_amd import microstructure as ms
    from paper_1603_08893_amd.fftnk import Solver

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    phase = ms.grf_threshold(N, ell=8.0, frac=0.3, seed=1603)
    s = Solver((N, N, N), precision=args.precision)
    s.set_phases(phase)
    s.set_material(TABLE)
    g64 = Solver((N, N, N), precision="fp64")
    g64.set_phases(phase)
    g64.set_material(TABLE)
    fl = g64.project(torch.from_numpy(ms.random_field((N, N, N), seed=43, scale=0.01).reshape(-1)).to(dev))
    fl.view(9, -1)[0::4] += 1.0
    s.set_linearization(fl)
    p = s.project(torch.from_numpy(ms.random_field((N, N, N), seed=42).reshape(-1)).to(dev))
    out = s.field()
    s.apply_operator(p, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for k in range(1, 6):
        e0.record()
        for _ in range(args.matvec_reps):
            s.launch_pass(k)
        e1.record()
        torch.cuda.synchronize()
        res["pass%d_ms" % k] = round(e0.elapsed_time(e1) / args.matvec_reps, 5)
    from paper_1603_08893_amd.fftnk import stream
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
    b = torch.empty_like(a)
    ms_copy, gbs = stream("copy", 8, b, a, reps=3)  # k_stream_copy<double>: 2^30 bytes read and written per launch
    res["copy_1GiB_ms"] = round(ms_copy, 4)
    res["copy_GB_s"] = round(gbs, 1)
    print(json.dumps({"operator_only": res, "precision": args.precision}), flush=True)


def _oracle_matvecs(job):
    """CPU-baseline worker (a separate process that never touches the GPU):
    `reps` oracle operator applications on an N^3 two-phase cell; seconds."""
    n_, reps, seed = job
    import oracle
    from paper_1603_08893_amd import microstructure as ms
    ph = (np.random.default_rng(seed).random((n_,) * 3) < 0.3).astype(np.uint8)
    K, mu = ms.phase_moduli(ph, TABLE)
    F = ms.near_identity_field((n_,) * 3, seed=seed + 1, scale=0.01)
    p = ms.random_field((n_,) * 3, seed=seed + 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.apply_operator(F, K, mu, p)
    return time.perf_counter() - t0


def _oracle_c3_solves(cells):
    """CPU-baseline worker (a separate process that never touches the GPU): one
    increment of each listed 32^3 cell of the 64-cell batch with the oracle;
    (seconds, statuses)."""
    import oracle
    from paper_1603_08893_amd import microstructure as ms
    out = []
    t0 = time.perf_counter()
    for r in cells:
        it = ms.c3_cell(r)
        K, mu = ms.phase_moduli(it["phase"], it["table"])
        st, _, _, _, _ = oracle.solve_increment(K, mu, oracle.identity_field(it["phase"].shape), it["Fbar"])
        out.append(int(st))
    return time.perf_counter() - t0, out


def extra(args):
    """Measurements beyond the headline: each prints one JSON line."""
    import torch
    from paper_1603_08893_amd import microstructure as ms
    from paper_1603_08893_amd.fftnk import J2, Solver, describe, homogenized_stress

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    which = [w.strip() for w in args.extra.split(",") if w.strip()]

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def emit(d):
        print(json.dumps(d), flush=True)

    if "sizes" in which:
        # the operator alone at several grid sizes: from 192^3 on, the FP64
        # half spectrum (>= 515 MB) exceeds the 256 MB last-level cache
        for n_ in (96, 192, 256):
            phase = ms.grf_threshold(n_, ell=8.0, frac=0.3, seed=1603)
            for prec in ("fp64", "fp32"):
                s = Solver((n_,) * 3, precision=prec)
                s.set_phases(phase)
                s.set_material(TABLE)
                fl = torch.from_numpy(ms.random_field((n_,) * 3, seed=43, scale=0.01).reshape(-1)).to(dev)
                g = Solver((n_,) * 3, precision="fp64")
                g.set_phases(phase)
                g.set_material(TABLE)
                fl = g.project(fl)
                del g
                fl.view(9, -1)[0::4] += 1.0
                s.set_linearization(fl)
                p = s.project(torch.from_numpy(ms.random_field((n_,) * 3, seed=42).reshape(-1)).to(dev))
                out = s.field()
                for _ in range(3):
                    s.apply_operator(p, out)
                reps = 20
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    s.apply_operator(p, out)
                e1.record()
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) / reps
                bpv = sum(pass_bytes_per_voxel(8 if prec == "fp64" else 4, n_).values())
                gbs = bpv * n_ ** 3 / (t * 1e-3) / 1e9
                emit({"extra": "operator", "grid": n_, "precision": prec, "ms": round(t, 4),
                      "matvecs_per_s": round(1e3 / t, 1), "bytes_per_voxel": round(bpv, 2), "GB_s": round(gbs, 1),
                      "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)})
                del s, fl, p, out
                torch.cuda.empty_cache()

    if "passes2d" in which:
        # the operator's passes one by one on the 2-D example's cell size and
        # its neighbours: 448 = 2^6 7, 450 = 2 3^2 5^2, 451 = 11 41 (prime
        # radices 11 and 41), 452 = 2^2 113; 20 back-to-back launches of each
        for n_ in (448, 450, 451, 452):
            shape = (n_, n_, 2)
            for prec in ("fp64", "fp32"):
                s = Solver(shape, precision=prec)
                s.set_phases(np.zeros(shape, dtype=np.uint8))
                s.set_material(TABLE)
                s.set_linearization(torch.from_numpy(ms.near_identity_field(shape, seed=12, scale=0.01).reshape(-1)))
                p = s.project(torch.from_numpy(ms.random_field(shape, seed=13).reshape(-1)).to(dev))
                out = s.field()
                s.apply_operator(p, out)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                us = {}
                for k in range(1, 6):
                    s.launch_pass(k)
                    e0.record()
                    for _ in range(20):
                        s.launch_pass(k)
                    e1.record()
                    torch.cuda.synchronize()
                    us[k] = round(e0.elapsed_time(e1) / 20 * 1e3, 2)
                pb = pass_bytes_per_voxel(8 if prec == "fp64" else 4, 2)
                emit({"extra": "passes2d", "grid": list(shape), "precision": prec, "pass_us": us,
                      "pass_GB_s": {k: round(pb[k] * n_ * n_ * 2 / (us[k] * 1e-6) / 1e9, 1) for k in us}})
                del s, p, out
                torch.cuda.empty_cache()

    if "j2tangent" in which:
        # J2 at 96^3 (the J2 workload's sphere cell), the first four simple-shear
        # increments, with the tangent recomputed per operator application and
        # with the compact tangent stored per linearisation point; St.V-K on
        # the same phase map for reference; CG kernels by profile_cg
        ph, frac = ms.rsa_spheres(96, 0.25, seed=1604)
        sched = ms.c4_schedule(20, 0.1)
        res = {"extra": "j2_tangent", "grid": 96, "sphere_fraction": round(frac, 4), "increments": 4}
        for name in ("svk", "j2_recomputed", "j2_stored"):
            s = Solver((96,) * 3, precision="fp64", j2_stored_tangent=(name == "j2_stored"))
            s.set_phases(ph)
            if name == "svk":
                s.set_material([(ms.K_SOFT, ms.MU_SOFT), (2 * ms.K_SOFT, 2 * ms.MU_SOFT)])
            else:
                s.set_material([(ms.K_SOFT, ms.MU_SOFT, 0.003, 0.01), (ms.K_SOFT, ms.MU_SOFT, 0.006, 0.01)], model=J2)
            s.solve_increment(sched[0], fields=False)  # warm-up
            s.reset_state()

            def run():
                out = []
                for Fb in sched[:4]:
                    out.append(s.solve_increment(Fb, fields=False))
                return out
            outs, sec = timed(run)
            cg = int(sum(sum(o[4][0]["cg_iters"]) for o in outs))
            k = s.profile_cg(20)
            res[name] = {"seconds": round(sec, 4), "cg_iterations": cg, "ms_per_cg_in_solve": round(sec * 1e3 / cg, 4),
                         "cg_kernels_ms": {kk: round(v, 4) for kk, v in k.items()},
                         "cg_iteration_ms": round(sum(k.values()), 4), "pbar_last": [float(v) for v in outs[-1][3][0]]}
            del s
            torch.cuda.empty_cache()
        a, b = res["j2_recomputed"]["pbar_last"], res["j2_stored"]["pbar_last"]
        res["pbar_rel_diff_stored_vs_recomputed"] = float(max(abs(x - y) for x, y in zip(a, b)) / max(abs(v) for v in a))
        emit(res)

    if "oddeven" in which:
        # App. C closes with odd against even grids ("one pixel more"): the
        # paper's cubic inclusion on 31^3 and 32^3 (same 9^3 cube) under simple
        # shear 0.05, the paper's shear 1 and a tensile load, G-hat zero at
        # Nyquist frequencies on both grids and identity there on the even one;
        # then the 2-D example (J2, chi = 2, pure shear to 1.2 in 250
        # increments) on the 451 x 451 stand-in micrograph and its 452 x 452
        # extension, P-bar along the load path
        from paper_1603_08893_amd.fftnk import OPT_NYQUIST
        loads = {"shear_0.05": ms.simple_shear(0.05), "shear_1": ms.simple_shear(1.0),
                 "tension": np.array([[1.03, 0.004, 0.0], [0.002, 1.02, 0.003], [0.0, -0.002, 1.025]]).reshape(9)}
        for lname, Fb in loads.items():
            res = {"extra": "odd_even_cubic_inclusion", "load": lname, "inclusion": 9}
            pb = {}
            for n_, nyq in ((31, 0), (32, 0), (32, 1)):
                s = Solver((n_,) * 3, precision="fp64")
                s.set_phases(ms.cubic_inclusion(n_, 9))
                s.set_material(TABLE)
                s.set_option(OPT_NYQUIST, nyq)
                st, _, _, Pb, S = s.solve_increment(Fb, fields=False, raise_on_error=False)
                key = "%d_%s" % (n_, "identity" if nyq else "zero")
                res[key] = {"status": int(st), "newton_solves": S[0]["n_solves"], "cg_iterations": S[0]["cg_iters"],
                            "pbar": [float(v) for v in Pb[0]]}
                if st == 0:
                    pb[key] = Pb[0]
                del s
            for a, b in (("32_zero", "31_zero"), ("32_identity", "31_zero"), ("32_identity", "32_zero")):
                if a in pb and b in pb:
                    res["pbar_rel_diff_%s_vs_%s" % (a, b)] = float(np.max(np.abs(pb[a] - pb[b])) / np.max(np.abs(pb[b])))
            emit(res)
        odd = ms.micrograph_2d(N=451)
        sched = ms.pure_shear_schedule(250, 1.2)
        traj = {}
        res = {"extra": "odd_even_2d_example", "chi": 2.0, "increments": len(sched)}
        for ph in (odd, ms.extend_by_one_pixel(odd, axes=(0, 1))):
            s = Solver(ph.shape, precision="fp64", j2_stored_tangent=True)
            s.set_phases(ph)
            s.set_material(ms.plane_strain_j2_table(2.0), model=J2)
            t0 = time.perf_counter()
            pbs, newton, status = [], [], 0
            for Fb in sched:
                st, _, _, Pb, S = s.solve_increment(Fb, fields=False, raise_on_error=False)
                if st:
                    status = st
                    break
                pbs.append(Pb[0].copy())
                newton.append(S[0]["n_solves"])
            torch.cuda.synchronize()
            traj[ph.shape[0]] = np.array(pbs)
            res["%d" % ph.shape[0]] = {"status": int(status), "increments_done": len(pbs),
                                       "seconds": round(time.perf_counter() - t0, 2),
                                       "newton_per_increment_mean": round(float(np.mean(newton)), 3),
                                       "pbar_01_every_25": [float(p[1]) for p in pbs[24::25]]}
            print("# oddeven 2-D %d done" % ph.shape[0], file=sys.stderr, flush=True)
            del s
            torch.cuda.empty_cache()
        m = min(len(traj[451]), len(traj[452]))
        if m:
            d = [float(np.max(np.abs(traj[452][k] - traj[451][k])) / np.max(np.abs(traj[451][k]))) for k in range(m)]
            res["pbar_rel_diff_452_vs_451"] = {"max": max(d), "last": d[-1], "every_25": d[24::25]}
        emit(res)

    if "cpu_baseline" in which:
        # the oracle timed on the host beside the GPU path: operator
        # applications at several sizes on one core (GPU operator time of the
        # same cell beside it), the paper's first example solved on one core,
        # and the all-core throughput of independent 64^3 applications
        import oracle
        import os
        import concurrent.futures as cf
        import multiprocessing as mp
        oracle.build()
        for n_ in (32, 64, 96, 128):
            reps = 3 if n_ >= 96 else 5
            t_cpu = _oracle_matvecs((n_, reps, 11))
            ph = (np.random.default_rng(11).random((n_,) * 3) < 0.3).astype(np.uint8)
            s = Solver((n_,) * 3, precision="fp64")
            s.set_phases(ph)
            s.set_material(TABLE)
            s.set_linearization(torch.from_numpy(ms.near_identity_field((n_,) * 3, seed=12, scale=0.01).reshape(-1)))
            p = torch.from_numpy(ms.random_field((n_,) * 3, seed=13).reshape(-1)).to(dev)
            out = s.field()
            for _ in range(3):
                s.apply_operator(p, out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                s.apply_operator(p, out)
            e1.record()
            torch.cuda.synchronize()
            t_gpu = e0.elapsed_time(e1) / 20
            emit({"extra": "cpu_baseline_operator", "grid": n_, "kind": "oracle", "cores": 1,
                  "cpu_ms": round(1e3 * t_cpu / reps, 1), "gpu_ms": round(t_gpu, 4),
                  "ratio": round(1e3 * t_cpu / reps / t_gpu, 1)})
            del s, p, out
        # the paper's first example (31^3, cubic inclusion, simple shear 0.05), one core
        ph = ms.cubic_inclusion(31, 9)
        K, mu = ms.phase_moduli(ph, TABLE)
        c0 = time.perf_counter()
        st, _, _, _, so = oracle.solve_increment(K, mu, oracle.identity_field((31,) * 3), ms.simple_shear(0.05))
        t_cpu = time.perf_counter() - c0
        s = Solver((31,) * 3, precision="fp64")
        s.set_phases(ph)
        s.set_material(TABLE)
        s.solve_increment(ms.simple_shear(0.05), fields=False)
        s.reset_state()
        (_, _, _, _, sg), t_gpu = timed(lambda: s.solve_increment(ms.simple_shear(0.05), fields=False))
        emit({"extra": "cpu_baseline_solve", "grid": 31, "kind": "oracle", "cores": 1, "status": int(st),
              "cpu_s": round(t_cpu, 3), "gpu_s": round(t_gpu, 4), "cg_iters_oracle": so["cg_iters"],
              "cg_iters_gpu": sg[0]["cg_iters"], "ratio": round(t_cpu / t_gpu, 1)})
        del s
        # all cores: independent 64^3 applications in worker processes (spawned)
        workers = max(1, min(16, os.cpu_count() or 1))
        jobs = [(64, 3, 100 + w) for w in range(workers)]
        c0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            t_w = list(ex.map(_oracle_matvecs, jobs))
        t_all = time.perf_counter() - c0
        # throughput over the slowest worker's compute time; the wall time
        # also counts starting the worker processes
        emit({"extra": "cpu_baseline_all_cores", "grid": 64, "kind": "oracle", "cores": workers,
              "matvecs": 3 * workers, "compute_seconds": round(max(t_w), 3),
              "matvecs_per_s": round(3 * workers / max(t_w), 3), "wall_seconds_with_startup": round(t_all, 2)})
        # all cores: the 16 cells of 32^3 of the 64-cell batch, one increment each, dealt out to the workers
        cells = [list(range(16))[w::workers] for w in range(workers)]
        cells = [c for c in cells if c]
        c0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=len(cells), mp_context=mp.get_context("spawn")) as ex:
            res_w = list(ex.map(_oracle_c3_solves, cells))
        t_all = time.perf_counter() - c0
        emit({"extra": "cpu_baseline_all_cores_solves", "cells": "the 16 cells of 32^3 of the 64-cell batch",
              "kind": "oracle", "cores": len(cells), "cell_increments": 16,
              "statuses": [st for _, sts in res_w for st in sts], "compute_seconds": round(max(t for t, _ in res_w), 3),
              "cell_increments_per_s": round(16 / max(t for t, _ in res_w), 4),
              "wall_seconds_with_startup": round(t_all, 2)})

    if "slab" in which:
        # one GPU's share of the 128^3 operator on 8 GPUs split into slabs
        # along a0: passes 1, 2, 4, 5 on a 16 x 128 x 128 slab, pass 3 on the
        # 1/8 of the a0 pencils a GPU holds after the slab -> pencil all-to-all
        # (timed as a 128 x 16 x 128 cell); the two all-to-alls are a model
        # (9 half-spectrum fields x 7/8 per GPU over 7 xGMI links of 153 GB/s)
        def pass_us(shape, k_list):
            s = Solver(shape, precision="fp64")
            s.set_phases((np.random.default_rng(5).random(shape) < 0.3).astype(np.uint8))
            s.set_material(TABLE)
            s.set_linearization(torch.from_numpy(ms.near_identity_field(shape, seed=6, scale=0.01).reshape(-1)))
            p = torch.from_numpy(ms.random_field(shape, seed=7).reshape(-1)).to(dev)
            out = s.field()
            s.apply_operator(p, out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            res = {}
            for k in k_list:
                e0.record()
                for _ in range(50):
                    s.launch_pass(k)
                e1.record()
                torch.cuda.synchronize()
                res[k] = 1e3 * e0.elapsed_time(e1) / 50
            del s, p, out
            torch.cuda.empty_cache()
            return res

        full = pass_us((128, 128, 128), [1, 2, 3, 4, 5])
        slab = pass_us((16, 128, 128), [1, 2, 4, 5])
        pen = pass_us((128, 16, 128), [3])
        local = sum(slab.values()) + pen[3]
        a2a_bytes = 9 * 16 * (128 * 128 * 64) / 8 * 7 / 8  # per GPU and direction, FP64 half spectrum
        a2a_us = a2a_bytes / (7 * 153e9) * 1e6
        emit({"extra": "slab_share", "cell": "128^3 on 8 GPUs (model), FP64", "gpus": 8,
              "full_cell_pass_us": {str(k): round(v, 1) for k, v in full.items()},
              "slab_16x128x128_pass_us": {str(k): round(v, 1) for k, v in slab.items()},
              "pencil_share_128x16x128_pass3_us": round(pen[3], 1),
              "local_us_per_operator": round(local, 1), "full_cell_us_per_operator": round(sum(full.values()), 1),
              "local_vs_full_over_8": round(local / (sum(full.values()) / 8), 3),
              "all_to_all_model_us": round(2 * a2a_us, 1),
              "operator_us_no_overlap": round(local + 2 * a2a_us, 1),
              "operator_us_full_overlap": round(max(local, 2 * a2a_us), 1)})

    if "tune" in which:
        # the plan autotuner: operator time under the default plan and under
        # the policy it picks (20 back-to-back applications each), per cell
        def op_ms(s, shape_list):
            p = s.field()
            p.copy_(torch.from_numpy(np.concatenate(
                [ms.random_field(d, seed=42 + r).reshape(-1) for r, d in enumerate(shape_list)])).to(dev))
            out = s.field()
            for _ in range(3):
                s.apply_operator(p, out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(20):
                s.apply_operator(p, out)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / 20

        cases = [("128^3", [(128,) * 3], "fp64"), ("128^3", [(128,) * 3], "fp32"), ("96^3", [(96,) * 3], "fp64"),
                 ("31^3", [(31,) * 3], "fp64"), ("192^3", [(192,) * 3], "fp64"), ("451x451x2", [(451, 451, 2)], "fp64"),
                 ("batch 32^3+48^3+64^3+96^3", [(32,) * 3, (48,) * 3, (64,) * 3, (96,) * 3], "fp32")]
        for label, shapes, prec in cases:
            s = Solver(shapes if len(shapes) > 1 else shapes[0], precision=prec)
            s.set_phases(np.concatenate([(np.random.default_rng(7 + r).random(d) < 0.3).astype(np.uint8).reshape(-1)
                                         for r, d in enumerate(shapes)]))
            s.set_material(TABLE)
            s.set_linearization(torch.from_numpy(np.concatenate(
                [ms.near_identity_field(d, seed=3 + r, scale=0.01).reshape(-1) for r, d in enumerate(shapes)])).to(dev))
            t0 = op_ms(s, shapes)
            (pol, tuner_ms), sec = timed(lambda: s.autotune(reps=5, use_cache=False))
            t1 = op_ms(s, shapes)
            rec = {"extra": "autotune", "cell": label, "precision": prec, "default_ms": round(t0, 4), "policy": pol,
                   "tuned_ms": round(t1, 4), "speedup": round(t0 / t1, 3), "tuner_seconds": round(sec, 3)}
            if label == "128^3" and prec == "fp64":
                # the spread the tuner chooses from: every policy that changes the launches
                seen, spread = set(), {}
                for q in range(64):
                    if (q >> 3) & 3 == 3:
                        continue
                    d = describe(shapes[0], prec, policy=q)["cells"][0]
                    key = (tuple(a["reg"] for a in d["axes"]), d["rt"], d["rt1"],
                           (d["m64"], d["m32"]) if min(d["axes"][0]["reg"], d["axes"][1]["reg"]) == 0 else None)
                    if key in seen:
                        continue
                    seen.add(key)
                    s.set_plan(q)
                    spread[str(q)] = round(op_ms(s, shapes), 4)
                s.set_plan(pol)
                rec["ms_per_policy"] = spread
            emit(rec)
            del s
            torch.cuda.empty_cache()

    if "nyq" in which:
        # App. C's two choices at Nyquist frequencies on the 128^3 two-phase
        # cell: operator and CG-kernel times, and one tensile increment (with
        # the identity choice the Nyquist rotations only have geometric
        # stiffness: CG needs more iterations, and under shear it breaks down)
        from paper_1603_08893_amd.fftnk import OPT_NYQUIST
        n_ = 128
        phase = ms.grf_threshold(n_, ell=8.0, frac=0.3, seed=1603)
        tension = np.array([[1.03, 0.004, 0.0], [0.002, 1.02, 0.003], [0.0, -0.002, 1.025]]).reshape(9)
        res = {"extra": "nyquist_choice", "grid": n_, "load": tension.tolist()}
        pbars = {}
        for choice in (0, 1):
            s = Solver((n_,) * 3, precision="fp64")
            s.set_phases(phase)
            s.set_material(TABLE)
            s.set_option(OPT_NYQUIST, choice)
            s.solve_increment(tension, fields=False, raise_on_error=False)  # warm-up
            s.reset_state()
            (st, _, _, Pb, stats), sec = timed(lambda: s.solve_increment(tension, fields=False, raise_on_error=False))
            pbars[choice] = Pb[0]
            ms_k = s.profile_cg(20)
            p = s.project(torch.from_numpy(ms.random_field((n_,) * 3, seed=42).reshape(-1)).to(dev))
            out = s.field()
            for _ in range(3):
                s.apply_operator(p, out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                s.apply_operator(p, out)
            e1.record()
            torch.cuda.synchronize()
            res["identity" if choice else "zero"] = {
                "status": int(st), "seconds": round(sec, 4), "newton_solves": stats[0]["n_solves"],
                "cg_iterations": stats[0]["cg_iters"], "operator_ms": round(e0.elapsed_time(e1) / 20, 4),
                "cg_iteration_ms": round(sum(ms_k.values()), 4), "pass3_ms": round(ms_k["pass3"], 4)}
            del s, p, out
            torch.cuda.empty_cache()
        res["pbar_rel_diff"] = float(np.max(np.abs(pbars[1] - pbars[0])) / np.max(np.abs(pbars[0])))
        emit(res)

    if "mixed" in which:
        # mixed control on the 128^3 two-phase cell: uniaxial stress (F11 =
        # 1.02 prescribed with the lower off-diagonal entries, the other
        # stress components zero) in one increment, against a deformation-
        # controlled increment to the Fbar it finds; then the full macroscopic
        # tangent (9 CG solves) at that state
        n_ = 128
        phase = ms.grf_threshold(n_, ell=8.0, frac=0.3, seed=1603)
        mask = np.array([0, 1, 1, 0, 1, 1, 0, 0, 1])
        guess = np.eye(3).reshape(9).copy()
        guess[0] = 1.02
        res = {"extra": "mixed_control", "grid": n_, "mask": mask.tolist(), "F11": 1.02, "tol_stress": 1e-8}
        for prec in ("fp64", "fp32"):
            s = Solver((n_,) * 3, precision=prec)
            s.set_phases(phase)
            s.set_material(TABLE)
            s.solve_increment_mixed(guess, mask, np.zeros(9), 1e-8, fields=False, raise_on_error=False)  # warm-up
            s.reset_state()
            (st, _, _, Pb, Fb, stats, outer), sec = timed(
                lambda: s.solve_increment_mixed(guess, mask, np.zeros(9), 1e-8, fields=False, raise_on_error=False))
            s.reset_state()
            (st2, _, _, Pb2, stats2), sec2 = timed(lambda: s.solve_increment(Fb[0], fields=False,
                                                                            raise_on_error=False))
            C, sec_c = timed(lambda: s.macro_tangent(eta_cg=1e-8))
            res[prec] = {"status": int(st), "seconds": round(sec, 4), "outer_passes": int(outer[0]),
                         "linear_solves": stats[0]["n_solves"], "cg_iterations": int(sum(stats[0]["cg_iters"])),
                         "Fbar": [round(float(v), 8) for v in Fb[0]], "pbar": [float(v) for v in Pb[0]],
                         "deformation_controlled_seconds": round(sec2, 4),
                         "deformation_controlled_cg_iterations": int(sum(stats2[0]["cg_iters"])),
                         "mixed_over_deformation_controlled": round(sec / sec2, 3),
                         "macro_tangent_seconds": round(sec_c, 4),
                         "macro_tangent_C11_C22_C12": [float(C[0][0, 0]), float(C[0][4, 4]), float(C[0][0, 4])]}
            del s
            torch.cuda.empty_cache()
        emit(res)

    if "krylov" in which:
        # the Krylov methods on the 128^3 two-phase cell: one increment
        # (simple shear 0.05, eta_NW 1e-5, eta_CG 1e-8) each, with Chebyshev /
        # Richardson bounds [0.9 min mu, 1.1 max 3K] and GMRES(30)
        n_ = 128
        phase = ms.grf_threshold(n_, ell=8.0, frac=0.3, seed=1603)
        lo = 0.9 * min(m for _, m in TABLE)
        hi = 1.1 * 3 * max(k for k, _ in TABLE)
        res = {"extra": "krylov_methods", "grid": n_, "bounds": [lo, hi], "gmres_restart": 30,
               "load": "simple shear 0.05"}
        for prec in ("fp64", "fp32"):
            for method in ("cg", "chebyshev", "richardson", "gmres"):
                s = Solver((n_,) * 3, precision=prec, gmres_restart=30 if method == "gmres" else 0)
                s.set_phases(phase)
                s.set_material(TABLE)
                s.set_krylov(method, lo, hi)
                s.solve_increment(ms.simple_shear(0.05), fields=False, raise_on_error=False)  # warm-up
                s.reset_state()
                (st, _, _, Pb, stats), sec = timed(lambda: s.solve_increment(ms.simple_shear(0.05), fields=False,
                                                                            raise_on_error=False))
                its = stats[0]["cg_iters"]
                res["%s_%s" % (method, prec)] = {
                    "status": int(st), "seconds": round(sec, 4), "iterations": its,
                    "ms_per_iteration": round(1e3 * sec / max(1, sum(its)), 4), "pbar00": float(Pb[0][0])}
                del s
                torch.cuda.empty_cache()
        emit(res)

    if "c2d" in which:
        # the 2-D example (Sec. 5): plane strain on a 451 x 451 x 2 cell (the
        # thresholded stand-in micrograph), J2 with linear hardening, pure shear
        # to lambda = 1.2 in 250 increments, phase contrasts sqrt(2), 2, 4, 8;
        # cumulative Newton / CG iterations and runtime against the macroscopic
        # equivalent log strain (2 / sqrt(3)) ln(lambda)
        n_, nincr = 451, 250
        ph = ms.micrograph_2d(N=n_)
        sched = ms.pure_shear_schedule(nincr, 1.2)
        for chi in (np.sqrt(2.0), 2.0, 4.0, 8.0):
            s = Solver(ph.shape, precision="fp64", j2_stored_tangent=True)
            s.set_phases(ph)
            s.set_material(ms.plane_strain_j2_table(chi), model=J2)
            s.solve_increment(sched[0], fields=False)  # warm-up (graphs), then start over
            s.reset_state()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            newton, cg, times, status, done = [], [], [], 0, 0
            for k, Fbar in enumerate(sched):
                st, _, _, Pb, stats = s.solve_increment(Fbar, fields=False, raise_on_error=False)
                if st:
                    status = st
                    break
                done += 1
                newton.append(stats[0]["n_solves"])
                cg.append(int(sum(stats[0]["cg_iters"])))
                times.append(time.perf_counter() - t0)
                if (k + 1) % 50 == 0:
                    print("# c2d chi %.3f increment %d %.1fs" % (chi, k + 1, times[-1]), file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            eps_p = s.get_history().view(7, -1)[6].view(n_, n_, 2)[:, :, 0].cpu().numpy()
            hard = ph[:, :, 0] == 1
            marks = list(range(24, done, 25))
            lam = [1.0 + 0.2 * (k + 1) / nincr for k in marks]
            emit({"extra": "c2d_plane_strain", "grid": [n_, n_, 2], "chi": round(float(chi), 4),
                  "hard_fraction": round(float(hard.mean()), 4), "increments_done": done, "status": int(status),
                  "seconds": round(sec, 3), "increments_per_s": round(done / sec, 3),
                  "newton_per_increment_mean": round(float(np.mean(newton)), 3),
                  "newton_per_increment_max": int(max(newton)),
                  "newton_iterations_by_increment": newton,
                  "eps_bar": [round(2 / np.sqrt(3) * np.log(l), 5) for l in lam],
                  "cumulative_newton": [int(np.sum(newton[:k + 1])) for k in marks],
                  "cumulative_cg": [int(np.sum(cg[:k + 1])) for k in marks],
                  "cumulative_seconds": [round(times[k], 3) for k in marks],
                  "max_eps_p_soft": float(eps_p[~hard].max()), "max_eps_p_hard": float(eps_p[hard].max()),
                  "pbar_last": [float(v) for v in Pb[0]]})
            del s
            torch.cuda.empty_cache()

    if "c3" in which:
        # 64 cells of four sizes, each with its own spheres, contrast and load,
        # one increment.  In two cells (33 and 41, 64^3, contrast 16 and 13)
        # the St. Venant-Kirchhoff tangent turns indefinite before the full
        # load is reached (compressive loads; the model is not rank-one convex
        # under strong compression): CG breaks down there, the oracle breaks
        # down in the same iteration, and load steps do not help (in four
        # steps cell 33 fails in the last one).  They are reported as failed.
        t0 = time.perf_counter()
        items = ms.c3_batch()
        print("# c3 inputs %.1fs" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
        dims = [(it["N"],) * 3 for it in items]
        ph = np.concatenate([(it["phase"].reshape(-1) + 2 * r).astype(np.uint8) for r, it in enumerate(items)])
        table = [row for it in items for row in it["table"]]
        nsub = 1
        Fb = [np.array([(np.eye(3).reshape(9) + (k + 1) / nsub * (it["Fbar"] - np.eye(3).reshape(9)))
                        for it in items]) for k in range(nsub)]
        res = {"extra": "c3_batched", "cells": len(items), "increments": nsub,
               "voxels": int(sum(np.prod(d) for d in dims)),
               "volume_fractions": [round(it["frac"], 4) for it in items]}

        def run(s):
            s.reset_state()
            out = []
            for k in range(nsub):
                out.append(s.solve_increment(Fb[k], fields=False, raise_on_error=False))
            return out

        pbars = {}
        for prec in ("fp64", "fp32"):
            s = Solver(dims, precision=prec)
            s.set_phases(ph)
            s.set_material(table)
            run(s)  # warm-up: graphs, caches
            outs, sec = timed(lambda: run(s))
            stats = [x for o in outs for x in o[4]]
            pbars[prec] = outs[-1][3]
            res[prec] = {"seconds": round(sec, 4), "cell_increments_per_s": round(nsub * len(items) / sec, 2),
                         "failed_cells": [r for r in range(len(items)) if any(o[4][r]["status"] for o in outs)],
                         "newton_solves": int(sum(x["n_solves"] for x in stats)),
                         "cg_iterations": int(sum(sum(x["cg_iters"]) for x in stats)),
                         "max_cg_per_solve": int(max(max(x["cg_iters"]) for x in stats))}
            print("# c3 %s %.2fs" % (prec, sec), file=sys.stderr, flush=True)
            del s
            torch.cuda.empty_cache()
        ok = [r for r in range(len(items)) if r not in res["fp64"]["failed_cells"] + res["fp32"]["failed_cells"]]
        res["fp32_pbar_rel_diff_vs_fp64"] = float(max(np.max(np.abs(pbars["fp32"][r] - pbars["fp64"][r])) /
                                                  np.max(np.abs(pbars["fp64"][r])) for r in ok))

        # the plain FP64 path: the same cells one after another, one context per size
        def one_by_one():
            for n_ in sorted(set(it["N"] for it in items)):
                s = Solver((n_,) * 3, precision="fp64")
                for r, it in enumerate(items):
                    if it["N"] != n_:
                        continue
                    s.set_phases(it["phase"])
                    s.set_material(it["table"])
                    s.reset_state()
                    for k in range(nsub):
                        s.solve_increment(Fb[k][r], fields=False, raise_on_error=False)
                del s
        one_by_one()  # warm-up
        _, sec1 = timed(one_by_one)
        res["fp64_one_by_one"] = {"seconds": round(sec1, 4), "cell_increments_per_s": round(nsub * len(items) / sec1, 2)}
        res["speedup_batched_fp32_vs_one_by_one_fp64"] = round(sec1 / res["fp32"]["seconds"], 3)
        res["speedup_batched_fp64_vs_one_by_one_fp64"] = round(sec1 / res["fp64"]["seconds"], 3)
        emit(res)
        torch.cuda.empty_cache()

    if "c4" in which:
        # finite-strain J2 at 96^3: spheres at 25 %, simple shear to 0.1 in 20 increments
        ph, frac = ms.rsa_spheres(96, 0.25, seed=1604)
        s = Solver((96,) * 3, precision="fp64", j2_stored_tangent=True)
        s.set_phases(ph)
        s.set_material([(ms.K_SOFT, ms.MU_SOFT, 0.003, 0.01), (ms.K_SOFT, ms.MU_SOFT, 0.006, 0.01)], model=J2)
        sched = ms.c4_schedule(20, 0.1)
        s.solve_increment(sched[0], fields=False)  # warm-up
        s.reset_state()
        solves, cgs, status, done = [], [], 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for Fbar in sched:
            st, _, _, Pb, stats = s.solve_increment(Fbar, fields=False, raise_on_error=False)
            if st:
                status = st
                break
            done += 1
            solves.append(stats[0]["n_solves"])
            cgs.append(int(sum(stats[0]["cg_iters"])))
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        eps_p = s.get_history().view(7, -1)[6]
        emit({"extra": "c4_j2", "grid": 96, "sphere_fraction": round(frac, 4), "increments_done": done,
              "status": int(status), "seconds": round(sec, 3), "increments_per_s": round(done / sec, 3),
              "newton_solves_per_increment": solves, "cg_iterations_per_increment": cgs,
              "pbar_last": [float(v) for v in Pb[0]], "plastic_voxel_fraction": float((eps_p > 0).float().mean()),
              "max_eps_p": float(eps_p.max())})
        del s
        torch.cuda.empty_cache()

    if "c5" in which:
        # adjoint: 8 load cases on 192^3 with a log-normal shear-modulus field
        n_ = 192
        mu = torch.from_numpy(ms.lognormal_field(n_, 0.5, 8.0, seed=1605)).to(dev)
        mu_t = torch.from_numpy(ms.lognormal_field(n_, 0.5, 8.0, seed=1606)).to(dev)
        cases = np.array(ms.c5_load_cases(0.05))
        s = Solver([(n_,) * 3] * len(cases), precision="fp64")
        s.set_phases(np.zeros(len(cases) * n_ ** 3, dtype=np.uint8))
        s.set_material([(ms.K_SOFT, ms.MU_SOFT)])
        with torch.no_grad():
            target, sec_t = timed(lambda: homogenized_stress(mu_t, s, cases))
        m = mu.clone().requires_grad_(True)
        Pb, sec_f = timed(lambda: homogenized_stress(m, s, cases))
        loss = ((Pb - target) ** 2).sum()
        _, sec_b = timed(lambda: loss.backward())
        emit({"extra": "c5_adjoint", "grid": n_, "load_cases": len(cases),
              "forward_seconds": round(sec_f, 3), "backward_seconds": round(sec_b, 3),
              "target_forward_seconds": round(sec_t, 3),
              "forward_cell_solves_per_s": round(len(cases) / sec_f, 3),
              "backward_over_forward": round(sec_b / sec_f, 3), "loss": float(loss.detach()),
              "grad_norm": float(m.grad.norm()), "grad_abs_max": float(m.grad.abs().max())})


if __name__ == "__main__":
    main()
