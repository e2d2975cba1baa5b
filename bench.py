"""Benchmark of the Lax / Hopf solver on one MI355X.

One step = one hj_solve call over the whole workload: every (point, guess)
slot runs its descent with restarts, the certificate, and the selection over
guesses.  The headline workload is the n=10 Hopf problem (4096 points in
[-3,3]^10, 16 guesses, 128 RK4 steps with the RK4-augmented quadrature,
adjoint-gradient descent, 200 iterations, certificate tolerance 1e-8); the
same workload is also run once with central-difference coordinate descent
for the adjoint-vs-FD speedup.

Prints ONE JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "certified u(x,t) solves/sec at n=10,32; adjoint vs central-FD descent speedup"
PEAK_FP64_VECTOR_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic work per unit (FMA = 2 flops, tanh or a division = 1), for
# H without drift in dimension n:
#   one RK4 stage of the forward solve:  16 n + 16
#   one stage of the adjoint sweep:      20 n + 14
# A forward solve is N steps of 4 stages, an adjoint sweep N steps of 4
# adjoint stages.  Recomputation inside the checkpointed adjoint is not
# counted: it is overhead of the implementation, not work of the method.
def fwd_flops(n, N):
    return N * 4 * (16 * n + 16)


def adj_flops(n, N):
    return N * 4 * (20 * n + 14)


def algorithmic_flops(wl, slot_fwd, slot_bwd):
    return float(slot_fwd.sum()) * fwd_flops(wl.n, wl.nsteps) + \
        float(slot_bwd.sum()) * adj_flops(wl.n, wl.nsteps)


def run_gpu(wl, steps, warmup, label, cfg=None):
    import torch
    from paper_1704_02524_amd import hj
    x, g = hj.device_inputs(wl)
    out = None
    for i in range(warmup):
        out = hj.solve(wl, x, g, out=out, **(cfg or {}))
        torch.cuda.synchronize()
        log(f"{label}: warmup {i + 1}/{warmup} done")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        # torch creates an event on its first record; the library then
        # re-records the same events around its descent kernel
        a.record()
        b.record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        out = hj.solve(wl, x, g, out=out, events=evs[i], **(cfg or {}))
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    log(f"{label}: {steps} steps, {wall * 1e3:.1f} ms/step, kernel "
        f"{np.mean(kern_ms):.1f} ms")
    host = {k: v.cpu().numpy() for k, v in out.items()}
    return wall, kern_ms, host


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 reference, single-threaded, on a prefix of the points with all
    their guesses, until about budget_s seconds of work."""
    from oracle.oracle import Oracle, build
    build()
    o = Oracle.from_workload(wl)
    O = Oracle.opts_from_workload(wl)
    t0 = time.perf_counter()
    n_pts = n_cert = 0
    while time.perf_counter() - t0 < budget_s and n_pts < wl.B:
        sub = wl.subset(n_pts, n_pts + 1)
        r = o.solve(sub.x, sub.guesses, O, diag=False)
        n_cert += int(r["cert"][0] == 1)
        n_pts += 1
    dt = time.perf_counter() - t0
    return dict(value=n_cert / dt, unit="certified solves/s", cores=1, kind="oracle",
                sample=f"first {n_pts} points of the same workload with all {wl.G} guesses "
                       f"({dt:.1f} s, {n_cert} certified), FP64 reference, 1 thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=4096)
    ap.add_argument("--no-cd", action="store_true", help="skip the central-FD comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference baseline")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default launch shape")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 "
                                   "(queries are independent: shard points across "
                                   "processes to use more GPUs)"}))
        sys.exit(2)

    import torch
    from paper_1704_02524_amd import tune
    from paper_1704_02524_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    wl = W.c1_hopf_n10(B=args.points, mode=W.GD_ADJ)
    log(f"workload {wl.name}: B={wl.B} G={wl.G} n={wl.n} N={wl.nsteps}")
    cfg = {} if args.no_tune else tune.tune(wl, verbose=True)
    log(f"launch configuration: {cfg or 'library default'}")
    wall, kern, host = run_gpu(wl, args.steps, args.warmup, "adjoint GD", cfg)
    n_cert = int((host["cert"] == 1).sum())
    value = n_cert / wall
    flops = algorithmic_flops(wl, host["slot_fwd"], host["slot_bwd"])
    k_s = float(np.mean(kern)) / 1e3
    achieved = flops / k_s / 1e12

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "certified solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: Hopf, n={wl.n}, {wl.B} points U[-3,3]^n, {wl.G} "
                        f"guesses N(0,I) (+2 restarts), t={wl.t}, {wl.nsteps} RK4 steps, "
                        f"RK4-augmented quadrature, adjoint gradient descent, "
                        f"{wl.max_iter} iterations, certificate tol {wl.cert_tol:g}",
            "points": wl.B, "guesses": wl.G, "n": wl.n, "nsteps": wl.nsteps,
            "certified_points": n_cert,
        },
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": None,
            "kernel": "k_solve_gd", "launch": cfg, "kernel_ms": float(np.mean(kern)),
            "algorithmic_flops_per_launch": flops,
        },
    }
    if not args.no_cd:
        wcd = wl.with_(mode=W.CD_FD)
        cfg_cd = {} if args.no_tune else tune.tune(wcd, tune_iters=2, verbose=True)
        log(f"launch configuration (CD): {cfg_cd or 'library default'}")
        wall_cd, kern_cd, host_cd = run_gpu(wcd, 1, 0, "central-FD CD", cfg_cd)
        fin = (host["cert"] >= 0) & (host_cd["cert"] >= 0)
        du = np.abs(host["u"][fin] - host_cd["u"][fin]) / np.maximum(1, np.abs(host["u"][fin]))
        flops_cd = algorithmic_flops(wcd, host_cd["slot_fwd"], host_cd["slot_bwd"])
        result["cd_fd"] = {
            "ms_per_step": wall_cd * 1e3,
            "certified_points": int((host_cd["cert"] == 1).sum()),
            "value": int((host_cd["cert"] == 1).sum()) / wall_cd,
            "achieved_tflops": flops_cd / (kern_cd[0] / 1e3) / 1e12,
            "max_rel_u_diff_vs_adjoint": float(du.max(initial=0.0)),
        }
        result["speedup_adjoint_vs_cd"] = wall_cd / wall
    if not args.no_cpu:
        log("CPU reference baseline ...")
        result["cpu_baseline"] = cpu_baseline(wl)
        log(f"CPU: {result['cpu_baseline']['value']:.3f} certified solves/s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
