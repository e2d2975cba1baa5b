"""Benchmark of the Lax / Hopf solver on one MI355X.

One step = one pass of the whole solve over the workload: every (point,
guess) slot runs its descent with restarts, the certificate, and the
selection over guesses (hj_solve; for the batched workload one replay of the
captured plan).  The default workload is the n=10 Hopf problem (4096 points
in [-3,3]^10, 16 guesses, 128 RK4 steps with the RK4-augmented quadrature,
adjoint-gradient descent, 200 iterations, certificate tolerance 1e-8); it is
also run once with central-difference coordinate descent for the
adjoint-vs-FD speedup.  --workload selects the other configurations
(n=32 linear drift in FP64 or FP32, n=100 FP32, n=2 Lax with coordinate
descent, 64 batched uneven instances).

Prints ONE JSON line.  Progress goes to stderr.
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
# MI355X published peaks (dense), TFLOP/s
PEAK = {("alu", "f64"): 78.6, ("alu", "f32"): 157.3, ("mfma", "f64"): 78.6,
        ("mfma", "f32"): 157.3}
WORKLOADS = ("hopf_n10", "lax_n32_drift", "lax_n32_drift_f32", "lax_n100_f32", "lax_n2",
             "batched", "batched_f32", "paper", "lax_friedrichs")

# The paper's section 5 runtimes (C++, one core of a 1.7 GHz Intel Core
# i7-4650U; "a x 10^-c s x k" per point with k guesses): point solves per
# second = 1 / (a 10^-c k).  Context for the like-for-like examples below,
# not a target (other hardware).
PAPER_RUNTIME = {
    "paper_ex2_minus_d2": 2.366e-5 * 5, "paper_ex2_plus_d2": 2.605e-5 * 5,
    "paper_ex2_minus_d7": 3.717e-4 * 5, "paper_ex2_rosenbrock": 3.847e-5,
    "paper_ex3_plus_d2": 6.865e-4 * 5, "paper_ex3_minus_d2": 1.417e-3 * 5,
    "paper_ex3_minus_d10": 2.470e-2 * 5, "paper_ex5_d2": 9.094e-2 * 20,
    "paper_ex5_d7": 5.428e-1 * 20,
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic work (FMA = 2 flops, tanh or a division = 1), the count the
# roofline uses: an RK4 stage costs F = 16 n + 4 n^2 [drift] + 12, a step
# 4 F + 12, a solve N steps; a gradient-descent iteration is the trial
# evaluation plus, when the step is accepted, one recomputation of the
# checkpointed trajectory and a vector-Jacobian sweep worth about 1.75
# solves (3.75 solves in all; 3.1 with drift, whose matrix products dominate
# both directions alike); a coordinate-descent sweep is 3n solves.
def method_flops(wl, slot_fwd, slot_bwd):
    dr = wl.A is not None
    f_st = 16 * wl.n + (4 * wl.n * wl.n if dr else 0) + 12
    per_solve = wl.nsteps * (4 * f_st + 12)
    bwd = 2.1 if dr else 2.75
    return (float(slot_fwd.sum()) + bwd * float(slot_bwd.sum())) * per_solve


# The kernel's own, tighter count, beside it: per dimension n
#   one RK4 stage of the forward solve:  16 n + 16
#   one stage of the adjoint sweep:      20 n + 14
# and with a drift matrix A in addition
#   forward stage: A gamma and A^T p (2 x 2 n^2) and their four updates (8 n)
#   adjoint stage: A^T lambda_gamma and A lambda_p (2 x 2 n^2) and 4 n;
# the recomputation inside the checkpointed adjoint is not counted.
def fwd_flops(n, N, drift=False):
    return N * 4 * (16 * n + 16 + ((4 * n * n + 8 * n) if drift else 0))


def adj_flops(n, N, drift=False):
    return N * 4 * (20 * n + 14 + ((4 * n * n + 4 * n) if drift else 0))


def own_flops(wl, slot_fwd, slot_bwd):
    dr = wl.A is not None
    return float(slot_fwd.sum()) * fwd_flops(wl.n, wl.nsteps, dr) + \
        float(slot_bwd.sum()) * adj_flops(wl.n, wl.nsteps, dr)


def _code_only(text):
    """C/C++ source without comments and blank lines (the sources hold no
    comment markers inside string literals)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def source_digest():
    """Digest of the code of the kernel sources and the C header, comments
    left out (identifies the build that counter measurements were taken
    on)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1704_02524_amd", "csrc")
    paths = [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith((".hip", ".hpp"))]
    for path in paths + [os.path.join(ROOT, "include", "hj.h")]:
        h.update(os.path.basename(path).encode())
        with open(path, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, launch):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/hbm_traffic.md: FETCH_SIZE and WRITE_SIZE, each scaled
    by what the counter reads for a device copy of known size), when it was
    taken on the current kernel sources with the same launch configuration;
    otherwise None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    try:
        with open(path) as f:
            txt = f.read()
        block = txt.split("```json", 1)[1].split("```", 1)[0]
        entries = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    dig = source_digest()
    for e in entries:
        if e.get("workload") == workload and e.get("source_digest") == dig and \
                e.get("launch") == launch:
            return e["fetch_kib"] * 1024 * e["fetch_factor"] + \
                e["write_kib"] * 1024 * e["write_factor"]
    return None


def phase_record(wl, host, launch, workload):
    """Executed instructions of the dominant kernels traced to their phases:
    instructions per step of the forward, recompute and reverse loops (static
    counts from the kernels' assembly, profiles/isa_phases_<workload>.md,
    used only while the kernel-source digest matches) times the steps each
    launch executed in each phase (lane-steps, from the per-slot forward and
    adjoint counts), beside each phase's algorithmic flops per step.  With a
    tail hand-off, a slot's first `tail_budget` evaluations ran in the
    descent launch and the rest in the continuation (its adjoint sweeps
    split in the same proportion, an estimate), on tail_lanes_per_task
    lanes each."""
    path = os.path.join(ROOT, "profiles", f"isa_phases_{workload}.md")
    try:
        with open(path) as f:
            e = json.loads(f.read().split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if e.get("source_digest") != source_digest() or wl.A is not None:
        return None
    N, n = wl.nsteps, wl.n
    K = int(launch.get("ckpt_K", 0) or 0)
    budget = int(launch.get("tail_budget", 0) or 0)
    ks = e["kernels"]
    first = ks["handoff"] if budget > 0 else ks["descent"]
    if K < 1 or first["lpt"] != launch.get("lanes_per_task"):
        return None
    fwd = host["slot_fwd"].astype(float)
    bwd = host["slot_bwd"].astype(float)
    launches = [("descent", first, fwd, bwd, 1)]
    if budget > 0:
        tail = ks.get("tail")
        if tail is None or tail["lpt"] != launch.get("tail_lanes_per_task"):
            return None
        f1 = np.minimum(fwd, budget)
        b1 = bwd * np.where(fwd > 0, f1 / np.maximum(fwd, 1), 1.0)
        launches = [("descent", first, f1, b1, 1), ("tail", tail, fwd - f1, bwd - b1, tail["lpt"])]
    step = 4 * (16 * n + 12) + 12
    alg = {"forward": step, "recompute": step, "reverse": 1.75 * step}
    out = {"source": "instructions per step from the kernels' assembly x lane-steps executed"}
    tot = 0.0
    for name, k, f, b, lanes in launches:
        steps = {"forward": f.sum() * N, "recompute": b.sum() * (N - (N + K - 1) // K),
                 "reverse": b.sum() * N}
        rec = {"shape": f"{k['npl']}x{k['lpt']}"}
        for ph in steps:
            c = k["phases"][ph]
            valu = c["fp64"] + c["agpr"] + c["valu_other"]
            rec[ph] = {"lane_steps": steps[ph] * lanes, "valu_per_step": valu,
                       "fp64_per_step": c["fp64"], "agpr_moves_per_step": c["agpr"],
                       "method_flops_per_step": alg[ph]}
            tot += steps[ph] * lanes * valu
        out[name] = rec
    for name, *_ in launches:
        for ph in ("forward", "recompute", "reverse"):
            r = out[name][ph]
            r["valu_share"] = r["lane_steps"] * r["valu_per_step"] / tot
    out["launch_lane_valu"] = tot
    return out


def _events(k):
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(k)]
    for a, b in evs:
        # torch creates an event on its first record; the library then
        # re-records the same events around its descent kernel
        a.record()
        b.record()
    torch.cuda.synchronize()
    return evs


def run_gpu(wl, steps, warmup, label, cfg=None):
    import torch
    from paper_1704_02524_amd import hj
    x, g = hj.device_inputs(wl)
    out = None
    for i in range(warmup):
        out = hj.solve(wl, x, g, out=out, **(cfg or {}))
        torch.cuda.synchronize()
        log(f"{label}: warmup {i + 1}/{warmup} done")
    evs = _events(steps)
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


def run_batched(wls, steps, warmup, group_cfg=None):
    """Replays of one captured plan; the events bracket the whole graph on
    the stream it is launched on."""
    import torch
    from paper_1704_02524_amd import hj
    plan = hj.BatchPlan(wls, group_cfg=group_cfg)
    log(f"batched plan: {plan.info()}")
    for i in range(warmup):
        plan.run()
        torch.cuda.synchronize()
        log(f"batched: warmup {i + 1}/{warmup} done")
    evs = _events(steps)
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record()
        outs = plan.run()
        evs[i][1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    log(f"batched: {steps} steps, {wall * 1e3:.1f} ms/step, graph {np.mean(kern_ms):.1f} ms")
    hosts = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    info = plan.info()
    plan.free()
    return wall, kern_ms, hosts, info


def cpu_baseline_slots(wls, budget_s=15.0):
    """The FP64 reference, single-threaded in this process, on (point, guess)
    slots taken in order (points in turn from the instances), until about
    budget_s seconds of work (the batched workloads).  Rate: certified slots
    / G per second, i.e. point solves per second when a point's G slots are
    solved in turn (a point counts as certified once any of its slots is,
    so this does not overstate it)."""
    from oracle.oracle import Oracle, build
    build()
    oracles = [(Oracle.from_workload(w), Oracle.opts_from_workload(w)) for w in wls]
    t0 = time.perf_counter()
    n_slots = n_cert = 0
    nxt = [0] * len(wls)  # next slot index (point * G + guess) per instance
    i = 0
    while time.perf_counter() - t0 < budget_s and \
            any(nxt[j] < wls[j].B * wls[j].G for j in range(len(wls))):
        j = i % len(wls)
        w = wls[j]
        if nxt[j] >= w.B * w.G:
            i += 1
            continue
        b, g = divmod(nxt[j], w.G)
        nxt[j] += 1
        if nxt[j] % w.G == 0:
            i += 1  # next instance after a whole point
        sub = w.subset(b, b + 1)
        o, O = oracles[j]
        r = o.solve(sub.x, sub.guesses[:, g:g + 1], O, diag=False)
        n_cert += int(r["cert"][0] == 1)
        n_slots += 1
    dt = time.perf_counter() - t0
    G = wls[0].G
    return dict(value=n_cert / G / dt, unit="certified solves/s", cores=1, kind="oracle",
                sample=f"{n_slots} (point, guess) slots of points taken in turn from the "
                       f"{len(wls)} instances ({dt:.1f} s, {n_cert} certified), FP64 "
                       f"reference, 1 thread; rate = certified slots / {G} guesses per second")


def host_cores():
    """Cores of this host's share: the affinity mask, at most 16 (the CPU
    share of one GPU on the measurement boxes)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_points(name, budget_s, workers):
    """The FP64 reference on whole points of a single-instance workload, in
    `workers` processes over disjoint points (worker w: points w, w +
    workers, ...), each until about budget_s seconds; rate = certified points
    over the wall time of the slowest worker.  Also the one-process rate."""
    import subprocess
    from oracle.oracle import build
    build()

    def run(k):
        procs = [subprocess.Popen([sys.executable, "-m", "oracle.cpu_rate", name, str(w), str(k),
                                   str(budget_s)], cwd=ROOT, stdout=subprocess.PIPE, text=True)
                 for w in range(k)]
        outs = []
        for pr in procs:
            out, _ = pr.communicate(timeout=budget_s * 4 + 120)
            if pr.returncode != 0:
                raise RuntimeError(f"oracle worker failed ({pr.returncode})")
            outs.append(json.loads(out.strip().splitlines()[-1]))
        return outs

    one = run(1)[0]
    many = run(workers)
    wall = max(o["seconds"] for o in many)
    pts = sum(o["points"] for o in many)
    cert = sum(o["certified"] for o in many)
    return dict(value=cert / wall, unit="certified solves/s", cores=workers, kind="oracle",
                sample=f"{pts} whole points of the same workload (all guesses and restarts), "
                       f"{workers} processes of the FP64 reference over disjoint points, "
                       f"{wall:.1f} s wall, {cert} certified",
                single_thread={"value": one["certified"] / one["seconds"], "cores": 1,
                               "points": one["points"], "seconds": one["seconds"]})


def copy_probe(nbytes):
    """A device-to-device copy of nbytes, so that a counter run over this
    process also sees a kernel of known traffic (nbytes read, nbytes
    written) to scale FETCH_SIZE / WRITE_SIZE by."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: {nbytes} bytes device to device")
    del a, b


def describe(wl):
    from paper_1704_02524_amd import workloads as W
    form = "Lax" if wl.formula == W.LAX else "Hopf"
    quad = "RK4-augmented" if wl.quad == W.RK4AUG else "trapezoid"
    mode = "adjoint gradient descent" if wl.mode == W.GD_ADJ else \
        "central-FD coordinate descent"
    lo, hi = float(wl.x.min()), float(wl.x.max())
    drift = ", linear drift <Ax,p> (A on the matrix cores)" if wl.A is not None else ""
    prec = "FP64" if wl.dtype == W.F64 else ("FP32 with FP64 certificate" if wl.cert_fp64
                                             else "FP32")
    return (f"{wl.name}: {form}, n={wl.n}{drift}, {wl.B} points U[{lo:.0f},{hi:.0f}]^n, "
            f"{wl.G} guesses (+{wl.R_max} restarts), t={wl.t:g}, {wl.nsteps} RK4 steps, "
            f"{quad} quadrature, {mode}, {wl.max_iter} iterations, certificate tol "
            f"{wl.cert_tol:g}, {prec}")


def build_workloads(name, points):
    from paper_1704_02524_amd import workloads as W
    if name == "hopf_n10":
        return [W.c1_hopf_n10(B=points or 4096, mode=W.GD_ADJ)]
    if name == "lax_n32_drift":
        return [W.c3_drift_n32(B=points or 65536)]
    if name == "lax_n32_drift_f32":
        return [W.c3_drift_n32(B=points or 65536, dtype=W.F32)]
    if name == "lax_n100_f32":
        return [W.c4_lax_n100(B=points or 262144)]
    if name == "lax_n2":
        return [W.c0_lax_n2(B=points or 1024)]
    if name in ("batched", "batched_f32"):
        return W.c2_batched(dtype=W.F32 if name == "batched_f32" else W.F64,
                            max_points=points)
    raise ValueError(name)


def roofline_of(wl, host, kern_ms, cfg, workload, kernel):
    """The dominant kernel against its roofline: algorithmic flops of one
    launch over its HIP-event duration (and the same on the scope table's
    count)."""
    from paper_1704_02524_amd import workloads as W
    dtype = "f64" if wl.dtype == W.F64 else "f32"
    bound = "mfma" if wl.A is not None else "alu"
    peak = PEAK[(bound, dtype)]
    k_s = float(np.mean(kern_ms)) / 1e3
    flops = method_flops(wl, host["slot_fwd"], host["slot_bwd"])
    flops_own = own_flops(wl, host["slot_fwd"], host["slot_bwd"])
    rec = roofline_record(bound, peak, k_s, flops, flops_own, measured_traffic(workload, cfg),
                          kernel, cfg)
    ph = phase_record(wl, host, cfg, workload)
    if ph is not None:
        rec["phases"] = ph
    return rec


METHOD_COUNT = ("RK4 stage 16n + 4n^2 [drift] + 12, step 4 stages + 12, solve N steps, "
                "GD iteration 3.75 solves (3.1 with drift) incl. the adjoint's recomputation, "
                "CD sweep 3n solves; FMA = 2, tanh or division = 1")
OWN_COUNT = ("per evaluation N x 4 x (16n + 16 [+ 4n^2 + 8n drift]), per adjoint sweep "
             "N x 4 x (20n + 14 [+ 4n^2 + 4n drift]); the adjoint's recomputation excluded")


def roofline_record(bound, peak, k_s, flops, flops_own, traffic, kernel, launch):
    """The roofline object: achieved = the algorithmic flops of one launch
    (method_flops) over the launch's HIP-event duration; the kernel's own,
    smaller count (no recomputation) beside it."""
    return {
        "bound": bound, "achieved": flops / k_s / 1e12, "peak": peak, "unit": "TFLOP/s",
        "frac": flops / k_s / 1e12 / peak, "traffic": traffic,
        "kernel": kernel, "launch": launch, "kernel_ms": k_s * 1e3,
        "algorithmic_flops_per_launch": flops, "flop_count": METHOD_COUNT,
        "own_count": {"flops_per_launch": flops_own, "achieved": flops_own / k_s / 1e12,
                      "frac": flops_own / k_s / 1e12 / peak, "flop_count": OWN_COUNT},
    }


def cd_comparison(wl, host, wall, cd_points, tune_cd):
    """Central-difference coordinate descent on the same GPU, on the first
    cd_points points (all of them when None).  The speedup is the ratio of
    certified solves per second; accuracy is compared on the points both
    descents certify."""
    from paper_1704_02524_amd import tune
    from paper_1704_02524_amd import workloads as W
    wcd = wl.with_(mode=W.CD_FD)
    if cd_points:
        wcd = wcd.subset(0, min(cd_points, wl.B))
    cfg_cd = tune.tune(wcd, tune_iters=2, verbose=True) if tune_cd else {}
    if wl.A is not None:
        cfg_cd = {}  # the matrix-core layout has one lane shape
    log(f"launch configuration (CD): {cfg_cd or 'library default'}")
    wall_cd, kern_cd, host_cd = run_gpu(wcd, 1, 0, "central-FD CD", cfg_cd)
    m = wcd.B
    both = (host["cert"][:m] == 1) & (host_cd["cert"] == 1)
    du = np.abs(host["u"][:m][both] - host_cd["u"][both]) / \
        np.maximum(1, np.abs(host["u"][:m][both]))
    tol = 1e-9 if wl.dtype == W.F64 else 1e-4
    cert_gd = int((host["cert"] == 1).sum())
    cert_cd = int((host_cd["cert"] == 1).sum())
    rate_gd = cert_gd / wall
    rate_cd = cert_cd / wall_cd
    flops_cd = method_flops(wcd, host_cd["slot_fwd"], host_cd["slot_bwd"])
    return {
        "cd_fd": {
            "points": m, "launch": cfg_cd, "ms_per_step": wall_cd * 1e3,
            "certified_points": cert_cd, "certified_fraction": cert_cd / m,
            "certified_fraction_adjoint": float((host["cert"][:m] == 1).mean()),
            "value": rate_cd, "achieved_tflops": flops_cd / (kern_cd[0] / 1e3) / 1e12,
            "points_both_certified": int(both.sum()),
            "max_rel_u_diff_vs_adjoint": float(du.max(initial=0.0)),
            "equal_accuracy": bool(du.max(initial=0.0) <= tol),
            "fewer_certified_than_adjoint": bool(cert_cd < int((host["cert"][:m] == 1).sum())),
        },
        # certified solves per second, adjoint over central differences
        "speedup_adjoint_vs_cd": rate_gd / rate_cd if rate_cd > 0 else None,
    }


def measure_single(wl, workload, steps, warmup, cfg):
    """One single-instance workload: timed solves, certified rate, roofline."""
    from paper_1704_02524_amd import workloads as W
    log(f"workload {wl.name}: B={wl.B} G={wl.G} n={wl.n} N={wl.nsteps}")
    log(f"launch configuration: {cfg or 'library default'}")
    mode_name = "adjoint GD" if wl.mode == W.GD_ADJ else "central-FD CD"
    wall, kern, host = run_gpu(wl, steps, warmup, mode_name, cfg)
    n_cert = int((host["cert"] == 1).sum())
    kernel = "k_solve_gd" if wl.mode == W.GD_ADJ else "k_solve_cd"
    if cfg.get("tail_budget"):
        kernel = (f"k_solve_gd with a tail hand-off after {cfg['tail_budget']} evaluations + "
                  f"k_solve_gd continuation on {cfg.get('tail_lanes_per_task', 2)} lanes per "
                  f"task (the interval between the events spans both launches)")
    return {
        "value": n_cert / wall, "unit": "certified solves/s", "ms_per_step": wall * 1e3,
        "dtype": "f64" if wl.dtype == W.F64 else "f32",
        "config": {"workload": describe(wl), "points": wl.B, "guesses": wl.G, "n": wl.n,
                   "nsteps": wl.nsteps, "certified_points": n_cert},
        "roofline": roofline_of(wl, host, kern, cfg, workload, kernel),
    }, wall, host


def paper_examples(grid):
    """The paper's section 5 examples with its own scheme (forward Euler,
    rectangle rule, forward differences, Algorithm 1), its step sizes,
    constants and numbers of guesses, on a grid x grid cross-section."""
    from paper_1704_02524_amd import workloads as W
    return [
        W.paper_ex2(-1, n=2, t=0.5, grid=grid), W.paper_ex2(1, n=2, t=0.5, grid=grid),
        W.paper_ex2(-1, n=7, t=0.2, grid=grid), W.paper_ex2_rosenbrock(grid=grid),
        W.paper_ex3(1, n=2, t=0.3, grid=grid), W.paper_ex3(-1, n=2, t=0.5, grid=grid),
        W.paper_ex3(-1, n=10, t=0.4, grid=grid), W.paper_ex5(n=2, t=0.3, grid=grid),
        W.paper_ex5(n=7, t=0.3, grid=grid),
    ] + [
        # the staggered discrete forms of section 3 on the same examples
        w.with_(name=w.name + "_staggered", ode=W.STAGGERED) for w in (
            W.paper_ex2(-1, n=2, t=0.5, grid=grid), W.paper_ex2_rosenbrock(grid=grid),
            W.paper_ex3(1, n=2, t=0.3, grid=grid), W.paper_ex5(n=2, t=0.3, grid=grid))
    ]


def bench_paper(args):
    """One line: the certified solves per second of each of the paper's
    examples on the GPU (the headline value is Example 2 with H-, d = 2),
    beside the paper's own per-point runtime as context."""
    grid = args.points or 64
    rows = []
    for wl in paper_examples(grid):
        wall, kern, host = run_gpu(wl, args.steps, args.warmup, wl.name, {})
        n_cert = int((host["cert"] == 1).sum())
        evals = float(host["slot_fwd"].sum())
        # algorithmic work: every objective evaluation is one solve of N
        # steps; a step costs one H / H_x / H_p evaluation and the integrand
        # (about 12 n flops for the quadratic family, 20 n + an exp pair for
        # the degree-1 one) and the Euler update (4 n); the fixed-point
        # sweeps of the staggered forms' implicit half-steps are not counted
        per_step = (16 if wl.h_kind == 0 else 24) * wl.n + 12
        flops = evals * wl.nsteps * per_step
        k_s = float(np.mean(kern)) / 1e3
        paper = PAPER_RUNTIME.get(wl.name)
        rows.append({
            "example": wl.name, "points": wl.B, "guesses": wl.G, "n": wl.n,
            "nsteps": wl.nsteps, "certified_points": n_cert, "value": n_cert / wall,
            "all_points_per_s": wl.B / wall, "ms_per_step": wall * 1e3,
            "evaluations": evals, "achieved_tflops": flops / k_s / 1e12,
            "paper_points_per_s_one_core": (1.0 / paper) if paper else None,
        })
    head = rows[0]
    peak = PEAK[("alu", "f64")]
    return {
        "metric": METRIC, "value": head["value"], "unit": "certified solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak",
        # the paper's own number for this example is from other hardware
        "vs_baseline": head["value"] * PAPER_RUNTIME["paper_ex2_minus_d2"],
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"paper: section 5 examples with the paper's scheme (forward "
                               f"Euler, rectangle rule, forward differences, Algorithm 1, "
                               f"M = 500, eps = 0.5e-7; four examples also with the staggered "
                               f"forms of section 3), {grid}x{grid} cross-section grid on "
                               f"[-3,3]^2, U[-2,2] guesses; value: Example 2 H-, d = 2",
                   "examples": rows},
        "roofline": {"bound": "alu", "achieved": head["achieved_tflops"], "peak": peak,
                     "unit": "TFLOP/s", "frac": head["achieved_tflops"] / peak,
                     "traffic": None, "kernel": "k_solve_paper"},
    }


def bench_lax_friedrichs(args):
    """The paper's Lax-Friedrichs comparison grid (dx = 0.005, dt = 0.001 on
    [-3,3]^2, t = 0.5) for the Example 2 oscillator H-, timed on the GPU:
    cell updates per second.  The roofline is the effective bandwidth of a
    one-step-per-pass scheme (each update reads one value and writes one,
    16 bytes, the neighbours coming from cache); the kernel itself keeps 4
    steps in LDS and moves less."""
    import torch
    from paper_1704_02524_amd import hj
    from paper_1704_02524_amd import workloads as W
    wl = W.paper_ex2(-1, grid=2)
    dx, dt, nt = 0.005, 0.001, 500
    nx = int(round(6.0 / dx)) + 1
    ts = []
    for i in range(args.warmup + args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        phi = hj.lax_friedrichs(wl, -3.0, -3.0, dx, dx, nx, nx, dt, nt, 3.0, 1.0)
        b.record()
        torch.cuda.synchronize()
        if i >= args.warmup:
            ts.append(a.elapsed_time(b) / 1e3)
    s = float(np.mean(ts))
    cells = nx * nx * nt
    gbs = cells * 16 / s / 1e9
    log(f"lax_friedrichs: {nx}x{nx} cells, {nt} steps, {s * 1e3:.2f} ms")
    del phi
    return {
        "metric": "Lax-Friedrichs grid cell updates/s", "value": cells / s,
        "unit": "cell updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"lax_friedrichs: Example 2 H- on [-3,3]^2, dx = {dx}, "
                               f"dt = {dt}, {nt} steps ({nx}x{nx} cells), 4 steps per launch "
                               f"on 64x32-cell LDS tiles"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                     "frac": gbs / 8000.0, "traffic": None, "kernel": "k_lf_steps"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=WORKLOADS, default="hopf_n10")
    ap.add_argument("--points", type=int, default=None,
                    help="query points (per instance for the batched workload)")
    ap.add_argument("--cd-points", type=int, default=None,
                    help="points of the central-FD comparison run (the n=10 workload runs it "
                         "on all points by default; other workloads only with this option)")
    ap.add_argument("--no-cd", action="store_true", help="skip the central-FD comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference baseline")
    ap.add_argument("--no-n32", action="store_true",
                    help="skip the n=32 drift record of the default (n=10) run")
    ap.add_argument("--n32-cd-points", type=int, default=8192,
                    help="points of the n=32 central-FD comparison")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of CPU reference work per process")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default launch shape")
    ap.add_argument("--launch", type=json.loads, default=None,
                    help='launch configuration of the descent as JSON, e.g. '
                         '\'{"lanes_per_task": 1, "ckpt_K": 16}\', instead of tuning')
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="bytes of a device copy run first (counter calibration)")
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

    if args.copy_probe:
        copy_probe(args.copy_probe)
    if args.workload == "paper":
        print(json.dumps(bench_paper(args)), flush=True)
        return
    if args.workload == "lax_friedrichs":
        print(json.dumps(bench_lax_friedrichs(args)), flush=True)
        return
    wls = build_workloads(args.workload, args.points)
    wl = wls[0]
    batched = len(wls) > 1
    dtype = "f64" if wl.dtype == W.F64 else "f32"
    if batched:
        log(f"workload {args.workload}: {len(wls)} instances, "
            f"{sum(w.B for w in wls)} points, {sum(w.B * w.G for w in wls)} tasks")
        tuning = None
        table = None
        if not args.no_tune:
            # the tuner's table against the library's default launch choices,
            # both timed on the full plan; the faster one is measured
            table = tune.tune_batched(wls, verbose=True)
            ms_def = tune.time_plan(wls, None, reps=2)
            ms_tuned = tune.time_plan(wls, table, reps=2) if table else ms_def
            log(f"batched tuning: default {ms_def:.1f} ms, tuned {ms_tuned:.1f} ms, "
                f"table {table}")
            tuning = {"table": table, "default_graph_ms": ms_def, "tuned_graph_ms": ms_tuned,
                      "gain": ms_def / ms_tuned, "used": "tuned" if ms_tuned < ms_def else
                      "default"}
            if ms_tuned >= ms_def:
                table = None
        wall, kern, hosts, info = run_batched(wls, args.steps, args.warmup, table)
        cfg = {"plan": info, "group_cfg": table}
        n_cert = int(sum((h["cert"] == 1).sum() for h in hosts))
        k_s = float(np.mean(kern)) / 1e3
        flops = sum(method_flops(w, h["slot_fwd"], h["slot_bwd"])
                    for w, h in zip(wls, hosts))
        flops_own = sum(own_flops(w, h["slot_fwd"], h["slot_bwd"])
                       for w, h in zip(wls, hosts))
        peak = PEAK[("alu", dtype)]
        rec = {
            "value": n_cert / wall, "unit": "certified solves/s", "ms_per_step": wall * 1e3,
            "dtype": dtype,
            "config": {
                "workload": f"{args.workload}: {len(wls)} Hopf instances, n in "
                            f"{sorted({w.n for w in wls})}, t~U[0.2,2], N in "
                            f"{sorted({w.nsteps for w in wls})}, {sum(w.B for w in wls)} "
                            f"points in total, {wl.G} guesses, adjoint gradient descent, one "
                            f"captured graph, {dtype.upper()}",
                "instances": len(wls), "points": int(sum(w.B for w in wls)), "guesses": wl.G,
                "certified_points": n_cert},
            "roofline": roofline_record("alu", peak, k_s, flops, flops_own,
                                        measured_traffic(args.workload, cfg),
                                        "k_solve_gd (batched launches of one graph)", cfg),
            "tuning": tuning,
        }
    else:
        if args.launch is not None:
            cfg = dict(args.launch)
        else:
            cfg = {} if args.no_tune else tune.tune(wl, verbose=True)
        rec, wall, host = measure_single(wl, args.workload, args.steps, args.warmup, cfg)

    result = {
        "metric": METRIC,
        "value": rec["value"],
        "unit": rec["unit"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": rec["dtype"],
        "data": "synthetic",
        "config": rec["config"],
        "roofline": rec["roofline"],
    }
    if rec.get("tuning") is not None:
        result["tuning"] = rec["tuning"]
    # the central-FD comparison: the whole n=10 workload by default; for the
    # other workloads only on request (--cd-points), since coordinate descent
    # costs 3n solves per sweep
    want_cd = args.workload == "hopf_n10" or args.cd_points is not None
    if not batched and wl.mode == W.GD_ADJ and want_cd and not args.no_cd:
        result.update(cd_comparison(wl, host, wall, args.cd_points, not args.no_tune))
    if not args.no_cpu:
        log("CPU reference baseline ...")
        if batched:
            result["cpu_baseline"] = cpu_baseline_slots(wls, args.cpu_budget)
        elif args.workload in ("hopf_n10", "lax_n32_drift"):
            result["cpu_baseline"] = cpu_baseline_points(args.workload, args.cpu_budget,
                                                         host_cores())
        else:
            result["cpu_baseline"] = cpu_baseline_slots(wls, args.cpu_budget)
        log(f"CPU: {result['cpu_baseline']['value']:.3f} certified solves/s")
    # the metric's second dimension: the n=32 linear-drift workload (65536
    # points, 8 guesses, 256 steps; checkpoint interval 3, the most the FP64
    # drift kernel's LDS segment holds) in the same run, with its own
    # matrix-core roofline, central-FD comparison on a prefix of the points
    # and CPU baseline
    if args.workload == "hopf_n10" and not args.no_n32:
        w32 = W.c3_drift_n32()
        cfg32 = {"ckpt_K": 3}
        rec32, wall32, host32 = measure_single(w32, "lax_n32_drift", 2, 1, cfg32)
        if not args.no_cd and args.n32_cd_points > 0:
            rec32.update(cd_comparison(w32, host32, wall32, args.n32_cd_points, False))
        if not args.no_cpu:
            rec32["cpu_baseline"] = cpu_baseline_points("lax_n32_drift", args.cpu_budget,
                                                        host_cores())
            log(f"CPU n=32: {rec32['cpu_baseline']['value']:.3f} certified solves/s")
        result["n32"] = rec32
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
