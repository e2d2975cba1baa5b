"""Autotuner for the launch configuration of hj_solve.

The tunable knobs do not change results: the lane shape (lanes per task,
which fixes how many vector components each lane holds) only changes the
summation order at rounding level, and the adjoint checkpoint interval K
changes nothing (the recomputed segments are bit-identical to the forward
solve).  For a workload the tuner times every candidate on the full point
set with the iteration cap lowered (so occupancy and per-iteration cost are
those of the real run), keeps the fastest, and caches the choice in a JSON
table keyed by the workload's shape.
"""
from __future__ import annotations

import json
import sys
import os
from typing import Dict, Optional

import torch

from . import hj
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")

# lanes-per-task values compiled for each dimension bound (mirrors the shape
# table of the library: a request the library cannot serve raises)
LPT_CHOICES = (1, 2, 4, 8, 16)


def _key(wl) -> str:
    return (f"n{wl.n}_N{wl.nsteps}_G{wl.G}_B{wl.B}_dt{wl.dtype}_mode{wl.mode}"
            f"_m{wl.m_kind}_q{wl.quad}_dr{int(wl.A is not None)}")


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(table: Dict[str, dict]) -> None:
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def candidates(wl):
    ks = [None]
    if wl.mode == W.GD_ADJ:
        ks = sorted({1, 4, 16, min(wl.ckpt_K, wl.nsteps)})
    out = []
    # a drift matrix runs on the matrix-core layout: 4 lanes per task only
    lpts = (4,) if wl.A is not None else LPT_CHOICES
    for lpt in lpts:
        if wl.A is None and -(-wl.n // lpt) > 16:  # more than 16 components per lane
            continue
        if wl.A is None and lpt > 1 and wl.n <= lpt:  # lanes without a component
            continue
        for K in ks:
            out.append(dict(lanes_per_task=lpt, **({} if K is None else {"ckpt_K": K})))
    return out


def time_config(wl, x, g, cfg, reps=2, warm=True) -> Optional[float]:
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    ev[0].record()
    ev[1].record()
    best = None
    try:
        out = hj.solve(wl, x, g, diag=False, **cfg) if warm else None
        for _ in range(reps):
            out = hj.solve(wl, x, g, diag=False, out=out, events=ev, **cfg)
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1])
            best = ms if best is None else min(best, ms)
    except hj.HJError:
        return None
    return best


def tune(wl, tune_iters: int = 20, use_cache: bool = True, verbose: bool = False) -> dict:
    """The fastest {lanes_per_task, ckpt_K} for this workload."""
    key = _key(wl)
    table = _load()
    if use_cache and key in table:
        return dict(table[key]["config"])
    # the probe runs tune_iters iterations per slot and accepts every finite
    # result, so no slot restarts: each candidate does the same work
    probe = wl.with_(max_iter=min(wl.max_iter, tune_iters), cert_tol=float("inf"))
    x, g = hj.device_inputs(probe)
    cands = candidates(wl)
    # one untimed run grows the workspace; long runs are then timed once
    first = time_config(probe, x, g, cands[0], reps=1)
    long_run = first is not None and first > 1000.0
    results = []
    for cfg in cands:
        ms = time_config(probe, x, g, cfg, reps=1 if long_run else 2, warm=not long_run)
        if verbose:
            print(f"[tune] {key} {cfg}: {ms} ms", file=sys.stderr, flush=True)
        if ms is not None:
            results.append((ms, cfg))
    if not results:
        return {}
    results.sort(key=lambda r: r[0])
    # near-ties (within 1.5 %, about the run-to-run spread of a probe) go to
    # the largest checkpoint interval (least scratch memory and traffic),
    # then to the fewest lanes per task, so the choice does not flip with
    # timing noise
    near = [r for r in results if r[0] <= 1.015 * results[0][0]]
    near.sort(key=lambda r: (-r[1].get("ckpt_K", 0), r[1]["lanes_per_task"]))
    best = near[0][1]
    table[key] = {"config": best, "ms": near[0][0],
                  "all": [{"ms": ms, **c} for ms, c in results]}
    try:
        _save(table)
    except OSError:
        pass
    return dict(best)
