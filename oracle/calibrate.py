"""Certificate-tolerance calibration on the FP64 reference (CPU only).

For each benchmark configuration, solve the first points with the reference
at the configured tolerance tau and collect the certificate residual rho of
every slot's reported attempt: the accepted (certified) slots give the p99
of rho at accepted optima, the rejected finite slots the smallest rho of a
rejected slot.  A tolerance is well placed when it sits at least ten times
above the first and at most a tenth of the second (an empty set of rejected
slots leaves the upper condition vacuous).

TEST INFRASTRUCTURE ONLY (calls nothing but the reference).
usage: python -m oracle.calibrate [--points N] [--procs P]"""
import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, build  # noqa: E402
from paper_1704_02524_amd import workloads as W  # noqa: E402


def configs(points):
    """(label, list of workloads restricted to the sampled points)."""
    c2 = W.c2_batched()
    c2f = W.c2_batched(dtype=W.F32)
    return [
        ("C0 n=2 Lax, central-FD CD", [W.c0_lax_n2().subset(0, points)]),
        ("C1 n=10 Hopf, adjoint GD", [W.c1_hopf_n10(B=4096).subset(0, points)]),
        ("C1 n=10 Hopf, central-FD CD", [W.c1_hopf_n10(B=4096, mode=W.CD_FD).subset(0, points // 4)]),
        ("C2 batched, FP64 options", [w.subset(0, 1) for w in c2]),
        ("C2 batched, FP32 options", [w.subset(0, 1) for w in c2f]),
        ("C3 n=32 drift", [W.c3_drift_n32(B=4096).subset(0, max(4, points // 4))]),
        ("C4 n=100, FP32 options", [W.c4_lax_n100(B=4096).subset(0, points)]),
    ]


def _solve_point(args):
    wl, b = args
    sub = wl.subset(b, b + 1)
    r = Oracle.from_workload(sub).solve(sub.x, sub.guesses, Oracle.opts_from_workload(sub))
    return r["slot_rho"][0].tolist(), r["slot_cert"][0].tolist()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", type=int, default=64)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    build()
    rows = []
    with ProcessPoolExecutor(args.procs) as ex:
        for label, wls in configs(args.points):
            jobs = [(w, b) for w in wls for b in range(w.B)]
            rho, cert = [], []
            for r, c in ex.map(_solve_point, jobs):
                rho += r
                cert += c
            rho, cert = np.array(rho), np.array(cert)
            tau = wls[0].cert_tol
            acc = rho[cert == 1]
            rej = rho[(cert == 0) & np.isfinite(rho)]
            p99 = float(np.percentile(acc, 99)) if acc.size else float("nan")
            mrej = float(rej.min()) if rej.size else float("inf")
            rows.append(dict(config=label, points=len(jobs), slots=int(rho.size), tau=tau,
                             accepted=int(acc.size), p99_accepted=p99,
                             rejected=int(rej.size), min_rejected=mrej,
                             lower_ok=bool(tau >= 10 * p99),
                             upper_ok=bool(tau <= 0.1 * mrej)))
            print(json.dumps(rows[-1]), flush=True)


if __name__ == "__main__":
    main()
