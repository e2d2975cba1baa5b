"""Rate of the FP64 reference on the host: solve whole points of a benchmark
workload (all guesses and restarts of each point) until a time budget is
spent, and print {"points", "certified", "seconds"} as JSON.

TEST INFRASTRUCTURE ONLY: run by the CPU-baseline leg of bench.py, one
process per core over disjoint point sets (points offset, offset + stride,
...).  usage: python -m oracle.cpu_rate WORKLOAD OFFSET STRIDE BUDGET_S"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_1704_02524_amd import workloads as W  # noqa: E402

MAKERS = {
    "hopf_n10": lambda: W.c1_hopf_n10(B=4096),
    "hopf_n10_cd": lambda: W.c1_hopf_n10(B=4096, mode=W.CD_FD),
    "lax_n32_drift": lambda: W.c3_drift_n32(B=65536),
}


def main():
    name, off, stride, budget = sys.argv[1], int(sys.argv[2]), int(sys.argv[3]), \
        float(sys.argv[4])
    wl = MAKERS[name]()
    o = Oracle.from_workload(wl)
    O = Oracle.opts_from_workload(wl)
    t0 = time.perf_counter()
    pts = cert = 0
    b = off
    while b < wl.B and time.perf_counter() - t0 < budget:
        r = o.solve(wl.x[b:b + 1], wl.guesses[b:b + 1], O, diag=False)
        pts += 1
        cert += int(r["cert"][0] == 1)
        b += stride
    print(json.dumps({"points": pts, "certified": cert,
                      "seconds": time.perf_counter() - t0}), flush=True)


if __name__ == "__main__":
    main()
