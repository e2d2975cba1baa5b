"""Point-by-point comparison of GPU solves with the FP64 reference.

Certificate flags must agree per point.  The only allowed exception is a point
inside the ambiguity band of the reference: a slot whose certificate residual
lies within a factor two of the tolerance (tau/2 <= rho <= 2 tau), where the
rounding of either side can decide the flag; such points are counted in
`band` so a test can report them (and bound how many there are)."""
import numpy as np

from oracle.oracle import Oracle
from paper_1704_02524_amd import workloads as W


def reference_point(wl, b):
    sub = wl.subset(b, b + 1)
    return _solve_one(sub)


def _solve_one(sub):
    return Oracle.from_workload(sub).solve(sub.x, sub.guesses, Oracle.opts_from_workload(sub))


def reference_points(wl, points, workers=8):
    """The reference at several points, in worker processes started fresh
    (spawn: they load only the CPU reference, never the GPU runtime)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    subs = [wl.subset(int(b), int(b) + 1) for b in points]
    with cf.ProcessPoolExecutor(max_workers=min(workers, len(subs)),
                                mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_solve_one, subs))


def in_band(ref, tol):
    rho = ref["slot_rho"][0]
    return bool(np.any((rho >= 0.5 * tol) & (rho <= 2.0 * tol)))


def check_point(wl, b, got_u, got_cert, got_arg, tol_u, tol_arg, band=None, ref=None):
    """u within tol_u * max(1, |u|), equal certificate flags (or the point is
    in the reference's ambiguity band), argopt within tol_arg (relative to
    max(1, |argopt|_inf)) where both certify."""
    ref = reference_point(wl, b) if ref is None else ref
    rc = int(ref["cert"][0])
    if got_cert != rc:
        assert in_band(ref, wl.cert_tol), (wl.name, b, got_cert, rc, ref["slot_rho"][0])
        if band is not None:
            band.append((wl.name, b))
        return
    if rc >= 0:
        err = abs(got_u - ref["u"][0]) / max(1.0, abs(ref["u"][0]))
        assert err <= tol_u, (wl.name, b, err)
        if rc == 1 and tol_arg is not None:
            aerr = np.abs(got_arg - ref["argopt"][0]).max() / \
                max(1.0, np.abs(ref["argopt"][0]).max())
            assert aerr <= tol_arg, (wl.name, b, aerr)


def tolerances(wl):
    """(u, argopt) tolerances: 1e-9 and 1e-6 in FP64, 1e-4 and 5e-3 in FP32."""
    return (1e-9, 1e-6) if wl.dtype == W.F64 else (1e-4, 5e-3)
