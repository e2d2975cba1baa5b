"""Linear-drift Hamiltonians H = <A x, p> + 1/2 m(|x|^2) sum d_i p_i^2 on the
matrix-core kernels, checked through the C interface against the FP64 CPU
reference: objective, y_N, residual and exact gradient at fixed v (1e-12 /
1e-10 relative in FP64, 1e-4 / 1e-3 in FP32), full solves (1e-9 max(1,|u|)
in FP64, 1e-4 in FP32, equal certificate flags), and the adjoint gradient
against central differences of the GPU objective."""
import math

import numpy as np
import pytest
import torch

from oracle.oracle import Oracle, build as build_oracle
from paper_1704_02524_amd import workloads as W

pytestmark = pytest.mark.gpu

build_oracle()


@pytest.fixture(scope="module")
def hj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_02524_amd import hj as _hj
    return _hj


def _dev(a, wl):
    dt = torch.float64 if wl.dtype == W.F64 else torch.float32
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda().contiguous()


def _drift(n, formula=W.LAX, m_kind=W.M_RAT, e=1, quad=W.RK4AUG, nsteps=24, B=5, G=3, seed=0,
           w=0.0, signs=False, dtype=W.F64, norm=0.9):
    """A random drift with spectral norm `norm` on top of the test family of
    the other parity tests."""
    rng = np.random.default_rng(1000 + seed)
    A = rng.standard_normal((n, n)) / math.sqrt(n)
    A *= norm / max(np.linalg.norm(A, 2), 1e-300)
    d = np.ones(n)
    if signs:
        d[0] = -1.0
    a = rng.uniform(1.3, 2.0, n)
    wl = W.Workload(name="drift", n=n, t=0.6, nsteps=nsteps, m_kind=m_kind, e=e, kappa=0.4,
                    s=float(n), w=w, d=d, A=A, a=a, j0=-0.5, formula=formula, quad=quad,
                    x=rng.uniform(-1.5, 1.5, (B, n)), guesses=rng.standard_normal((B, G, 3, n)),
                    dtype=dtype)
    return W._as_dtype(wl) if dtype == W.F32 else wl


EVAL_CASES = [
    # n, formula, m_kind, e, quad, signs, w, B, G   (B*G tasks: full and partial waves)
    (1, W.LAX, W.M_RAT, 1, W.RK4AUG, False, 0.0, 5, 3),
    (5, W.LAX, W.M_RAT, 2, W.TRAPZ, False, 0.0, 7, 5),
    (16, W.HOPF, W.M_TANH, 1, W.RK4AUG, True, 0.0, 4, 4),
    (20, W.LAX, W.M_CONST, 1, W.RK4AUG, False, 0.7, 3, 3),
    (32, W.LAX, W.M_RAT, 1, W.RK4AUG, False, 0.0, 5, 7),
    (33, W.HOPF, W.M_RAT, 1, W.TRAPZ, True, -0.3, 2, 3),
    (64, W.LAX, W.M_TANH, 2, W.RK4AUG, False, 0.0, 3, 2),
]


@pytest.mark.parametrize("case", EVAL_CASES, ids=lambda c: f"n{c[0]}_f{c[1]}_m{c[2]}")
def test_drift_eval_matches_reference_fp64(hj, case):
    n, formula, m_kind, e, quad, signs, w, B, G = case
    wl = _drift(n, formula, m_kind, e, quad, signs=signs, w=w, B=B, G=G)
    v = wl.guesses[:, :, 0, :].copy()
    out = hj.evaluate(wl, _dev(wl.x, wl), _dev(v, wl), grad=True, yN=True, ckpt_K=5)
    torch.cuda.synchronize()
    o = Oracle.from_workload(wl)
    for b in range(B):
        for g in range(G):
            phi, yN = o.eval(wl.x[b], v[b, g])
            _, gv, gx = o.grad_tangent(wl.x[b], v[b, g])
            assert abs(out["phi"][b, g].item() - phi) <= 1e-12 * max(1.0, abs(phi)), (b, g)
            np.testing.assert_allclose(out["yN"][b, g].cpu().numpy(), yN, rtol=1e-12,
                                       atol=1e-12 * np.abs(yN).max())
            assert out["rho"][b, g].item() == pytest.approx(o.certificate(yN), rel=1e-9,
                                                            abs=1e-12)
            np.testing.assert_allclose(out["grad_v"][b, g].cpu().numpy(), gv, rtol=0,
                                       atol=1e-10 * max(1.0, np.abs(gv).max()))
            np.testing.assert_allclose(out["grad_x"][b, g].cpu().numpy(), gx, rtol=0,
                                       atol=1e-10 * max(1.0, np.abs(gx).max()))


@pytest.mark.parametrize("n", [4, 32, 50])
def test_drift_eval_matches_reference_fp32(hj, n):
    wl = _drift(n, dtype=W.F32, B=4, G=5)
    v = wl.guesses[:, :, 0, :].copy()
    out = hj.evaluate(wl, _dev(wl.x, wl), _dev(v, wl), grad=True, ckpt_K=8)
    torch.cuda.synchronize()
    o = Oracle.from_workload(wl)
    for b in range(4):
        for g in range(5):
            phi, _ = o.eval(wl.x[b], v[b, g])
            _, gv, _ = o.grad_tangent(wl.x[b], v[b, g])
            assert abs(out["phi"][b, g].item() - phi) <= 1e-4 * max(1.0, abs(phi))
            np.testing.assert_allclose(out["grad_v"][b, g].cpu().numpy(), gv, rtol=0,
                                       atol=1e-3 * max(1.0, np.abs(gv).max()))


def test_drift_checkpoint_interval_does_not_change_the_gradient(hj):
    wl = _drift(32, nsteps=37)
    x, v = _dev(wl.x, wl), _dev(wl.guesses[:, :, 0, :].copy(), wl)
    ref = hj.evaluate(wl, x, v, grad=True, ckpt_K=1)
    for K in [3, 16, 37]:
        out = hj.evaluate(wl, x, v, grad=True, ckpt_K=K)
        assert torch.equal(out["grad_v"], ref["grad_v"]), K
        assert torch.equal(out["phi"], ref["phi"]), K


def test_drift_adjoint_gradient_vs_central_differences(hj):
    """The exact discrete gradient against central differences of the GPU
    objective with step 1e-6 (the n = 32 drift workload's horizon and mesh)."""
    wl = W.c3_drift_n32(B=2)
    wl = wl.with_(guesses=wl.guesses[:, :2].copy())
    v = wl.guesses[:, :, 0, :].copy()
    x = _dev(wl.x, wl)
    out = hj.evaluate(wl, x, _dev(v, wl), grad=True)
    gv = out["grad_v"].cpu().numpy()
    sig = 1e-6
    fd = np.zeros_like(gv)
    for j in range(wl.n):
        vp, vm = v.copy(), v.copy()
        vp[:, :, j] += sig
        vm[:, :, j] -= sig
        fp = hj.evaluate(wl, x, _dev(vp, wl))["phi"].cpu().numpy()
        fm = hj.evaluate(wl, x, _dev(vm, wl))["phi"].cpu().numpy()
        fd[:, :, j] = (fp - fm) / (2 * sig)
    rel = np.abs(fd - gv).max() / np.abs(gv).max()
    print(f"drift n=32: adjoint vs central FD (step 1e-6) max relative error {rel:.2e}")
    assert rel < 1e-6


def _oracle_solve(wl):
    return Oracle.from_workload(wl).solve(wl.x, wl.guesses, Oracle.opts_from_workload(wl))


def _compare_solve(res, ref, tol_u, tol_arg):
    u = res["u"].cpu().numpy()
    arg = res["argopt"].cpu().numpy()
    np.testing.assert_array_equal(res["cert"].cpu().numpy(), ref["cert"])
    fin = ref["cert"] >= 0
    err = np.abs(u[fin] - ref["u"][fin]) / np.maximum(1.0, np.abs(ref["u"][fin]))
    assert err.max(initial=0.0) <= tol_u, err.max()
    c1 = ref["cert"] == 1
    if c1.any():
        aerr = np.abs(arg[c1] - ref["argopt"][c1]).max() / max(1.0, np.abs(ref["argopt"][c1]).max())
        assert aerr <= tol_arg, aerr


def _c3_small(B=3, G=4, nsteps=32, dtype=W.F64, mode=W.GD_ADJ):
    wl = W.c3_drift_n32(B=B, dtype=dtype)
    return wl.with_(guesses=wl.guesses[:, :G].copy(), nsteps=nsteps, mode=mode)


def test_drift_solve_matches_reference(hj):
    wl = _c3_small()
    res = hj.solve(wl, *hj.device_inputs(wl))
    ref = _oracle_solve(wl)
    torch.cuda.synchronize()
    _compare_solve(res, ref, 1e-9, 1e-6)
    assert (ref["cert"] == 1).all()


def test_drift_solve_cd_matches_reference(hj):
    wl = _drift(6, B=3, G=3, nsteps=16).with_(mode=W.CD_FD, max_iter=80, eps_step=1e-10,
                                             cert_tol=1e-6, alpha0=1 / 3)
    res = hj.solve(wl, *hj.device_inputs(wl))
    ref = _oracle_solve(wl)
    torch.cuda.synchronize()
    # The solve counts are not compared: the MFMA sums A gamma in another order
    # than the reference, and the central-difference quotient magnifies that
    # rounding by 1/sigma, so the sweep at which the step test trips may differ.
    _compare_solve(res, ref, 1e-9, 1e-6)


def test_drift_solve_fp32_with_fp64_certificate(hj):
    wl = _c3_small(B=2, G=3, dtype=W.F32)
    res = hj.solve(wl, *hj.device_inputs(wl))
    ref = _oracle_solve(wl)
    torch.cuda.synchronize()
    u = res["u"].cpu().numpy()
    print("FP32 drift slot residuals", res["slot_rho"].cpu().numpy().ravel(),
          "reference", ref["slot_rho"].ravel())
    np.testing.assert_array_equal(res["cert"].cpu().numpy(), ref["cert"])
    assert (np.abs(u - ref["u"]) / np.maximum(1, np.abs(ref["u"]))).max() <= 1e-4


@pytest.mark.parametrize("mode", [W.GD_ADJ, W.CD_FD])
def test_drift_persistent_schedule_equals_static(hj, mode):
    wl = _c3_small(B=40, G=3, nsteps=16, mode=mode)
    if mode == W.CD_FD:
        wl = wl.with_(max_iter=6)
    x, g = hj.device_inputs(wl)
    a = {k: v.cpu().numpy() for k, v in hj.solve(wl, x, g, schedule=hj.SCHED_STATIC).items()}
    b = {k: v.cpu().numpy() for k, v in hj.solve(wl, x, g, schedule=hj.SCHED_PERSISTENT).items()}
    for k in a:
        np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]), err_msg=k)


def test_drift_batched_plan_is_rejected(hj):
    wl = _c3_small(B=2, G=2)
    with pytest.raises(hj.HJError):
        hj.BatchPlan([wl])
