"""Tail hand-off of the FP64 adjoint descent: slots still descending after a
budget of objective evaluations leave their whole descent state in a record
and a second launch of a wider lane shape resumes them.  With the descent's
own lane shape the continuation must reproduce the single launch bit for
bit (the state transfer loses nothing); with a wider shape the results may
differ only by the rounding of its sums, and agree with the FP64
reference."""
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


def _host(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _restart_workload():
    """A slice of the n = 10 Hopf workload whose tight certificate tolerance
    makes some attempts fail and restart, so that resumed slots also run
    restarts after the hand-off."""
    wl = W.c1_hopf_n10(B=48)
    return wl.with_(cert_tol=1e-9, max_iter=60)


@pytest.mark.parametrize("budget", [1, 37, 90])
@pytest.mark.parametrize("schedule", ["static", "persistent"])
def test_tail_with_the_same_shape_is_bitwise(hj, budget, schedule):
    """Hand-off after 1 evaluation (every slot), mid-descent, and late; the
    continuation with the descent's own lanes per task (1) gives every
    per-slot record and the selection exactly as without the hand-off."""
    for wl in (W.c1_hopf_n10(B=64), _restart_workload()):
        x, g = hj.device_inputs(wl)
        sch = hj.SCHED_STATIC if schedule == "static" else hj.SCHED_PERSISTENT
        a = _host(hj.solve(wl, x, g, lanes_per_task=1, ckpt_K=4, schedule=sch))
        b = _host(hj.solve(wl, x, g, lanes_per_task=1, ckpt_K=4, schedule=sch,
                           tail_budget=budget, tail_lanes_per_task=1))
        for k in a:
            np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]),
                                          err_msg=f"{k} budget {budget}")
        if budget == 1:
            assert (a["slot_attempts"] >= 1).all()


@pytest.mark.parametrize("tail_lpt", [2, 4])
def test_tail_with_a_wider_shape_matches_the_reference(hj, tail_lpt):
    """Hand-off to two lanes per task (the descent's padded dimension) and to
    four (a padded dimension of its own, 12, with parameter rows of its own):
    equal certificates and u within 1e-9 of the single launch and of the
    reference (sampled points, every slot of them recomputed)."""
    wl = W.c1_hopf_n10(B=256)
    x, g = hj.device_inputs(wl)
    a = _host(hj.solve(wl, x, g, lanes_per_task=1, ckpt_K=4))
    b = _host(hj.solve(wl, x, g, lanes_per_task=1, ckpt_K=4, tail_budget=60,
                       tail_lanes_per_task=tail_lpt))
    np.testing.assert_array_equal(a["cert"], b["cert"])
    assert (np.abs(a["u"] - b["u"]) <= 1e-9 * np.maximum(1, np.abs(a["u"]))).all()
    handed = (a["slot_fwd"] > 60).sum()
    assert handed > 0
    o = Oracle.from_workload(wl)
    ref = o.solve(wl.x, wl.guesses, Oracle.opts_from_workload(wl), 0, 12)
    np.testing.assert_array_equal(b["cert"][:12], ref["cert"][:12])
    err = np.abs(b["u"][:12] - ref["u"][:12]) / np.maximum(1, np.abs(ref["u"][:12]))
    assert err.max() <= 1e-9, err.max()


def test_tail_with_restarts_after_the_hand_off(hj):
    wl = _restart_workload()
    x, g = hj.device_inputs(wl)
    a = _host(hj.solve(wl, x, g, lanes_per_task=1, ckpt_K=4))
    b = _host(hj.solve(wl, x, g, lanes_per_task=1, ckpt_K=4, tail_budget=30,
                       tail_lanes_per_task=2))
    assert (a["slot_attempts"] > 1).any()
    np.testing.assert_array_equal(a["cert"], b["cert"])
    np.testing.assert_array_equal(a["slot_attempts"], b["slot_attempts"])
    fin = np.isfinite(a["u"])
    assert (np.abs(a["u"][fin] - b["u"][fin]) <= 1e-9 * np.maximum(1, np.abs(a["u"][fin]))).all()


def test_tail_errors_are_reported(hj):
    wl = W.c1_hopf_n10(B=8)
    x, g = hj.device_inputs(wl)
    with pytest.raises(hj.HJError, match="tail-continuation kernel"):
        hj.solve(wl, x, g, lanes_per_task=1, tail_budget=10, tail_lanes_per_task=16)
    w32 = W._as_dtype(wl) if hasattr(W, "_as_dtype") else wl.with_(dtype=W.F32)
    with pytest.raises(hj.HJError, match="tail hand-offs"):
        hj.solve(w32, *hj.device_inputs(w32), tail_budget=10)
    with pytest.raises(hj.HJError, match="tail_budget"):
        hj.solve(wl, x, g, tail_budget=-1)
    wp = W.paper_ex2(-1, grid=2)
    with pytest.raises(hj.HJError, match="tail hand-offs"):
        hj.solve(wp, *hj.device_inputs(wp), tail_budget=10)
    wd = W.c3_drift_n32(B=4)
    with pytest.raises(hj.HJError, match="tail hand-offs"):
        hj.solve(wd, *hj.device_inputs(wd), tail_budget=10)


def test_tail_in_the_fixed_scratch_of_the_noalloc_entry(hj):
    """hj_solve_noalloc with a hand-off gives hj_solve's results: the records
    and the continuation's checkpoints fit the fixed scratch."""
    wl = W.c1_hopf_n10(B=128)
    x, g = hj.device_inputs(wl)
    cfg = dict(lanes_per_task=1, ckpt_K=4, tail_budget=40, tail_lanes_per_task=2)
    a = _host(hj.solve(wl, x, g, **cfg))
    b = _host(hj.solve(wl, x, g, noalloc=True, **cfg))
    for k in a:
        np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]), err_msg=k)


@pytest.mark.parametrize("n,lpt,tail_lpt", [(10, 2, 4), (7, 1, 2), (7, 1, 4), (3, 1, 2)])
def test_tail_on_other_shapes(hj, n, lpt, tail_lpt):
    """Other descent and continuation shapes, ragged dimensions (n = 7 and 3
    pad to 8 and 4 components): equal certificates and u within 1e-9 of the
    single launch."""
    base = W.c1_hopf_n10(B=96)
    rng = np.random.default_rng(n)
    wl = base.with_(n=n, d=base.d[:n].copy(), a=base.a[:n].copy(),
                    x=np.ascontiguousarray(base.x[:, :n]),
                    guesses=np.ascontiguousarray(base.guesses[..., :n]),
                    s=float(n))
    x, g = hj.device_inputs(wl)
    a = _host(hj.solve(wl, x, g, lanes_per_task=lpt))
    b = _host(hj.solve(wl, x, g, lanes_per_task=lpt, tail_budget=45,
                       tail_lanes_per_task=tail_lpt))
    assert (a["slot_fwd"] > 45).any()
    np.testing.assert_array_equal(a["cert"], b["cert"])
    fin = np.isfinite(a["u"])
    assert (np.abs(a["u"][fin] - b["u"][fin]) <= 1e-9 * np.maximum(1, np.abs(a["u"][fin]))).all()
