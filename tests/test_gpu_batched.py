"""Persistent (work-queue) scheduling and batched instances in one
graph-captured launch sequence, checked against the single-problem path and
the FP64 reference."""
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


@pytest.mark.parametrize("lpt", [1, 2])
@pytest.mark.parametrize("mode", [W.GD_ADJ, W.CD_FD])
def test_persistent_schedule_equals_static(hj, lpt, mode):
    """Lane groups that pop tasks from the queue compute exactly what one
    group per task computes (results are indexed by task, not by lane)."""
    wl = W.c1_hopf_n10(B=96, mode=mode)
    if mode == W.CD_FD:
        wl = wl.with_(guesses=wl.guesses[:, :4].copy(), max_iter=30)
    x, g = hj.device_inputs(wl)
    a = _host(hj.solve(wl, x, g, lanes_per_task=lpt, schedule=hj.SCHED_STATIC))
    # a persistent launch with far fewer groups than tasks
    b = _host(hj.solve(wl, x, g, lanes_per_task=lpt, schedule=hj.SCHED_PERSISTENT))
    for k in a:
        np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]), err_msg=k)


def _batch(n_inst=8, max_points=20, dtype=W.F64, G=4):
    wls = W.c2_batched(dtype=dtype, n_inst=n_inst, max_points=max_points)
    return [w.with_(guesses=w.guesses[:, :G].copy(), max_iter=120) for w in wls]


@pytest.mark.parametrize("dtype", [W.F64, W.F32])
def test_batched_equals_single_solves_and_graph_replays(hj, dtype):
    """The captured plan (its shape groups as concurrent graph branches)
    gives every instance what a single solve gives it, on every replay, with
    eager work between the replays."""
    wls = _batch(dtype=dtype)
    plan = hj.BatchPlan(wls)
    info = plan.info()
    assert info["tasks"] == sum(w.B * w.G for w in wls)
    assert info["launches"] == len({w.n for w in wls})
    singles = [_host(hj.solve(w, *hj.device_inputs(w))) for w in wls]
    for rep in range(3):
        outs = plan.run()
        torch.cuda.synchronize()
        for w, out, ref in zip(wls, outs, singles):
            got = _host(out)
            np.testing.assert_array_equal(got["cert"], ref["cert"])
            np.testing.assert_allclose(got["u"], ref["u"], rtol=1e-13, atol=1e-13)
            np.testing.assert_array_equal(got["slot_fwd"], ref["slot_fwd"])
            np.testing.assert_allclose(np.nan_to_num(got["argopt"]),
                                       np.nan_to_num(ref["argopt"]), rtol=1e-12, atol=1e-12)
        # eager work between replays: clobber the outputs and run other kernels
        for out in outs:
            for v in out.values():
                v.zero_()
        _ = torch.randn(1 << 20, device="cuda").sum().item()
        torch.cuda.synchronize()
    plan.free()


# launch choices by dimension class, none of them the library's default
_TABLE = [dict(n_max=4, lanes_per_task=2, ckpt_K=8, cont_lanes_per_task=1),
          dict(n_max=8, lanes_per_task=1, ckpt_K=32, cont_lanes_per_task=4),
          dict(n_max=16, lanes_per_task=2, cont_lanes_per_task=4),
          dict(n_max=32, lanes_per_task=8, ckpt_K=4, cont_lanes_per_task=4)]


@pytest.mark.parametrize("dtype", [W.F64, W.F32])
def test_group_cfg_plan_equals_single_solves_with_that_launch(hj, dtype):
    """A plan with a per-class launch table gives every instance what a
    single solve with that class's lanes per task and checkpoint interval
    gives it, on every replay."""
    wls = _batch(dtype=dtype)
    plan = hj.BatchPlan(wls, group_cfg=_TABLE)
    assert plan.info()["launches"] == len({w.n for w in wls})
    singles = []
    for w in wls:
        c = next(c for c in _TABLE if w.n <= c["n_max"])
        over = {k: v for k, v in c.items() if k != "n_max"}
        singles.append(_host(hj.solve(w, *hj.device_inputs(w), **over)))
    for rep in range(2):
        outs = plan.run()
        torch.cuda.synchronize()
        for w, out, ref in zip(wls, outs, singles):
            got = _host(out)
            np.testing.assert_array_equal(got["cert"], ref["cert"], err_msg=w.name)
            np.testing.assert_allclose(got["u"], ref["u"], rtol=1e-13, atol=1e-13)
            np.testing.assert_array_equal(got["slot_fwd"], ref["slot_fwd"])
        for out in outs:
            for v in out.values():
                v.zero_()
        torch.cuda.synchronize()
    plan.free()


def test_group_cfg_checkpoint_interval_changes_nothing(hj):
    """The checkpoint interval only trades memory for recomputation: the
    recomputed segments are those of the forward solve, bit for bit."""
    wls = _batch(n_inst=6, max_points=12)
    a = hj.BatchPlan(wls)
    b = hj.BatchPlan(wls, group_cfg=[dict(n_max=64, ckpt_K=3)])
    ra = [_host(o) for o in a.run()]
    torch.cuda.synchronize()
    rb = [_host(o) for o in b.run()]
    torch.cuda.synchronize()
    for x, y in zip(ra, rb):
        for k in x:
            np.testing.assert_array_equal(np.nan_to_num(x[k]), np.nan_to_num(y[k]), err_msg=k)
    a.free()
    b.free()


def test_group_cfg_errors(hj):
    wls = _batch(n_inst=3, max_points=4)
    with pytest.raises(hj.HJError, match=">= 0"):
        hj.BatchPlan(wls, group_cfg=[dict(n_max=64, ckpt_K=-1)])
    with pytest.raises(hj.HJError, match="lanes per task"):
        hj.BatchPlan(wls, group_cfg=[dict(n_max=64, lanes_per_task=3)])
    with pytest.raises(hj.HJError, match="continuation"):
        hj.BatchPlan(wls, group_cfg=[dict(n_max=64, cont_lanes_per_task=16)])


def test_batched_matches_reference(hj):
    wls = _batch(n_inst=6, max_points=6)
    plan = hj.BatchPlan(wls)
    outs = plan.run()
    torch.cuda.synchronize()
    for w, out in zip(wls, outs):
        got = _host(out)
        o = Oracle.from_workload(w)
        ref = o.solve(w.x[:2], w.guesses[:2], Oracle.opts_from_workload(w))
        np.testing.assert_array_equal(got["cert"][:2], ref["cert"])
        fin = ref["cert"] >= 0
        err = np.abs(got["u"][:2][fin] - ref["u"][fin]) / np.maximum(1, np.abs(ref["u"][fin]))
        assert err.max(initial=0.0) <= 1e-9, (w.name, err)
    plan.free()


def test_batched_fp32(hj):
    wls = _batch(n_inst=4, max_points=8, dtype=W.F32)
    plan = hj.BatchPlan(wls)
    outs = plan.run()
    torch.cuda.synchronize()
    for w, out in zip(wls, outs):
        got = _host(out)
        ref = Oracle.from_workload(w).solve(w.x[:2], w.guesses[:2], Oracle.opts_from_workload(w))
        np.testing.assert_array_equal(got["cert"][:2], ref["cert"])
        fin = ref["cert"] >= 0
        err = np.abs(got["u"][:2][fin] - ref["u"][fin]) / np.maximum(1, np.abs(ref["u"][fin]))
        assert err.max(initial=0.0) <= 1e-4, (w.name, err)
    plan.free()


@pytest.mark.parametrize("dtype,mode", [(W.F64, W.GD_ADJ), (W.F32, W.GD_ADJ),
                                        (W.F64, W.CD_FD)])
@pytest.mark.parametrize("lpt", [1, 2])
def test_persistent_many_tasks_per_group_equals_static(hj, dtype, mode, lpt):
    """A persistent launch capped at 64 lane groups (each group runs about 24
    tasks in turn, with restarts) gives every slot the result a one-task
    launch gives it, bit for bit: nothing of a finished task carries over."""
    wl = W.c1_hopf_n10(B=96)
    if dtype == W.F32:
        # FP32 restarts: without the FP64 continuation an attempt the
        # certificate rejects restarts in FP32
        wl = W._as_dtype(wl.with_(eps_step=1e-6, cert_tol=1e-4, fp64_continue=False))
    wl = wl.with_(max_iter=60, mode=mode)
    if mode == W.CD_FD:
        wl = wl.with_(guesses=wl.guesses[:, :4].copy(), max_iter=20)
    x, g = hj.device_inputs(wl)
    a = _host(hj.solve(wl, x, g, lanes_per_task=lpt, schedule=hj.SCHED_STATIC))
    b = _host(hj.solve(wl, x, g, lanes_per_task=lpt, schedule=hj.SCHED_PERSISTENT,
                       max_groups=64))
    assert (a["slot_attempts"] > 1).any()  # restarts happen
    for k in a:
        np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]), err_msg=k)


def test_batched_persistent_equals_single(hj):
    """Batched instances in a persistent launch of 32 lane groups per shape
    agree slot by slot with single-instance static solves."""
    wls = _batch(n_inst=4, max_points=24)
    plan = hj.BatchPlan(wls, max_groups=32)
    outs = plan.run()
    torch.cuda.synchronize()
    for w, out in zip(wls, outs):
        ref = _host(hj.solve(w, *hj.device_inputs(w), schedule=hj.SCHED_STATIC))
        got = _host(out)
        for k in ("slot_fwd", "slot_iters", "slot_attempts", "cert"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        np.testing.assert_allclose(got["u"], ref["u"], rtol=1e-13, atol=1e-13)
    plan.free()


@pytest.mark.parametrize("lpt", [1, 2])
def test_fp64_continuation_persistent_equals_static(hj, lpt):
    """FP32 descent whose rejected attempts continue in FP64: the hand-off
    list is filled in whatever order the lane groups finish, and a
    persistent launch of 64 groups (and a continuation launch of 64 groups)
    still gives every slot the static launch's result bit for bit."""
    wl = W._as_dtype(W.c1_hopf_n10(B=96).with_(eps_step=1e-6, cert_tol=1e-6, max_iter=60))
    x, g = hj.device_inputs(wl)
    a = _host(hj.solve(wl, x, g, lanes_per_task=lpt, schedule=hj.SCHED_STATIC))
    b = _host(hj.solve(wl, x, g, lanes_per_task=lpt, schedule=hj.SCHED_PERSISTENT,
                       max_groups=64))
    # some slots were handed off: without the continuation they end otherwise
    c = _host(hj.solve(wl, x, g, lanes_per_task=lpt, schedule=hj.SCHED_STATIC,
                       fp64_continue=0))
    assert (c["slot_iters"] != a["slot_iters"]).any()
    for k in a:
        np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]), err_msg=k)


def test_fp64_continuation_certifies_what_the_reference_certifies(hj):
    """Long-horizon FP32 instances of the batched workload (n = 4 and 8,
    t about 1.8), where FP32 descent alone stops above the tolerance on some
    slots: with the FP64 continuation every point's certificate flag is the
    FP64 reference's, and u agrees to 1e-4."""
    wls = W.c2_batched(dtype=W.F32)
    for i, npts in ((60, 32), (7, 32), (33, 12)):
        wl = wls[i].subset(0, npts)
        x, g = hj.device_inputs(wl)
        without = _host(hj.solve(wl, x, g, fp64_continue=0))
        got = _host(hj.solve(wl, x, g))
        ref = Oracle.from_workload(wl).solve(wl.x, wl.guesses, Oracle.opts_from_workload(wl))
        print(f"instance {i}: uncertified slots FP32 only {(without['slot_cert'] != 1).sum()}, "
              f"with continuation {(got['slot_cert'] != 1).sum()}, "
              f"reference {(ref['slot_cert'] != 1).sum()}")
        np.testing.assert_array_equal(got["cert"], ref["cert"], err_msg=wl.name)
        fin = ref["cert"] >= 0
        err = np.abs(got["u"][fin] - ref["u"][fin]) / np.maximum(1, np.abs(ref["u"][fin]))
        assert err.max(initial=0.0) <= 1e-4, (wl.name, err)


def test_fp64_continuation_on_a_wider_lane_shape(hj):
    """The continuation launch on a shape with more lanes per task than the
    descent's (the same padded dimension): the same certificates as the
    FP64 reference, and persistent == static bit for bit on that shape."""
    from paper_1704_02524_amd import tune
    wls = W.c2_batched(dtype=W.F32)
    for i, npts in ((60, 32), (7, 32), (33, 12)):
        wl = wls[i].subset(0, npts)
        lpt = tune._default_lpt(wl.n, True)
        wider = [c for c in tune.cont_lpts(wl.n, lpt) if c > lpt]
        if not wider:
            continue
        cl = wider[-1]
        x, g = hj.device_inputs(wl)
        got = _host(hj.solve(wl, x, g, cont_lanes_per_task=cl, schedule=hj.SCHED_STATIC))
        per = _host(hj.solve(wl, x, g, cont_lanes_per_task=cl, schedule=hj.SCHED_PERSISTENT,
                             max_groups=16))
        for k in got:
            np.testing.assert_array_equal(np.nan_to_num(got[k]), np.nan_to_num(per[k]),
                                          err_msg=k)
        ref = Oracle.from_workload(wl).solve(wl.x, wl.guesses, Oracle.opts_from_workload(wl))
        np.testing.assert_array_equal(got["cert"], ref["cert"], err_msg=wl.name)
        fin = ref["cert"] >= 0
        err = np.abs(got["u"][fin] - ref["u"][fin]) / np.maximum(1, np.abs(ref["u"][fin]))
        assert err.max(initial=0.0) <= 1e-4, (wl.name, cl, err)
