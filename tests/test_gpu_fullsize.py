"""Full-size launches of the n=10 Hopf (adjoint descent and central-difference
coordinate descent), n=32 drift, n=100 FP32 and batched workloads, in the
configurations bench.py times, with sampled points checked against the FP64
reference one by one (the reference solves a point in about a second; a
central-difference point in a few).  u to 1e-9 max(1, |u|) in FP64 and 1e-4
in FP32; certificate flags equal per point in both (FP32 runs continue in
FP64 the attempts the FP64 certificate rejects); argopt to 1e-6 (FP64) or
5e-3 (FP32) where certified."""
import numpy as np
import pytest
import torch

from oracle.oracle import build as build_oracle
from paper_1704_02524_amd import workloads as W

from parity_util import check_point, reference_points, tolerances

pytestmark = pytest.mark.gpu

build_oracle()


@pytest.fixture(scope="module")
def hj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_02524_amd import hj as _hj
    return _hj


def _check(wl, res, points, band=None, random=0, seed=0):
    """The given points and `random` more drawn uniformly, recomputed by the
    reference in parallel worker processes."""
    u, cert, arg = (res[k].cpu().numpy() for k in ("u", "cert", "argopt"))
    tu, ta = tolerances(wl)
    pts = list(dict.fromkeys(int(b) for b in points))
    if random:
        rng = np.random.default_rng(seed)
        pts += [int(b) for b in rng.choice(wl.B, random, replace=False) if int(b) not in pts]
    refs = reference_points(wl, pts) if len(pts) > 2 else [None] * len(pts)
    for b, ref in zip(pts, refs):
        check_point(wl, b, u[b], cert[b], arg[b], tu, ta, band, ref=ref)
    print(f"{wl.name}: {len(pts)} points checked against the reference")
    return u, cert, arg


def test_drift_n32_full_size_sampled(hj):
    """65536 points x 8 guesses, 256 steps, A on the matrix cores (the
    checkpoint interval does not change results: bit-identical gradients)."""
    wl = W.c3_drift_n32()
    res = hj.solve(wl, *hj.device_inputs(wl), ckpt_K=16)
    torch.cuda.synchronize()
    cert = res["cert"].cpu().numpy()
    assert (cert == 1).mean() > 0.999
    _check(wl, res, [0, 31337, 65535] + list(np.where(cert != 1)[0][:2]), random=24, seed=1)


@pytest.mark.parametrize("tail", [0, 100], ids=["one_launch", "tail_handoff"])
def test_hopf_n10_full_size_sampled(hj, tail):
    """4096 points x 16 guesses on one lane per task with checkpoints every
    16 steps (4 in the LDS plan), alone and, as the headline benchmark times
    it, with the slots still descending after 100 evaluations handed to a
    two-lane continuation launch."""
    wl = W.c1_hopf_n10(B=4096)
    res = hj.solve(wl, *hj.device_inputs(wl), lanes_per_task=1, ckpt_K=16, tail_budget=tail,
                   tail_lanes_per_task=2 if tail else 0)
    torch.cuda.synchronize()
    cert = res["cert"].cpu().numpy()
    assert (cert == 1).mean() > 0.999
    _check(wl, res, [0, 1111, 2048, 4095] + list(np.where(cert != 1)[0][:2]), random=40,
           seed=2)


def test_hopf_n10_central_fd_full_size_sampled(hj):
    """The central-difference coordinate descent of the n=10 workload over all
    4096 points (the comparison leg of the benchmark), sampled points
    including every point it leaves uncertified."""
    wl = W.c1_hopf_n10(B=4096, mode=W.CD_FD)
    res = hj.solve(wl, *hj.device_inputs(wl), lanes_per_task=1)
    torch.cuda.synchronize()
    cert = res["cert"].cpu().numpy()
    assert (cert == 1).mean() > 0.999
    _check(wl, res, [0, 2048, 4095] + list(np.where(cert != 1)[0][:3]), random=16, seed=3)


def test_lax_n100_fp32_full_size_sampled(hj):
    """262144 points x 4 guesses, FP32 descent with the FP64 certificate, in
    a persistent launch (more tasks than resident lane groups), on 16 lanes
    of 7 components per task at two waves per SIMD."""
    wl = W.c4_lax_n100()
    res = hj.solve(wl, *hj.device_inputs(wl), lanes_per_task=16, ckpt_K=8)
    torch.cuda.synchronize()
    cert = res["cert"].cpu().numpy()
    assert (cert == 1).mean() > 0.999
    _check(wl, res, [0, 123457, 262143] + list(np.where(cert != 1)[0][:2]), random=64,
           seed=4)


@pytest.mark.parametrize("dtype", [W.F64, W.F32])
def test_batched_full_size_sampled(hj, dtype):
    """All 64 instances in one captured plan; three points (the first, the
    last, one drawn) of each of sixteen instances (different n, t, N) and up
    to eight uncertified points against the reference, certificate flags
    compared per point in both dtypes."""
    wls = W.c2_batched(dtype=dtype)
    plan = hj.BatchPlan(wls)
    outs = plan.run()
    torch.cuda.synchronize()
    tot = sum(w.B for w in wls)
    ncert = sum(int((o["cert"] == 1).sum().item()) for o in outs)
    assert ncert / tot > 0.999, (ncert, tot)
    band = []
    unc = [(i, int(b)) for i, o in enumerate(outs)
           for b in np.where(o["cert"].cpu().numpy() != 1)[0]][:8]
    rng = np.random.default_rng(5)
    picks = {}
    for i in range(0, 64, 4):
        picks.setdefault(i, []).extend([0, wls[i].B - 1, int(rng.integers(wls[i].B))])
    for i, b in unc:
        picks.setdefault(i, []).append(b)
    for i, pts in picks.items():
        _check(wls[i], outs[i], pts, band)
    assert len(band) <= 2, band
    plan.free()
