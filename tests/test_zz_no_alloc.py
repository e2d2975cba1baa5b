"""hj_solve_noalloc, the entry point for callers that cannot allocate device
memory: through the C interface its results equal hj_solve's, on two calls
in a row (the second smaller, so it runs in what the first left in the
shared scratch), including a solve that only fits the fixed scratch as a
persistent launch with fewer lane groups; a solve too large for it is
refused with HJ_ENOMEM."""
import numpy as np
import pytest
import torch

from paper_1704_02524_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_02524_amd import hj as _hj
    return _hj


def _host(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _same(a, b):
    for k in a:
        np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]), err_msg=k)


@pytest.mark.parametrize("dtype", [W.F64, W.F32])
def test_noalloc_equals_solve_on_two_calls(hj, dtype):
    wl = W.c1_hopf_n10(B=4096)
    if dtype == W.F32:
        wl = W._as_dtype(wl.with_(eps_step=1e-6, cert_tol=1e-4))
    big = wl.subset(0, 1024)      # 16384 slots: needs a persistent launch to fit
    small = wl.subset(1024, 1100)  # 1216 slots, a partial last wave
    xb, gb = hj.device_inputs(big)
    xs, gs = hj.device_inputs(small)
    ref_b = _host(hj.solve(big, xb, gb))
    ref_s = _host(hj.solve(small, xs, gs))
    got_b = _host(hj.solve(big, xb, gb, noalloc=True))
    got_s = _host(hj.solve(small, xs, gs, noalloc=True))
    torch.cuda.synchronize()
    _same(got_b, ref_b)
    _same(got_s, ref_s)
    assert (got_b["cert"] == 1).mean() > 0.99


def test_noalloc_refuses_a_solve_larger_than_its_scratch(hj):
    wl = W.c1_hopf_n10(B=4096)
    big = wl.with_(x=np.repeat(wl.x, 16, 0), guesses=np.repeat(wl.guesses, 16, 0))
    x, g = hj.device_inputs(big)
    with pytest.raises(hj.HJError, match="scratch"):
        hj.solve(big, x, g, noalloc=True)
