"""The tuner's choice of a tail hand-off, with the timings replaced by a
table (no GPU): the fastest budget wins unless a larger one is within 1.5%,
no hand-off unless it gains 2%, and only FP64 adjoint descents without drift
are tuned."""
import pytest

from paper_1704_02524_amd import tune
from paper_1704_02524_amd import workloads as W


def _fake(monkeypatch, table, none_ms):
    def time_config(wl, x, g, cfg, reps=2, warm=True):
        if "tail_budget" not in cfg:
            return none_ms
        return table.get((cfg["tail_budget"], cfg["tail_lanes_per_task"]))
    monkeypatch.setattr(tune, "time_config", time_config)
    monkeypatch.setattr(tune.hj, "device_inputs", lambda wl: (None, None))


def test_fastest_budget_and_near_ties(monkeypatch):
    wl = W.c1_hopf_n10(B=8)  # max_iter 200: budgets 80, 100, 121, 141, 161
    table = {(80, 2): 140.0, (100, 2): 125.0, (121, 2): 116.6, (141, 2): 121.0,
             (161, 2): 124.0, (141, 4): 123.0}
    _fake(monkeypatch, table, 144.0)
    assert tune.tune_tail(wl, {"lanes_per_task": 1})["config"] == \
        {"tail_budget": 121, "tail_lanes_per_task": 2}
    # a larger budget within 1.5 % of the fastest is preferred
    table[(141, 2)] = 117.5
    assert tune.tune_tail(wl, {})["config"]["tail_budget"] == 141


def test_no_hand_off_without_a_gain(monkeypatch):
    wl = W.c1_hopf_n10(B=8)
    _fake(monkeypatch, {(121, 2): 143.0}, 144.0)
    assert tune.tune_tail(wl, {})["config"] == {}


@pytest.mark.parametrize("over", [dict(dtype=W.F32), dict(mode=W.CD_FD)])
def test_only_fp64_adjoint_descents(monkeypatch, over):
    wl = W.c1_hopf_n10(B=8).with_(**over)
    _fake(monkeypatch, {(121, 2): 100.0}, 144.0)
    assert tune.tune_tail(wl, {})["config"] == {}
