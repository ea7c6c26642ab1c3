"""Autotuner host logic (no GPU): cache keys, cached shapes applied without
timing, and the coordinate-descent pick on a fake graph whose job time is a
known function of the shape."""
import numpy as np

from paper_1710_01144_amd import tune


class FakeGraph:
    def __init__(self, cost):
        self.row_ptr = np.array([0, 2, 3, 5, 6], dtype=np.int32)
        self.shape = {"unroll": 8, "unroll_small": 4, "min_edges": 512, "min_edges_small": 512,
                      "level_wgs_per_cu": 4}
        self.cost = cost
        self.jobs = 0

    def get_tuning(self):
        return dict(self.shape)

    def set_tuning(self, **kw):
        self.shape.update(kw)

    def greedy_group(self, k, order="plain", block=0, mlp_params=None, block_growth=0):
        self.jobs += 1
        cost = self.cost(self.shape)
        if block_growth:
            cost += abs(block - 128) / 100.0 + abs(block_growth - 4) / 10.0
        return [0, 1], [5, 3], {"ms_total": cost}


def _cost(s):
    # best at unroll 16, min_edges_small 128, level_wgs_per_cu 2; others neutral
    return (10.0 + (0 if s["unroll"] == 16 else 1) + abs(s["min_edges_small"] - 128) / 1000.0
            + (0 if s["level_wgs_per_cu"] == 2 else 0.5))


def test_signature_and_key():
    g = FakeGraph(_cost)
    sig = tune.signature(g)
    assert sig.startswith("n4-nnz6-maxdeg2-")
    assert tune.job_key(sig, 50, "plain", 64) == sig + "|k50|plain|b64"


def test_coordinate_descent_and_cache(tmp_path):
    path = str(tmp_path / "tune.json")
    g = FakeGraph(_cost)
    out = tune.autotune(g, 5, cache_path=path, reps=1)
    assert not out["cached"]
    assert out["shape"] == {"unroll": 16, "unroll_small": 4, "min_edges": 512, "min_edges_small": 128,
                            "level_wgs_per_cu": 2}
    assert g.get_tuning() == out["shape"]
    assert out["ms_tuned"] < out["ms_default"]
    # one timing per grid value other than the starting one, plus the start
    assert out["trials"] == 1 + sum(len(v) - 1 for v in tune.GRID.values())
    g2 = FakeGraph(_cost)
    out2 = tune.autotune(g2, 5, cache_path=path, reps=1)
    assert out2["cached"] and g2.jobs == 0 and g2.get_tuning() == out["shape"]
    # another job size is a separate entry
    g3 = FakeGraph(_cost)
    assert not tune.autotune(g3, 6, cache_path=path, reps=1)["cached"]


def test_schedule_tuner_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "tune.json")
    g = FakeGraph(_cost)
    out = tune.autotune_schedule(g, 5, cache_path=path, reps=1)
    assert (out["block"], out["growth"]) == (128, 4) and not out["cached"]
    assert out["ms"] < out["ms_default"]
    assert len(out["table"]) == len(tune.SCHEDULES)
    g2 = FakeGraph(_cost)
    out2 = tune.autotune_schedule(g2, 5, cache_path=path, reps=1)
    assert out2["cached"] and g2.jobs == 0 and out2["block"] == 128


def test_schedule_tuner_rejects_changed_picks():
    class Flaky(FakeGraph):
        def greedy_group(self, k, order="plain", block=0, mlp_params=None, block_growth=0):
            self.jobs += 1
            return [block % 3, 1], [5, 3], {"ms_total": 1.0}
    import pytest
    with pytest.raises(AssertionError):
        tune.autotune_schedule(Flaky(_cost), 5, schedules=[(32, 1), (64, 1)], reps=1)
