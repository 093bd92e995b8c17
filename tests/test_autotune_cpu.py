"""Autotuning cache logic (host only): the shape key and the JSON cache."""
import json

from paper_0907_1720_amd import autotune
from paper_0907_1720_amd import workloads as W


def _probs(sizes, prec=W.F32_DEV):
    return [W.kdv(1.0, n, 40.0 / n, 1e-6, 2.0, -20.0, prec=prec) for n in sizes]


def test_shape_key_counts_buckets_not_order():
    a = autotune.shape_key(_probs([300, 5000, 700, 260]), 500)
    b = autotune.shape_key(_probs([260, 700, 5000, 300]), 500)
    assert a == b
    assert "n8x2" in a and "n9x1" in a and "n12x1" in a
    assert autotune.shape_key(_probs([300]), 500) != autotune.shape_key(_probs([300]), 501)
    assert autotune.shape_key(_probs([300], W.F64), 500) != autotune.shape_key(_probs([300]), 500)


class _FakeBatch:
    def __init__(self):
        self.tuned = 0
        self.applied = None

    def autotune(self, probe_steps):
        self.tuned += 1
        return {"path": 0, "tile_steps": 16, "tile_wgs": 2, "res_chunks": 4, "candidates": 9,
                "best_node_updates_per_s": 2.0, "default_node_updates_per_s": 1.0}

    def apply_tuning(self, t):
        self.applied = t


def test_cache_hit_applies_without_timing(tmp_path):
    path = str(tmp_path / "tune.json")
    probs = _probs([300, 700])
    b1 = _FakeBatch()
    t1 = autotune.tuned(b1, probs, 100, path)
    assert b1.tuned == 1 and not t1["cached"]
    assert json.load(open(path))[autotune.shape_key(probs, 100)]["tile_steps"] == 16
    b2 = _FakeBatch()
    t2 = autotune.tuned(b2, probs, 100, path)
    assert b2.tuned == 0 and t2["cached"] and b2.applied["res_chunks"] == 4
