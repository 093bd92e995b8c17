"""Autotuning cache: planner settings per batch shape.

The native tuner (lbm_batch_autotune) times candidate settings on a copy of a
batch.  This module keys its result on the batch shape -- the count of
instances per (lattice size q, precision, N bucket of powers of two) and the
probe step count -- and keeps it in a JSON file, so that a later batch of the
same shape takes the settings without timing them again.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional, Sequence

from . import lbm
from .workloads import Problem


def shape_key(problems: Sequence[Problem], probe_steps: int) -> str:
    hist: dict = {}
    for p in problems:
        k = (p.lattice(), int(p.prec), int(math.floor(math.log2(max(1, p.n)))))
        hist[k] = hist.get(k, 0) + 1
    parts = [f"q{q}p{pr}n{b}x{c}" for (q, pr, b), c in sorted(hist.items())]
    return f"steps{int(probe_steps)}|" + ",".join(parts)


def tuned(batch: "lbm.Batch", problems: Sequence[Problem], probe_steps: int,
          cache_path: Optional[str] = None) -> dict:
    """Applies cached settings for this batch shape, or tunes and caches them."""
    key = shape_key(problems, probe_steps)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        batch.apply_tuning(cache[key])
        return dict(cache[key], cached=True)
    t = batch.autotune(probe_steps)
    if cache_path:
        cache[key] = t
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return dict(t, cached=False)
