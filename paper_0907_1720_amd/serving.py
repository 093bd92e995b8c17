"""Serving driver: Poisson arrivals of solve requests into an lbm.Server.

The scheduling (admission by arena budget, step blocks, retirement) is the
library's; this loop only releases requests at their arrival times, runs
scheduling rounds and records completion times.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np

from . import lbm


def run_poisson(server: "lbm.Server", requests: Sequence, rate: float, seed: int = 0,
                keep_results: bool = False) -> Dict:
    """requests: objects with .problem, .phi0, .steps.  rate: arrivals per second."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20261203, 5, seed])))
    arrivals = np.cumsum(g.exponential(1.0 / rate, len(requests)))
    arrivals -= arrivals[0]
    nu0, ms0, _ = server.stats()
    t0 = time.perf_counter()
    nxt = 0
    outstanding: Dict[int, int] = {}
    latency = np.full(len(requests), np.nan)
    results: List = [None] * len(requests)
    statuses = np.zeros(len(requests), dtype=np.int32)
    queued = active = 0
    while nxt < len(requests) or outstanding:
        now = time.perf_counter() - t0
        while nxt < len(requests) and arrivals[nxt] <= now:
            r = requests[nxt]
            outstanding[server.submit(r.problem, r.phi0, r.steps)] = nxt
            nxt += 1
        if not outstanding:
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
            continue
        active, queued, retired = server.step()
        if retired:
            t = time.perf_counter() - t0
            for rid in list(outstanding):
                res = server.poll(rid)
                if res is None:
                    continue
                i = outstanding.pop(rid)
                latency[i] = t - arrivals[i]
                statuses[i] = res[1]
                if keep_results:
                    results[i] = res[0]
    wall = time.perf_counter() - t0
    nu1, ms1, _ = server.stats()
    out = {
        "requests": len(requests),
        "rate_per_s": rate,
        "wall_s": wall,
        "node_updates": nu1 - nu0,
        "node_updates_per_s": (nu1 - nu0) / wall,
        "device_ms": ms1 - ms0,
        "p50_latency_s": float(np.percentile(latency, 50)),
        "p99_latency_s": float(np.percentile(latency, 99)),
        "mean_latency_s": float(np.mean(latency)),
        "nonfinite": int(np.sum(statuses != 0)),
    }
    if keep_results:
        out["results"] = results
        out["latency"] = latency
    return out
