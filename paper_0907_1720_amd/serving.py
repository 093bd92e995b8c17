"""Serving driver: Poisson arrivals of solve requests into an lbm.Server.

The scheduling (admission by arena budget, step blocks, retirement) is the
library's; this loop only releases requests at their arrival times, pumps the
server's non-blocking rounds (lbm_server_pump) and records per-request
latency and queue wait.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np

from . import lbm


def arrival_times(count: int, rate: float, seed: int = 0) -> np.ndarray:
    """Poisson arrivals (seconds from the first) of `count` requests at `rate` per second."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20261203, 5, seed])))
    t = np.cumsum(g.exponential(1.0 / rate, count))
    return t - t[0]


def run_poisson(server: "lbm.Server", requests: Sequence, rate: float, seed: int = 0,
                keep_results: bool = False) -> Dict:
    """requests: objects with .problem, .phi0, .steps.  rate: arrivals per second.

    Requests are submitted when their arrival time has passed; between
    arrivals the loop pumps the server, which admits, launches and retires
    rounds without blocking.  Latency = completion (seen by the loop) minus
    arrival; queue wait = admission minus arrival.  node_updates_per_s divides
    all the work by the wall time including the drain after the last arrival;
    window_node_updates_per_s counts only the rounds finished by the last
    arrival, over that time (the rate the server keeps up with while requests
    arrive)."""
    arrivals = arrival_times(len(requests), rate, seed)
    nu0, ms0, _ = server.stats()
    t0 = time.perf_counter()
    nxt = 0
    outstanding: Dict[int, int] = {}
    submitted = np.zeros(len(requests))
    latency = np.full(len(requests), np.nan)
    queue_wait = np.full(len(requests), np.nan)
    service = np.full(len(requests), np.nan)
    results: List = [None] * len(requests)
    statuses = np.zeros(len(requests), dtype=np.int32)
    sizes = np.array([r.problem.n * r.steps for r in requests], dtype=np.float64)
    running = 0
    nu_window = None
    while nxt < len(requests) or outstanding:
        now = time.perf_counter() - t0
        while nxt < len(requests) and arrivals[nxt] <= now:
            r = requests[nxt]
            outstanding[server.submit(r.problem, r.phi0, r.steps)] = nxt
            submitted[nxt] = now
            nxt += 1
            if nxt == len(requests):
                # work finished while the arrivals lasted (rounds are counted when they end)
                nu_window = (server.stats()[0] - nu0, now)
        if not outstanding:
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
            continue
        running, _, _, retired = server.pump()
        if retired or not running:
            t = time.perf_counter() - t0
            for rid in list(outstanding):
                res = server.poll(rid)
                if res is None:
                    continue
                i = outstanding.pop(rid)
                latency[i] = t - arrivals[i]
                qs, ss = server.timing(rid)
                queue_wait[i] = (submitted[i] - arrivals[i]) + qs
                service[i] = ss
                statuses[i] = res[1]
                if keep_results:
                    results[i] = res[0]
        if running:
            # the round is on the device: wait a little (50 us: the GPU idles from
            # a round's end until the next pump launches the next one), or until
            # the next arrival
            nxt_t = arrivals[nxt] - (time.perf_counter() - t0) if nxt < len(requests) else 1e-3
            time.sleep(max(0.0, min(5e-5, nxt_t)))
    wall = time.perf_counter() - t0
    nu1, ms1, _ = server.stats()
    span = float(arrivals[-1]) if len(arrivals) > 1 else 0.0
    out = {
        "requests": len(requests),
        "rate_per_s": rate,
        "wall_s": wall,
        "arrival_span_s": span,
        "offered_node_updates_per_s": float(sizes.sum() / span) if span > 0 else None,
        "node_updates": nu1 - nu0,
        "node_updates_per_s": (nu1 - nu0) / wall,
        "window_node_updates_per_s": (nu_window[0] / nu_window[1]
                                      if nu_window is not None and nu_window[1] > 0 else None),
        "device_ms": ms1 - ms0,
        "p50_latency_s": float(np.percentile(latency, 50)),
        "p99_latency_s": float(np.percentile(latency, 99)),
        "mean_latency_s": float(np.mean(latency)),
        "p50_queue_wait_s": float(np.percentile(queue_wait, 50)),
        "p99_queue_wait_s": float(np.percentile(queue_wait, 99)),
        "mean_queue_wait_s": float(np.mean(queue_wait)),
        "p50_service_s": float(np.percentile(service, 50)),
        "nonfinite": int(np.sum(statuses != 0)),
    }
    if keep_results:
        out["results"] = results
        out["latency"] = latency
        out["queue_wait"] = queue_wait
        out["statuses"] = statuses
    return out
