"""Host logic of the serving measurement: the Poisson driver against a
simulated server (no GPU), and the knee of a sweep."""
import numpy as np

import bench
from paper_0907_1720_amd import serving


class _Problem:
    def __init__(self, n):
        self.n = n


class _Request:
    def __init__(self, n, steps):
        self.problem = _Problem(n)
        self.phi0 = np.zeros(n)
        self.steps = steps


class _SimServer:
    """Rounds of `block` steps that take `round_s` seconds each; requests are
    admitted when a round starts and retired when it ends, as the library's
    pump does."""

    def __init__(self, block=100, round_s=2e-3):
        import time
        self.time = time
        self.block, self.round_s = block, round_s
        self.queue, self.active, self.done = [], {}, {}
        self.nu = 0.0
        self.round_end = None
        self.round_steps = {}
        self.next_id = 1
        self.t_sub, self.t_adm, self.t_ret = {}, {}, {}

    def submit(self, p, phi0, steps):
        rid = self.next_id
        self.next_id += 1
        self.queue.append((rid, p.n, steps))
        self.t_sub[rid] = self.time.perf_counter()
        return rid

    def pump(self):
        now = self.time.perf_counter()
        retired = 0
        if self.round_end is not None:
            if now < self.round_end:
                return 1, len(self.active), len(self.queue), 0
            for rid, k in self.round_steps.items():
                n, left = self.active[rid]
                self.nu += n * k
                left -= k
                if left == 0:
                    del self.active[rid]
                    self.done[rid] = np.full(n, float(rid))
                    self.t_ret[rid] = now
                    retired += 1
                else:
                    self.active[rid] = (n, left)
            self.round_end = None
        for rid, n, steps in self.queue:
            self.active[rid] = (n, steps)
            self.t_adm[rid] = now
        self.queue = []
        if self.active:
            self.round_steps = {rid: min(self.block, left) for rid, (n, left) in self.active.items()}
            self.round_end = now + self.round_s
        return int(bool(self.active)), len(self.active), 0, retired

    def poll(self, rid):
        if rid not in self.done:
            return None
        return self.done.pop(rid), 0

    def timing(self, rid):
        return self.t_adm[rid] - self.t_sub[rid], self.t_ret[rid] - self.t_adm[rid]

    def stats(self):
        return self.nu, 0.0, 0


def test_poisson_driver_accounts_every_request():
    reqs = [_Request(100 + 7 * i, 100 * (1 + i % 4)) for i in range(40)]
    srv = _SimServer(block=100, round_s=2e-3)
    out = serving.run_poisson(srv, reqs, rate=400.0, seed=3, keep_results=True)
    total = sum(r.problem.n * r.steps for r in reqs)
    assert out["requests"] == 40 and out["nonfinite"] == 0
    assert out["node_updates"] == total
    # every result is its own request's (the simulated server fills phi with the id)
    for i, res in enumerate(out["results"]):
        assert res.shape == (reqs[i].problem.n,) and np.all(res == res[0])
    assert np.all(out["latency"] > 0) and np.all(out["queue_wait"] >= 0)
    # a request of s steps needs s / block rounds after its admission
    assert out["p50_service_s"] >= 2e-3
    assert 0.0 <= out["p50_latency_s"] <= out["p99_latency_s"]
    # the work finished by the last arrival is part of all the work, over less time
    span = out["arrival_span_s"]
    assert out["window_node_updates_per_s"] * span <= total + 1e-9
    assert out["offered_node_updates_per_s"] == total / span
    assert out["node_updates_per_s"] == total / out["wall_s"]


def test_knee_is_first_rate_below_the_fraction():
    sweep = [
        {"rate_per_s": 32.0, "offered_node_updates_per_s": 1.0e9, "window_node_updates_per_s": 0.98e9},
        {"rate_per_s": 64.0, "offered_node_updates_per_s": 2.0e9, "window_node_updates_per_s": 1.7e9},
        {"rate_per_s": 128.0, "offered_node_updates_per_s": 4.0e9, "window_node_updates_per_s": 3.1e9},
        {"rate_per_s": 256.0, "offered_node_updates_per_s": 8.0e9, "window_node_updates_per_s": 4.0e9},
    ]
    assert bench.serving_knee(sweep) == 128.0
    assert bench.serving_knee(sweep, frac=0.9) == 64.0
    assert bench.serving_knee(sweep[:2]) is None
    # a rate whose window saw nothing finish counts as below
    assert bench.serving_knee([dict(sweep[0], window_node_updates_per_s=None)]) == 32.0
