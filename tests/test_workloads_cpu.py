"""The seeded extension workloads that bench.py times: they are the settings the
tests pin (Table VIII's bounded example), stable, and reproducible."""
import json
import os

import numpy as np

from oracle import lbm_oracle as O
from paper_0907_1720_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_table8_workload_is_the_pinned_table_setting():
    with open(os.path.join(HERE, "golden", "paper_tables.json")) as fh:
        t = json.load(fh)["table_VIII_s1"]
    p, x, ex = W.table8_bounded()
    assert (p.dx, p.dt, p.tau, p.lattice()) == (t["dx"], t["dt"], t["tau"], t["lattice"])
    assert (x[0], x[-1]) == tuple(t["domain"]) and p.n == x.size and p.bc == 2
    # 100 steps of the oracle's bounded mode stay at the paper's error level
    out = O.run_bounded(W.Problem(p.alpha, p.pi, p.n, p.dx, p.dt, p.tau, q=5), x, ex, 100, "nee", report=[100])
    assert O.global_relative_error(out[100], ex(x, 1.0)) < 1e-5


def test_extension_batches_are_seeded_and_positive():
    a = W.power_batch_instance(3)
    b = W.power_batch_instance(3)
    assert a.problem == b.problem and np.array_equal(a.phi0, b.phi0)
    assert a.phi0.min() >= 1.0 and a.problem.gpi[1][0][0] in (1.5, 2.5)
    for q in (4, 6):
        e = W.even_lattice_instance(5, q)
        assert e.problem.lattice() == q and 256 <= e.problem.n <= 4096
