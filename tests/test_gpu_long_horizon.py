"""Long-horizon parity at full size, in the launch configuration the benchmark
times: the 1024-run Kuramoto-Sivashinsky batches (N = 1024, 4096, 8192) to
t = 5, 10 and 20, and the 512-instance Kawahara + K(2,2) batch for 5000 steps,
in FP64 and in FP32 deviation storage.  Sampled instances are compared element
by element with reference states that tests/golden/make_long_horizon.py wrote
with the CPU oracle alone; every instance must stay finite and conserve sum
phi.  Config 4's results are also compared with the closed-form solutions.

Tolerances (relative L2 and max-abs relative to max |phi|, both asserted).
FP64: 1e-12, or five times the distance between two FP64 evaluation orders of
the oracle itself where that is larger.  Over 10^5 steps the scheme carries
rounding forward: the oracle against itself in another order differs by up to
3.7e-12 at N = 8192, t = 20 (tau = 20), while a relative change of 1e-15 in
phi0 moves the result by at most 1e-13 -- the rounding of every step, not the
initial state, sets the attainable agreement (both measures are stored with
the references).  FP32 deviation storage: Kuramoto-Sivashinsky 1e-3 at
N = 1024 and 3e-3 at N = 4096, 8192 (tau = 10, 20: the stored deviations'
rounding accumulates over more, more weakly relaxed steps), config 4 1e-4.
Against the closed forms: the scheme's own error (N = 2048) or, at N = 16384,
the FP32 storage rounding dominates; bounds 6e-4 and 1e-4.  The measured
errors are printed.
"""
import os
import sys

import numpy as np
import pytest

from paper_0907_1720_amd import lbm
from paper_0907_1720_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "long_horizon.npz")
FP64_TOL = 1e-12
FP32_TOL_KS = {1024: 1e-3, 4096: 3e-3, 8192: 3e-3}
FP32_TOL = 1e-4
KS_TIMES = (5, 10, 20)


def fp64_tols(gold, key):
    """(relL2, max-abs) tolerance: 1e-12 or 5x the oracle's order distance."""
    o2, om = gold[key + "_order"]
    return max(FP64_TOL, 5 * o2), max(FP64_TOL, 5 * om)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lbm.library()
    yield


@pytest.fixture(scope="module")
def gold():
    return dict(np.load(GOLD))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def errs(got, want):
    """(relative L2, max-abs relative to max |want|)"""
    return (float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            float(np.max(np.abs(got - want)) / np.max(np.abs(want))))


@pytest.mark.parametrize("prec", [W.F64, W.F32_DEV])
@pytest.mark.parametrize("n", [1024, 4096, 8192])
def test_config3_ks_batch_to_t20(gold, n, prec):
    insts = [W.config3_instance(n, i, prec=prec) for i in range(1024)]
    marks = [int(gold[f"ks_n{n}_i0_t{t}_steps"]) for t in KS_TIMES]
    say("case config3 batch n", n, "prec", prec, "marks", marks)
    b = lbm.Batch([i.problem for i in insts])
    b.load_phi([i.phi0 for i in insts])
    done = 0
    for t, m in zip(KS_TIMES, marks):
        b.advance(m - done)
        done = m
        for i in (0, 1023):
            key = f"ks_n{n}_i{i}_t{t}"
            if key not in gold:
                continue
            got, st = b.read_phi(i)
            assert st == lbm.OK
            e2, em = errs(got, gold[key])
            s2, sm = gold[key + "_sens"]
            o2, om = gold[key + "_order"]
            t2, tm = fp64_tols(gold, key) if prec == W.F64 else (FP32_TOL_KS[n],) * 2
            say(f"  t={t} inst {i}: relL2 {e2:.2e} maxabs {em:.2e} (oracle: other FP64 order {o2:.1e} {om:.1e}, "
                f"phi0 (1 + 1e-15) {s2:.1e} {sm:.1e})")
            assert e2 <= t2 and em <= tm, (key, e2, em, t2, tm)
    # every run finite, sum phi conserved
    drift = 0.0
    for i, inst in enumerate(insts):
        got, st = b.read_phi(i)
        assert st == lbm.OK, i
        drift = max(drift, abs(got.sum() - inst.phi0.sum()) / np.abs(inst.phi0).sum())
    b.close()
    say(f"  worst sum-phi drift over 1024 runs {drift:.2e}")
    assert drift <= (1e-12 if prec == W.F64 else 1e-4)


@pytest.mark.parametrize("prec", [W.F64, W.F32_DEV])
def test_config4_batch_5000_steps(gold, prec):
    insts = [W.config4_instance(i, prec=prec) for i in range(512)]
    say("case config4 batch prec", prec)
    b = lbm.Batch([i.problem for i in insts])
    b.load_phi([i.phi0 for i in insts])
    b.advance(5000)
    for i in range(4):
        got, st = b.read_phi(i)
        assert st == lbm.OK
        want = gold[f"c4_i{i}"]
        e2, em = errs(got, want)
        t2, tm = fp64_tols(gold, f"c4_i{i}") if prec == W.F64 else (FP32_TOL, FP32_TOL)
        ex = insts[i].exact(5000 * insts[i].problem.dt)
        ge = float(np.linalg.norm(got - ex) / np.linalg.norm(ex))
        oe = float(gold[f"c4_i{i}_exact_rel2"])
        say(f"  inst {i} {insts[i].problem.name} n={insts[i].problem.n}: vs oracle relL2 {e2:.2e} maxabs {em:.2e}; "
            f"vs closed form {ge:.4e} (oracle {oe:.4e})")
        assert e2 <= t2 and em <= tm, (i, e2, em)
        assert ge <= (6e-4 if insts[i].problem.n == 2048 else 1e-4), ge
    drift = 0.0
    for i, inst in enumerate(insts):
        got, st = b.read_phi(i)
        assert st == lbm.OK, i
        drift = max(drift, abs(got.sum() - inst.phi0.sum()) / np.abs(inst.phi0).sum())
    b.close()
    say(f"  worst sum-phi drift over 512 instances {drift:.2e}")
    assert drift <= (1e-12 if prec == W.F64 else 1e-4)
