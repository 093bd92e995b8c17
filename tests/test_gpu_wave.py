"""Travelling-wave boundary values evaluated on the device
(lbm_advance_bounded_wave, lbm_batch_advance_bounded_wave, lbm_wave_rows).

The closed forms of the paper's bounded examples (Sec. IV; Tables I, II and
IV-VIII) are written below in numpy from the same definitions the oracle's
table pins use; the device rows must agree with them to a few ulps, and a
bounded run fed by device rows must agree with the same run fed by host rows
(<= 1e-13 in relative L2, every element 2e-13 of max |phi|: the rows differ by
the last bits of exp/cosh/tanh) and with the CPU oracle (<= 1e-12).  Device rows are deterministic, so the
resident and streaming paths and batch vs single solves agree bit for bit.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest

from oracle import lbm_oracle as O
from paper_0907_1720_amd import lbm
from paper_0907_1720_amd import workloads as W
from test_oracle_pins import _table_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lbm.library()
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def maxerr(a, b):
    """The relative L2 error, or half the largest element error relative to
    max |b| where that is larger: a tolerance `tol` on it bounds the L2 error by
    tol and every element by 2 tol (a rounding-driven difference peaks at up to
    about twice its L2 size; 1.6x measured here)."""
    return max(float(np.linalg.norm(a - b) / np.linalg.norm(b)),
               0.5 * float(np.max(np.abs(a - b)) / np.max(np.abs(b))))


def rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def np_wave(w, x, t):
    """phi* = a + b h(z)^p + d h(z)^r, z = k (x - xc - c t), in numpy."""
    z = w["k"] * (x - w["xc"] - w["c"] * t)
    h = {"sech": lambda: 1.0 / np.cosh(z),
         "tanh": lambda: np.tanh(z),
         "logistic": lambda: 1.0 / (1.0 + np.exp(z)),
         "cos": lambda: np.where(np.abs(z) <= np.pi / 2, np.cos(z), 0.0)}[w["shape"]]()
    return w["a"] + w["b"] * h ** w["p"] + w.get("d", 0.0) * h ** w.get("r", 0.0)


# the tables' closed forms as waves (see _table_problem)
s3, s2 = math.sqrt(3), math.sqrt(2)
TABLE_WAVES = {
    "table_VI_s1_c10": dict(shape="sech", a=0.0, b=-3 / math.sqrt(10), p=2.0, k=0.5 * math.sqrt(0.2), xc=0.0, c=0.16),
    "table_V_s1_c10": dict(shape="sech", a=0.0, b=105 / 169, p=4.0, k=1 / (2 * math.sqrt(13)), xc=0.0, c=36 / 169),
    "table_IV_q7_c10": dict(shape="tanh", a=1 / 6, b=s3 / (2 * s2), p=1.0, k=s3 / (4 * s2),
                            xc=-0.5 / (s3 / (4 * s2)), c=29 / 144),
    "table_VIII_s1": W.table8_wave(),
    "table_VII_s1_c10": dict(shape="sech", a=0.0, b=105 / 169, p=4.0, k=1 / (2 * math.sqrt(13)), xc=20.0,
                             c=205 / 169),
    "table_II_c10": dict(shape="tanh", a=5.0, b=-3 * 15 / (19 * math.sqrt(19)), p=1.0,
                         d=15 / (19 * math.sqrt(19)), r=3.0, k=1 / (2 * math.sqrt(19)), xc=-25.0, c=5.0),
    "table_I_c10": dict(shape="tanh", a=5.0, b=-9 * (15 / 19) * math.sqrt(11 / 19), p=1.0,
                        d=11 * (15 / 19) * math.sqrt(11 / 19), r=3.0, k=0.5 * math.sqrt(11 / 19), xc=-12.0, c=5.0),
}


def _wave(w, x_first, t0=0.0):
    return lbm.make_wave(w["shape"], w["a"], w["b"], w["p"], w["k"], w["xc"], w["c"], x_first, t0,
                         d=w.get("d", 0.0), r=w.get("r", 0.0))


def _bounded(p, kind):
    return dataclasses.replace(p, bc=lbm.BC_DIRICHLET_EQ if kind == "eq" else lbm.BC_DIRICHLET_NEE)


@pytest.mark.parametrize("key", sorted(TABLE_WAVES))
def test_table_waves_are_the_tables_closed_forms(key):
    """The wave parameters reproduce each table's exact solution (numpy only)."""
    t, p, x, ex, kind = _table_problem(key)
    for tt in (0.0, 0.7, 3.1):
        assert np.allclose(np_wave(TABLE_WAVES[key], x, tt), ex(x, tt), rtol=1e-14, atol=1e-15)


EXTRA_WAVES = {
    "sech_real_power": dict(shape="sech", a=1.0, b=0.3, p=1.5, k=0.4, xc=-2.0, c=0.7),
    "logistic_two_terms": dict(shape="logistic", a=0.2, b=1.0, p=2.0, d=-0.5, r=0.5, k=-1.3, xc=1.0, c=-0.2),
    "compacton": dict(shape="cos", a=0.0, b=4 / 3, p=2.0, k=0.25, xc=-3.0, c=1.0),
}


@pytest.mark.parametrize("key", sorted(TABLE_WAVES) + sorted(EXTRA_WAVES))
def test_device_rows_match_numpy(key):
    w = TABLE_WAVES.get(key) or EXTRA_WAVES[key]
    n, dx, dt, layers, steps, x_first, t0 = 201, 0.1, 0.01, 3, 400, -10.0, 0.37
    p = _bounded(W.kdv_burgers(2.0, 0.1, n, dx, dt, 1.5, x_first), "eq")
    s = lbm.Solver(p)
    rows = s.wave_rows(_wave(w, x_first, t0), steps, layers)
    s.close()
    nodes = np.r_[0:layers, n - layers:n]
    xb = x_first + nodes * dx
    tt = t0 + (np.arange(steps) + 1.0) * dt
    want = np_wave(w, xb[None, :], tt[:, None])
    say("case wave rows", key, float(np.max(np.abs(rows - want))))
    assert rows.shape == (steps, 2 * layers)
    assert np.allclose(rows, want, rtol=1e-14, atol=1e-15 * max(1.0, float(np.max(np.abs(want)))))


@pytest.mark.parametrize("key,steps", [("table_VI_s1_c10", 200), ("table_V_s1_c10", 120),
                                       ("table_IV_q7_c10", 100), ("table_VIII_s1", 500),
                                       ("table_VII_s1_c10", 150), ("table_II_c10", 1200),
                                       ("table_I_c10", 80)])
def test_wave_run_matches_host_rows_and_oracle(key, steps):
    t, p, x, ex, kind = _table_problem(key)
    bp = _bounded(p, kind)
    layers = p.lattice() // 2
    xb = np.concatenate([x[:layers], x[-layers:]])
    rows = np.stack([ex(xb, k * p.dt) for k in range(1, steps + 1)])
    s = lbm.Solver(bp)
    s.load_phi(ex(x, 0.0))
    s.advance_bounded(rows, layers)
    host = s.read_phi()
    s.load_phi(ex(x, 0.0))
    s.advance_bounded_wave(_wave(TABLE_WAVES[key], x[0]), steps, layers)
    dev = s.read_phi()
    s.close()
    want = O.run_bounded(p, x, ex, steps, kind, layers=layers, report=[steps])[steps]
    say("case wave run", key, f"{maxerr(dev, host):.2e}", f"{maxerr(dev, want):.2e}")
    assert maxerr(dev, host) <= 1e-13
    assert maxerr(dev, want) <= 1e-12


def test_wave_paths_agree_bitwise_and_calls_continue():
    """Resident and per-step streaming paths from the same device rows; two calls
    (the second with t0 advanced) equal one call."""
    t, p, x, ex, kind = _table_problem("table_VIII_s1")
    bp = _bounded(p, kind)
    w = TABLE_WAVES["table_VIII_s1"]
    outs = []
    for path in (lbm.PATH_AUTO, lbm.PATH_STREAM):
        s = lbm.Solver(bp)
        s.set_path(path)
        s.load_phi(ex(x, 0.0))
        s.advance_bounded_wave(_wave(w, x[0]), 300)
        outs.append(s.read_phi())
        s.close()
    assert np.array_equal(outs[0], outs[1])
    s = lbm.Solver(bp)
    s.load_phi(ex(x, 0.0))
    s.advance_bounded_wave(_wave(w, x[0]), 170)
    s.advance_bounded_wave(_wave(w, x[0], 170 * p.dt), 130)
    two = s.read_phi()
    s.close()
    assert np.array_equal(two, outs[0])


def test_batch_wave_sweep_equals_single_solves():
    t, p, x, ex, kind = _table_problem("table_VIII_s1")
    bp = _bounded(p, kind)
    w = _wave(TABLE_WAVES["table_VIII_s1"], x[0])
    taus = [0.97, 1.2, 1.7, 2.5]
    probs = [dataclasses.replace(bp, tau=tt) for tt in taus] + [W.kdv(0.5, 300, 0.1, 1e-4, 2.0, 0.0)]
    b = lbm.Batch(probs)
    b.load_phi([ex(x, 0.0)] * len(taus) + [np.full(300, 0.3)])
    b.advance_bounded_wave([w] * len(taus) + [None], 400)
    got = [b.read_phi(i)[0] for i in range(len(taus))]
    b.close()
    for tt, g in zip(taus, got):
        s = lbm.Solver(dataclasses.replace(bp, tau=tt))
        s.load_phi(ex(x, 0.0))
        s.advance_bounded_wave(w, 400)
        assert np.array_equal(g, s.read_phi()), tt
        s.close()


def test_invalid_waves_are_rejected():
    t, p, x, ex, kind = _table_problem("table_VIII_s1")
    s = lbm.Solver(_bounded(p, kind))
    s.load_phi(ex(x, 0.0))
    good = TABLE_WAVES["table_VIII_s1"]
    bad = [dict(good, shape=0), dict(good, shape=5), dict(good, p=-1.0), dict(good, k=float("nan")),
           dict(good, shape="tanh", p=1.5), dict(good, shape="tanh", p=1.0, r=0.5)]
    for w in bad:
        wv = _wave(dict(w, shape="sech") if w["shape"] in (0, 5) else w, x[0])
        if w["shape"] in (0, 5):
            wv.shape = w["shape"]
        with pytest.raises(lbm.LBMError) as e:
            s.advance_bounded_wave(wv, 10)
        assert e.value.status == lbm.INVALID_ARG, w
    before = s.read_phi()
    assert np.array_equal(before, ex(x, 0.0)) or rel2(before, ex(x, 0.0)) < 1e-15
    s.close()
    periodic = lbm.Solver(W.kdv(0.5, 300, 0.1, 1e-4, 2.0, 0.0))
    with pytest.raises(lbm.LBMError) as e:
        periodic.advance_bounded_wave(_wave(good, 0.0), 10)
    assert e.value.status == lbm.INVALID_ARG
    periodic.close()
