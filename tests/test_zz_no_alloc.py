"""lbm_advance_noalloc through the C ABI against the handle path
(lbm_create / lbm_load_phi / lbm_advance / lbm_read_phi) on the same inputs:
bitwise equal, on two calls in a row with the second smaller (the fixed
scratch keeps the first call's contents), in FP64 and FP32 deviation storage
and on both lattices; plus the size limit and the argument checks.
"""
import numpy as np
import pytest

from paper_0907_1720_amd import lbm
from paper_0907_1720_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    t.cuda.set_device(0)
    lbm.library()
    return t


def say(*a):
    print(*a, flush=True)


def _handle(p, phi0, steps):
    s = lbm.Solver(p)
    s.load_phi(phi0)
    s.advance(steps)
    out = s.read_phi()
    s.close()
    return out


def _noalloc(torch, p, phi0, steps):
    a = torch.tensor(phi0, dtype=torch.float64, device="cuda")
    out = torch.full_like(a, float("nan"))
    lbm.advance_noalloc(p, a, steps, out)
    return out.cpu().numpy()


def _kdv(n, prec):
    L = 40.0
    dx = L / n
    p = W.kdv(1.0, n, dx, 0.05 * dx ** 3, 2.0, -20.0, prec=prec)
    return p, W.kdv_soliton(p.grid(), 0.0, 1.2, 1.0, -4.0, period=L)


def _kawahara(n, prec):
    L = 120.0
    dx = L / n
    p = W.kawahara(n, dx, 1.3e-5 * (dx / 0.0586) ** 5, 3.0, -60.0, prec=prec)
    return p, W.kawahara_soliton(p.grid(), 0.0, 7.0, period=L)


@pytest.mark.parametrize("prec", [W.F64, W.F32_DEV])
@pytest.mark.parametrize("make,sizes,steps", [(_kdv, (3000, 777), (900, 301)),
                                              (_kawahara, (2900, 513), (700, 251))])
def test_noalloc_matches_handle_path_twice(torch, prec, make, sizes, steps):
    for n, k in zip(sizes, steps):
        p, phi0 = make(n, prec)
        say("case noalloc", p.name, "n", n, "steps", k, "prec", prec)
        want = _handle(p, phi0, k)
        got = _noalloc(torch, p, phi0, k)
        assert np.array_equal(got, want), float(np.max(np.abs(got - want)))


def test_noalloc_mkdv_and_zero_steps(torch):
    L, n = 40.0, 1500
    dx = L / n
    p = W.mkdv(0.8, n, dx, 0.05 * dx ** 3 / 0.8, 2.0, -20.0, prec=W.F32_DEV)
    phi0 = W.mkdv_soliton(p.grid(), 0.0, 1.0, 0.8, 3.0, period=L)
    say("case noalloc mkdv")
    assert np.array_equal(_noalloc(torch, p, phi0, 1000), _handle(p, phi0, 1000))
    assert np.array_equal(_noalloc(torch, p, phi0, 0), _handle(p, phi0, 0))


def test_noalloc_rejects_beyond_its_limit(torch):
    # 4097 FP64 D1Q5 nodes do not fit one workgroup's LDS; 9000 exceed the scratch
    for n, prec in ((4097, W.F64), (9000, W.F32_DEV)):
        p, phi0 = _kdv(n, prec)
        a = torch.tensor(phi0, dtype=torch.float64, device="cuda")
        with pytest.raises(lbm.LBMError) as e:
            lbm.advance_noalloc(p, a, 10, torch.empty_like(a))
        assert e.value.status == lbm.INVALID_ARG
    # a non-finite phi0 is refused before any device work besides its copy
    p, phi0 = _kdv(600, W.F64)
    phi0[5] = np.nan
    a = torch.tensor(phi0, dtype=torch.float64, device="cuda")
    with pytest.raises(lbm.LBMError) as e:
        lbm.advance_noalloc(p, a, 10, torch.empty_like(a))
    assert e.value.status == lbm.INVALID_ARG
    # and a valid call afterwards is unaffected
    p, phi0 = _kdv(600, W.F64)
    assert np.array_equal(_noalloc(torch, p, phi0, 200), _handle(p, phi0, 200))
