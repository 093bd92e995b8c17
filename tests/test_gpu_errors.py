"""Error paths on the GPU, forced from the host so that every kernel still ends
normally: the bounded device waits of the resident chunk queue and of the slab
halo exchange (lbm_batch_test_stall), and requests that the server must refuse
at submission instead of failing at admission.
"""
import numpy as np
import pytest

from paper_0907_1720_amd import lbm
from paper_0907_1720_amd import workloads as W

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


def _kdv(n, prec):
    L = 40.0
    dx = L / n
    p = W.kdv(1.0, n, dx, 0.05 * dx ** 3, 2.0, -20.0, prec=prec)
    return p, W.kdv_soliton(p.grid(), 0.0, 1.0, 1.0, -5.0, period=L)


def _solo(p, phi0, steps, path):
    s = lbm.Solver(p)
    s.set_path(path)
    s.load_phi(phi0)
    s.advance(steps)
    out = s.read_phi()
    s.close()
    return out


@pytest.mark.parametrize("prec", [W.F64, W.F32_DEV])
def test_resident_chunk_wait_gives_up(prec):
    # one job, two chunks, one workgroup: chunk 0 is taken and never run, so the
    # wait of chunk 1 can only end by giving up (after 2 ms)
    p, phi0 = _kdv(512, prec)
    say("case resident stall prec", prec)
    b = lbm.Batch([p])
    b.set_path(lbm.PATH_RESIDENT)
    b.set_resident(0, 2)
    b.load_phi([phi0])
    b.test_stall(1, 2000)
    b.advance(400)
    _, st = b.read_phi(0)
    assert st == lbm.TIMEOUT
    # back to normal: the same batch gives the solo result again
    b.test_stall(0, 0)
    b.load_phi([phi0])
    b.advance(400)
    got, st = b.read_phi(0)
    b.close()
    assert st == lbm.OK
    assert np.array_equal(got, _solo(p, phi0, 400, lbm.PATH_RESIDENT))


@pytest.mark.parametrize("prec", [W.F64, W.F32_DEV])
def test_slab_halo_wait_gives_up(prec):
    # 20000 nodes on the slab path: about ten slabs; slab 0 never raises its
    # flag, so its neighbours give up after 2 ms, then the rest one block later
    p, phi0 = _kdv(20000, prec)
    say("case slab stall prec", prec)
    b = lbm.Batch([p])
    b.set_path(lbm.PATH_SLAB)
    b.load_phi([phi0])
    b.test_stall(2, 2000)
    b.advance(200)
    _, st = b.read_phi(0)
    assert st == lbm.TIMEOUT
    b.test_stall(0, 0)
    b.load_phi([phi0])
    b.advance(200)
    got, st = b.read_phi(0)
    b.close()
    assert st == lbm.OK
    assert np.array_equal(got, _solo(p, phi0, 200, lbm.PATH_SLAB))


def test_test_stall_arguments():
    p, phi0 = _kdv(256, W.F64)
    b = lbm.Batch([p])
    for what, us in ((3, 0), (-1, 0), (1, -5)):
        with pytest.raises(lbm.LBMError) as e:
            b.test_stall(what, us)
        assert e.value.status == lbm.INVALID_ARG
    b.close()


def test_server_refuses_at_submission_what_admission_would_reject():
    # a real-power model (phi^(1/2)) needs phi >= 0: a negative phi0 is refused
    # at submission, and the requests around it complete
    good = [W.serving_request(i, n_max=600, steps_min=200, steps_max=400) for i in range(2)]
    pw = W.power_batch_instance(0, steps=300)
    bad_phi = pw.phi0.copy()
    bad_phi[7] = -0.5
    srv = lbm.Server(1 << 26, max_slots=8, max_n=4096, block_steps=200)
    ids = [srv.submit(good[0].problem, good[0].phi0, good[0].steps)]
    with pytest.raises(lbm.LBMError) as e:
        srv.submit(pw.problem, bad_phi, pw.steps)
    assert e.value.status == lbm.INVALID_ARG
    ids.append(srv.submit(pw.problem, pw.phi0, pw.steps))
    ids.append(srv.submit(good[1].problem, good[1].phi0, good[1].steps))
    got = {}
    for _ in range(1000):
        srv.step()
        for rid in ids:
            if rid not in got:
                r = srv.poll(rid)
                if r is not None:
                    got[rid] = r
        if len(got) == len(ids):
            break
    srv.close()
    assert len(got) == len(ids)
    for (phi, st), inst in zip((got[i] for i in ids), (good[0], pw, good[1])):
        assert st == lbm.OK
        assert np.array_equal(phi, _solo(inst.problem, inst.phi0, inst.steps, lbm.PATH_AUTO))
