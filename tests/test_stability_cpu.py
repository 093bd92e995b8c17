"""Host-side von Neumann pre-check (lbm_stability) against an independent
eigenvalue computation, and the serving mix against it."""
import dataclasses

import numpy as np
import pytest

from oracle import lbm_oracle as O
from paper_0907_1720_amd import lbm
from paper_0907_1720_amd import workloads as W


def _numpy_growth(p, phis, nk=129):
    """Spectral radius of E(kappa)((1 - w)I + w f_eq'(phi) 1^T) with numpy's eigvals."""
    mdl = O.build_model(dataclasses.replace(p, prec=W.F64))
    om = 1.0 / p.tau
    worst = 0.0
    for pb in phis:
        h = 1e-6 * max(1.0, abs(pb))
        w = (O.equilibrium(mdl, np.array([pb + h])) - O.equilibrium(mdl, np.array([pb - h])))[:, 0] / (2 * h)
        for k in np.linspace(0, np.pi, nk)[1:]:
            A = np.diag(np.exp(-1j * k * mdl.e)) @ ((1 - om) * np.eye(mdl.q) + om * np.outer(w, np.ones(mdl.q)))
            worst = max(worst, np.max(np.abs(np.linalg.eigvals(A))))
    return worst


@pytest.mark.parametrize("p,lo,hi", [
    (W.k22(296, 120 / 296, 0.1 * (120 / 296) ** 3, 2.0, -60.0), 0.0, 1.7),      # unstable grid mode
    (W.k22(296, 120 / 296, 0.1 * (120 / 296) ** 3, 5.0, -60.0), 0.0, 1.7),      # stable
    (W.kdv(1.0, 800, 0.05, 2e-4, 5.0, -20.0), 0.0, 3.0),
    (W.kawahara(500, 0.24, 0.015, 3.0, -60.0), 0.0, 0.63),
    (W.kuramoto_sivashinsky(1024, 32 * np.pi / 1024, 2.9e-4, 2.0, 0.0), -1.3, 1.3),
])
def test_stability_matches_numpy_eigenvalues(p, lo, hi):
    g, amp = lbm.stability(p, lo, hi, 1000)
    want = _numpy_growth(p, np.linspace(lo, hi, 5))
    assert abs(g - want) < 1e-9 * max(1.0, want) + 1e-10
    assert amp == pytest.approx(g ** 1000, rel=1e-12)


def test_serving_mix_is_linearly_stable():
    """Every request of the serving mix (except the physically unstable KS band)
    amplifies by at most 1e3 over its run."""
    for i in range(96):
        r = W.serving_request(i)
        if r.problem.name == "ks":
            continue
        g, amp = lbm.stability(r.problem, float(r.phi0.min()), float(r.phi0.max()), r.steps)
        assert amp <= 1e3, (i, r.problem.name, r.problem.n, r.steps, g)
