"""Batched relaxation-time sweeps.

The paper picks, for every example, the relaxation time tau that gives the
smallest global relative error E against the exact solution (Sec. IV, tau_opt).
Here that search is one batch: the problem at every candidate tau (each
instance with its own coefficient tables), advanced together in one pass of
the resident kernels, with E computed per tau from the read-out.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

from . import lbm
from .workloads import Problem


def global_relative_error(phi: np.ndarray, exact: np.ndarray) -> float:
    """E = sum |phi - phi*| / sum |phi*| (Sec. IV)."""
    return float(np.sum(np.abs(phi - exact)) / np.sum(np.abs(exact)))


def tau_sweep(problem: Problem, phi0: np.ndarray, steps: int, taus: Sequence[float],
              exact: Optional[np.ndarray] = None, stream: Optional[int] = None,
              phib: Optional[np.ndarray] = None) -> dict:
    """Runs `problem` at every tau in `taus` for `steps` steps in one batch.

    A bounded problem (bc != 0, the setting of the paper's examples) needs
    `phib`, the exact phi at its outer layers after every step, shape
    (steps, 2 layers) -- the same for every tau.

    Returns {"tau": [...], "status": [...], "phi": [...], "E": [...], "tau_opt": t}:
    taus the library rejects (tau <= 1/2, a vanishing tau_k that a term needs)
    get status INVALID_ARG / SINGULAR_TAU and no run; a run that blows up gets
    NONFINITE and E = inf.  E and tau_opt need `exact` (phi* at t = steps dt)."""
    runs, out = [], {"tau": list(taus), "status": [], "phi": [], "E": [], "tau_opt": None}
    for t in taus:
        p = dataclasses.replace(problem, tau=float(t))
        st = lbm.validate(p)
        out["status"].append(st)
        if st == lbm.OK:
            runs.append(p)
    b = lbm.Batch(runs, stream=stream) if runs else None
    if b is not None:
        b.load_phi([phi0] * len(runs))
        if problem.bc:
            if phib is None or len(phib) != steps:
                raise ValueError("a bounded sweep needs phib rows for every step")
            b.advance_bounded([phib] * len(runs))
        else:
            b.advance(int(steps))
    k = 0
    for i, st in enumerate(out["status"]):
        if st != lbm.OK:
            out["phi"].append(None)
            out["E"].append(math.inf)
            continue
        phi, s = b.read_phi(k)
        k += 1
        out["status"][i] = s
        out["phi"].append(phi)
        ok = s == lbm.OK and exact is not None
        out["E"].append(global_relative_error(phi, exact) if ok else math.inf)
    if b is not None:
        b.close()
    if exact is not None and any(math.isfinite(e) for e in out["E"]):
        out["tau_opt"] = out["tau"][int(np.argmin(out["E"]))]
    return out
