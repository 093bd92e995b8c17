"""Seeded synthetic workloads: problem specifications and initial states.

This module only *describes* problems (PDE coefficients, the polynomial
fluxes Pi_k, grid, time step, relaxation time) and draws initial states
phi(x, 0).  It contains none of the lattice Boltzmann arithmetic; both the
HIP library and the CPU oracle consume the same `Problem` objects and the
same phi0 arrays.

PDE class (Sec. II.A, eq. NPDE):

    d_t phi + sum_{k=1..m} alpha_k d_x^k Pi_k(phi) = 0,   alpha_1 = 1.

Every Pi_k is a polynomial in phi, stored as ascending coefficients.

Random numbers come from numpy's PCG64 seeded by
SeedSequence([BASE_SEED, config_id, instance_id]).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 20261203

F64 = 0
F32_DEV = 1           # FP32 deviation storage, FP64 relaxation
F32_DEV_ARITH32 = 2   # FP32 deviation storage, FP32 relaxation


@dataclasses.dataclass
class Problem:
    """One 1D periodic solve.  alpha[k], pi[k] for k = 1..6 (index 0 unused)."""

    alpha: Tuple[float, ...]            # length 7; alpha[1] is 1 by convention
    pi: Tuple[Tuple[float, ...], ...]   # length 7; pi[k] ascending coefficients, () = absent
    n: int                              # number of nodes, periodic
    dx: float
    dt: float
    tau: float
    m: int = 0                          # 0: highest k with alpha_k != 0
    q: int = 0                          # 0: 5 if m <= 4 else 7 (Sec. III)
    scheme: int = 1                     # 1: all q moments; 2: top moment set to zero
    am: int = 0                         # 0: corrected auxiliary moments, 1: as printed
    prec: int = F64
    x0: float = 0.0                     # x_i = x0 + i*dx
    name: str = ""
    bc: int = 0                         # 0 periodic; 1 / 2 bounded: equilibrium / NEE layers
    # non-polynomial Pi_k: gpi[k] = ((exponent, coefficient), ...) replaces pi[k]
    # when non-empty (real powers of phi, Sec. III.C)
    gpi: Tuple[Tuple[Tuple[float, float], ...], ...] = ()

    def has_pi(self, k: int) -> bool:
        return (k < len(self.gpi) and len(self.gpi[k]) > 0) or len(self.pi[k]) > 0

    def order(self) -> int:
        if self.m:
            return self.m
        m = 1
        for k in range(2, 7):
            if self.alpha[k] != 0.0 and self.has_pi(k):
                m = k
        return m

    def lattice(self) -> int:
        if self.q:
            return self.q
        return 5 if self.order() <= 4 else 7

    def grid(self) -> np.ndarray:
        return self.x0 + self.dx * np.arange(self.n, dtype=np.float64)


def _alpha(**kw) -> Tuple[float, ...]:
    a = [0.0] * 7
    a[1] = 1.0
    for k, v in kw.items():
        a[int(k[1:])] = float(v)
    return tuple(a)


def _pis(**kw) -> Tuple[Tuple[float, ...], ...]:
    p = [()] * 7
    for k, v in kw.items():
        p[int(k[1:])] = tuple(float(c) for c in v)
    return tuple(p)


# ---------------------------------------------------------------------------
# equation families
# ---------------------------------------------------------------------------

def kdv(delta: float, n: int, dx: float, dt: float, tau: float, x0: float, **kw) -> Problem:
    """phi_t + phi phi_x + delta phi_xxx = 0: Pi_1 = phi^2/2, Pi_3 = phi."""
    return Problem(_alpha(a3=delta), _pis(p1=(0, 0, 0.5), p3=(0, 1)), n, dx, dt, tau,
                   x0=x0, name="kdv", **kw)


def mkdv(delta: float, n: int, dx: float, dt: float, tau: float, x0: float, **kw) -> Problem:
    """phi_t + phi^2 phi_x + delta phi_xxx = 0: Pi_1 = phi^3/3, Pi_3 = phi."""
    return Problem(_alpha(a3=delta), _pis(p1=(0, 0, 0, 1.0 / 3.0), p3=(0, 1)), n, dx, dt, tau,
                   x0=x0, name="mkdv", **kw)


def kdv_burgers(nu: float, delta: float, n, dx, dt, tau, x0, **kw) -> Problem:
    """phi_t + phi phi_x - nu phi_xx + delta phi_xxx = 0."""
    return Problem(_alpha(a2=-nu, a3=delta), _pis(p1=(0, 0, 0.5), p2=(0, 1), p3=(0, 1)),
                   n, dx, dt, tau, x0=x0, name="kdv_burgers", **kw)


def kuramoto_sivashinsky(n, dx, dt, tau, x0, **kw) -> Problem:
    """phi_t + phi phi_x + phi_xx + phi_xxxx = 0."""
    return Problem(_alpha(a2=1.0, a4=1.0), _pis(p1=(0, 0, 0.5), p2=(0, 1), p4=(0, 1)),
                   n, dx, dt, tau, x0=x0, name="ks", **kw)


def kawahara(n, dx, dt, tau, x0, **kw) -> Problem:
    """phi_t + phi phi_x + phi_xxx - phi_xxxxx = 0 (m = 5, D1Q7)."""
    return Problem(_alpha(a3=1.0, a5=-1.0), _pis(p1=(0, 0, 0.5), p3=(0, 1), p5=(0, 1)),
                   n, dx, dt, tau, x0=x0, name="kawahara", **kw)


def dissipative_fifth_order(nu, delta, mu, eps, n, dx, dt, tau, x0, **kw) -> Problem:
    """phi_t + phi phi_x - nu phi_xx + delta phi_xxx + mu phi_xxxx + eps phi_xxxxx = 0
    (m = 5; with enough diffusion nu it runs stably on D1Q6)."""
    return Problem(_alpha(a2=-nu, a3=delta, a4=mu, a5=eps),
                   _pis(p1=(0, 0, 0.5), p2=(0, 1), p3=(0, 1), p4=(0, 1), p5=(0, 1)),
                   n, dx, dt, tau, x0=x0, name="dissipative5", **kw)


def power_kdv(power, delta, n, dx, dt, tau, x0, nu=0.0, **kw) -> Problem:
    """phi_t + phi^power phi_x - nu phi_xx + delta phi_xxx = 0 with a real power
    >= 0 (Sec. III.C family with beta u^n u_x): Pi_1 = phi^(power+1)/(power+1);
    needs phi >= 0."""
    return Problem(_alpha(a2=-nu, a3=delta), _pis(p2=(0, 1) if nu else (), p3=(0, 1)), n, dx, dt, tau,
                   x0=x0, name="power_kdv",
                   gpi=((), ((power + 1.0, 1.0 / (power + 1.0)),), (), (), (), (), ()), **kw)


def family_b(a, b, npow, a2, p, a3, qpow, n, dx, dt, tau, x0, **kw) -> Problem:
    """phi_t + a phi phi_x + b phi^npow phi_x + a2 (phi^p)_xx + a3 (phi^qpow)_xxx = 0
    (the third-order family of Sec. III.C with real n, p, q; p, q >= 1)."""
    return Problem(_alpha(a2=a2, a3=a3), _pis(), n, dx, dt, tau, x0=x0, name="family_b",
                   gpi=((), ((2.0, a / 2.0), (npow + 1.0, b / (npow + 1.0))), ((p, 1.0),), ((qpow, 1.0),),
                        (), (), ()), **kw)


def family_a(a, b, npow, alphas, n, dx, dt, tau, x0, **kw) -> Problem:
    """phi_t + a phi phi_x + b phi^npow phi_x + sum_k alpha_k d^k phi = 0, k = 2..6
    (the sixth-order family of Sec. III.C with a real n)."""
    al = dict(zip(("a2", "a3", "a4", "a5", "a6"), alphas))
    return Problem(_alpha(**al), _pis(p2=(0, 1), p3=(0, 1), p4=(0, 1), p5=(0, 1), p6=(0, 1)), n, dx, dt, tau,
                   x0=x0, name="family_a",
                   gpi=((), ((2.0, a / 2.0), (npow + 1.0, b / (npow + 1.0))), (), (), (), (), ()), **kw)


def k22(n, dx, dt, tau, x0, **kw) -> Problem:
    """K(2,2): phi_t + (phi^2)_x + (phi^2)_xxx = 0: Pi_1 = Pi_3 = phi^2."""
    return Problem(_alpha(a3=1.0), _pis(p1=(0, 0, 1.0), p3=(0, 0, 1.0)), n, dx, dt, tau,
                   x0=x0, name="k22", **kw)


# ---------------------------------------------------------------------------
# closed-form travelling waves (initial states and exact references)
# ---------------------------------------------------------------------------

def _periodic_images(fn, x, period, images=2):
    out = np.zeros_like(x)
    for k in range(-images, images + 1):
        out += fn(x + k * period)
    return out


def kdv_soliton(x, t, c, delta, xc, period=None):
    """3c sech^2(sqrt(c/delta)/2 (x - c t - xc)): exact for phi_t + phi phi_x + delta phi_xxx = 0."""
    k = 0.5 * math.sqrt(c / delta)
    fn = lambda y: 3.0 * c / np.cosh(k * (y - c * t - xc)) ** 2
    return fn(x) if period is None else _periodic_images(fn, x, period)


def mkdv_soliton(x, t, c, delta, xc, period=None):
    """sqrt(6c) sech(sqrt(c/delta)(x - c t - xc)): exact for phi_t + phi^2 phi_x + delta phi_xxx = 0."""
    k = math.sqrt(c / delta)
    fn = lambda y: math.sqrt(6.0 * c) / np.cosh(k * (y - c * t - xc))
    return fn(x) if period is None else _periodic_images(fn, x, period)


def kawahara_soliton(x, t, xc, period=None):
    """(105/169) sech^4((x - 36t/169 - xc)/(2 sqrt 13)) for phi_t + phi phi_x + phi_xxx - phi_xxxxx = 0."""
    fn = lambda y: (105.0 / 169.0) / np.cosh((y - 36.0 * t / 169.0 - xc) / (2.0 * math.sqrt(13.0))) ** 4
    return fn(x) if period is None else _periodic_images(fn, x, period)


def k22_compacton(x, t, c, xc, period=None):
    """(4c/3) cos^2((x - ct - xc)/4) on |x - ct - xc| <= 2 pi, zero elsewhere (K(2,2))."""
    def fn(y):
        s = y - c * t - xc
        return np.where(np.abs(s) <= 2.0 * math.pi, (4.0 * c / 3.0) * np.cos(s / 4.0) ** 2, 0.0)
    return fn(x) if period is None else _periodic_images(fn, x, period)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def rng(config: int, instance: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, config, instance])))


@dataclasses.dataclass
class Instance:
    problem: Problem
    phi0: np.ndarray
    steps: int
    exact: Optional[object] = None      # callable t -> phi*(x, t) when a closed form exists


def config1(variant: str = "a") -> Instance:
    """Single KdV soliton, delta = 1, periodic [-20, 20), N = 800, c = 1, xc = -5.

    variant a: dt = 2e-4, tau = 5, 10^4 steps (t = 2).
    variant b: dt = 1.25e-5, tau = 2, 1.6e5 steps (t = 2).
    """
    n, L = 800, 40.0
    dx = L / n
    dt, tau, steps = {"a": (2e-4, 5.0, 10000), "b": (1.25e-5, 2.0, 160000)}[variant]
    p = kdv(1.0, n, dx, dt, tau, -20.0)
    x = p.grid()
    phi0 = kdv_soliton(x, 0.0, 1.0, 1.0, -5.0, period=L)
    return Instance(p, phi0, steps, exact=lambda t: kdv_soliton(x, t, 1.0, 1.0, -5.0, period=L))


def config2_instance(i: int, prec: int = F64, steps: int = 5000) -> Instance:
    """Instance i of the 4096-instance KdV/mKdV batch on periodic [-20, 20)."""
    g = rng(2, i)
    is_mkdv = bool(g.random() < 0.5)
    delta = float(g.uniform(0.5, 2.0))
    n = int(round(math.exp(g.uniform(math.log(256.0), math.log(4096.0)))))
    c = float(g.uniform(0.2, 2.0))
    xc = float(g.uniform(-20.0, 20.0))
    L = 40.0
    dx = L / n
    dt = 0.05 * dx ** 3 / delta
    make = mkdv if is_mkdv else kdv
    p = make(delta, n, dx, dt, 2.0, -20.0, prec=prec)
    x = p.grid()
    sol = mkdv_soliton if is_mkdv else kdv_soliton
    phi0 = sol(x, 0.0, c, delta, xc, period=L)
    return Instance(p, phi0, steps, exact=lambda t: sol(x, t, c, delta, xc, period=L))


def config2(count: int = 4096, prec: int = F64, steps: int = 5000) -> List[Instance]:
    return [config2_instance(i, prec, steps) for i in range(count)]


KS_SETTINGS = {1024: (2.0, 2.9e-4), 4096: (10.0, 3.1e-4), 8192: (20.0, 1.7e-4)}


def config3_instance(n: int, i: int, prec: int = F64, t_end: float = 20.0) -> Instance:
    """Kuramoto-Sivashinsky on periodic [0, 32 pi), cos(x/16)(1 + sin(x/16)) + N(0, 1e-3^2)."""
    tau, dt = KS_SETTINGS[n]
    L = 32.0 * math.pi
    dx = L / n
    p = kuramoto_sivashinsky(n, dx, dt, tau, 0.0, prec=prec)
    x = p.grid()
    g = rng(3, n * 100000 + i)
    phi0 = np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0)) + g.normal(0.0, 1e-3, n)
    return Instance(p, phi0, int(round(t_end / dt)))


def config4_instance(i: int, prec: int = F64, steps: int = 5000) -> Instance:
    """Kawahara (D1Q7) or K(2,2) (D1Q5) soliton/compacton on periodic [-60, 60)."""
    g = rng(4, i)
    L = 120.0
    kind = ("kawahara", "k22")[(i // 2) % 2]
    n = (2048, 16384)[i % 2]
    dx = L / n
    if kind == "kawahara":
        xc = float(g.uniform(-60.0, 60.0))
        dt = 1.3e-5 * (dx / 0.0586) ** 5
        p = kawahara(n, dx, dt, 3.0, -60.0, prec=prec)
        x = p.grid()
        phi0 = kawahara_soliton(x, 0.0, xc, period=L)
        ex = lambda t: kawahara_soliton(x, t, xc, period=L)
    else:
        c = float(g.uniform(0.5, 1.5))
        xc = float(g.uniform(-40.0, 40.0))
        dt = 0.1 * dx ** 3
        p = k22(n, dx, dt, 2.0, -60.0, prec=prec)
        x = p.grid()
        phi0 = k22_compacton(x, 0.0, c, xc, period=L)
        ex = lambda t: k22_compacton(x, t, c, xc, period=L)
    return Instance(p, phi0, steps, exact=ex)


def table8_bounded(tau: float = 0.97, prec: int = F64):
    """The bounded KdV-Burgers example of Sec. IV (Table VIII):
    u_t + u u_x - 9e-4 u_xx + 2e-5 u_xxx = 0 on [-4, 4] with both end points,
    dx = dt = 0.01, D1Q5, non-equilibrium extrapolation boundaries, and its
    travelling front 2 xi (1 - 1 / (1 + exp(2 nu (x - xi t)))^2),
    nu = -gamma / (10 delta), xi = 6 gamma^2 / (25 delta).
    Returns (problem, x, exact(x, t))."""
    ga, de = 9e-4, 2e-5
    nu, xi = -ga / (10 * de), 6 * ga ** 2 / (25 * de)

    def exact(x, t):
        return 2 * xi * (1 - 1 / (1 + np.exp(2 * nu * (x - xi * t))) ** 2)

    n = 801
    x = np.linspace(-4.0, 4.0, n)
    p = Problem(_alpha(a2=-ga, a3=de), _pis(p1=(0, 0, 0.5), p2=(0, 1), p3=(0, 1)), n, 0.01, 0.01, tau,
                q=5, prec=prec, x0=-4.0, name="kdv_burgers_table8", bc=2)
    return p, x, exact


def table8_wave() -> dict:
    """Table VIII's front as a travelling wave phi* = a + b h(z)^p with the
    logistic h(z) = 1 / (1 + e^z), z = k (x - xc - c t): a = 2 xi, b = -2 xi,
    p = 2, k = 2 nu, xc = 0, c = xi (the same closed form as table8_bounded)."""
    ga, de = 9e-4, 2e-5
    nu, xi = -ga / (10 * de), 6 * ga ** 2 / (25 * de)
    return dict(shape="logistic", a=2 * xi, b=-2 * xi, p=2.0, k=2 * nu, xc=0.0, c=xi)


def power_batch_instance(i: int, prec: int = F64, steps: int = 2000) -> Instance:
    """Real-power batch: phi_t + phi^n phi_x + delta phi_xxx = 0, n = 0.5 or 1.5
    (Bernoulli 1/2), delta ~ U[0.5, 2], N log-uniform [256, 4096] on [-20, 20),
    dt = 0.05 dx^3 / delta, tau = 2; a Gaussian bump of height ~ U[0.1, 0.4] on
    the background 1 (phi stays positive)."""
    g = rng(7, i)
    power = 0.5 if g.random() < 0.5 else 1.5
    delta = float(g.uniform(0.5, 2.0))
    n = int(round(math.exp(g.uniform(math.log(256), math.log(4096)))))
    dx = 40.0 / n
    p = power_kdv(power, delta, n, dx, 0.05 * dx ** 3 / delta, 2.0, -20.0, prec=prec)
    x = p.grid()
    xc, h = float(g.uniform(-15.0, 15.0)), float(g.uniform(0.1, 0.4))
    phi0 = 1.0 + h * np.exp(-((x - xc) / 2.0) ** 2)
    return Instance(p, np.ascontiguousarray(phi0), steps)


def even_lattice_instance(i: int, q: int, prec: int = F64, steps: int = 2000) -> Instance:
    """Batch on the lattices without rest velocity: D1Q4 KdV-Burgers (nu = 3,
    delta = 0.1) or D1Q6 phi_t + phi phi_x - 3 phi_xx + 1e-3 phi_xxx +
    0.0625 phi_xxxx - 1e-3 phi_xxxxx = 0, dx = 0.1, dt = 0.01, tau = 2 (the
    diffusion keeps the checkerboard mode damped); N log-uniform [256, 4096];
    a smooth random periodic state."""
    g = rng(8 + q, i)
    n = int(round(math.exp(g.uniform(math.log(256), math.log(4096)))))
    if q == 4:
        p = kdv_burgers(3.0, 0.1, n, 0.1, 0.01, 2.0, 0.0, q=4, prec=prec)
    else:
        p = dissipative_fifth_order(3.0, 1e-3, 0.0625, -1e-3, n, 0.1, 0.01, 2.0, 0.0, q=6, prec=prec)
    x = np.arange(n) / n
    phi0 = 0.5 + 0.3 * np.sin(2 * np.pi * x + float(g.uniform(0, 6))) + 0.1 * np.cos(6 * np.pi * x)
    return Instance(p, phi0, steps)


def random_m6_problem(g: np.random.Generator, n: int) -> Problem:
    """Random sixth-order equation: alpha_k ~ U[-1, 1] with alpha_6 := -|alpha_6| (a
    dissipative top order), Pi_k random cubics without constant term, dx = 0.1,
    tau = 1.5 and dt = 0.05 min_k dx^k / |alpha_k|."""
    a = [0.0, 1.0] + [float(g.uniform(-1.0, 1.0)) for _ in range(5)]
    a[6] = -abs(a[6])
    pis = [()] + [(0.0,) + tuple(float(v) for v in g.uniform(-1.0, 1.0, 3)) for _ in range(6)]
    dx = 0.1
    dt = 0.05 * min(dx ** k / abs(a[k]) for k in range(2, 7) if a[k] != 0.0)
    return Problem(tuple(a), tuple(pis), n, dx, dt, 1.5, x0=0.0, name="random_m6")


# ---------------------------------------------------------------------------
# serving mix: one request = (problem, phi0, steps)
# ---------------------------------------------------------------------------

SERVING_FAMILIES = ("kdv", "mkdv", "kdv_burgers", "k22", "ks", "kawahara", "random_m6")
KS_TAU_RULE = ((2048, 2.0), (4096, 10.0), (1 << 40, 20.0))
# KS time step dt = C(tau) dx^4; the constants reproduce the (tau, dt) settings
# of the Kuramoto-Sivashinsky batch (2, 2.9e-4) at N = 1024, (10, 3.1e-4) at
# N = 4096 and (20, 1.7e-4) at N = 8192 on [0, 32 pi)
KS_DT_CONST = {2.0: 3.125, 10.0: 855.7916666666666, 20.0: 7411.625}


def serving_request(i: int, n_min: int = 128, n_max: int = 16384, steps_min: int = 1000,
                    steps_max: int = 100000) -> Instance:
    """Request i of the serving mix: a uniformly drawn family, N and steps
    log-uniform, precision FP32 deviation or FP64 with probability 1/2; Kawahara
    requests use scheme 2 and random sixth-order ones the printed auxiliary
    moments with probability 1/2."""
    g = rng(5, i)
    fam = SERVING_FAMILIES[int(g.integers(len(SERVING_FAMILIES)))]
    n = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
    steps = int(round(math.exp(g.uniform(math.log(steps_min), math.log(steps_max)))))
    prec = F32_DEV if g.random() < 0.5 else F64
    if fam in ("kdv", "mkdv", "kdv_burgers"):
        L = 40.0
        dx = L / n
        delta = float(g.uniform(0.5, 2.0))
        c = float(g.uniform(0.2, 2.0))
        xc = float(g.uniform(-20.0, 20.0))
        dt = 0.05 * dx ** 3 / delta
        if fam == "kdv":
            p = kdv(delta, n, dx, dt, 2.0, -20.0, prec=prec)
            phi0 = kdv_soliton(p.grid(), 0.0, c, delta, xc, period=L)
        elif fam == "mkdv":
            p = mkdv(delta, n, dx, dt, 2.0, -20.0, prec=prec)
            phi0 = mkdv_soliton(p.grid(), 0.0, c, delta, xc, period=L)
        else:
            nu = float(g.uniform(0.01, 0.1))
            p = kdv_burgers(nu, delta, n, dx, dt, 2.0, -20.0, prec=prec)
            phi0 = kdv_soliton(p.grid(), 0.0, c, delta, xc, period=L)
    elif fam == "ks":
        # coarser grids do not resolve the KS length scales on [0, 32 pi) (and the
        # time-step rule is unstable there): at least 1024 nodes
        n = max(n, 1024)
        L = 32.0 * math.pi
        dx = L / n
        tau = next(t for lim, t in KS_TAU_RULE if n <= lim)
        p = kuramoto_sivashinsky(n, dx, KS_DT_CONST[tau] * dx ** 4, tau, 0.0, prec=prec)
        x = p.grid()
        phi0 = np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0)) + g.normal(0.0, 1e-3, n)
    elif fam in ("kawahara", "k22"):
        L = 120.0
        dx = L / n
        if fam == "kawahara":
            # the dx^5 rule of the Kawahara batch, capped at a lattice speed c >= 10;
            # below 2048 nodes tau = 8 (at tau = 3 the grid-scale mode of coarse
            # grids grows up to ~0.6% per step)
            p = kawahara(n, dx, min(1.3e-5 * (dx / 0.0586) ** 5, 0.1 * dx), 3.0 if n >= 2048 else 8.0, -60.0,
                         prec=prec)
            phi0 = kawahara_soliton(p.grid(), 0.0, float(g.uniform(-60.0, 60.0)), period=L)
            # scheme 2 (top moment zero, the variant of Sec. IV's Kawahara-type
            # examples) for half of the requests
            if g.random() < 0.5:
                p = dataclasses.replace(p, scheme=2)
        else:
            # tau = 5: at the batch's tau = 2 the grid-scale mode grows 0.015% per
            # step on fine grids and up to 0.5% on coarse ones (von Neumann), too much
            # for runs of up to 1e5 steps
            p = k22(n, dx, 0.1 * dx ** 3, 5.0, -60.0, prec=prec)
            phi0 = k22_compacton(p.grid(), 0.0, float(g.uniform(0.5, 1.5)), float(g.uniform(-40.0, 40.0)),
                                 period=L)
    else:
        # tau = 3: at tau = 1.5 the grid-scale mode grows ~0.1-0.6% per step
        p = random_m6_problem(g, n)
        p = dataclasses.replace(p, prec=prec, tau=3.0)
        x = p.grid() / (n * p.dx)
        phi0 = 0.3 * np.sin(2 * np.pi * x) + 0.1 * np.cos(6 * np.pi * x + float(g.uniform(0, 6)))
        # the auxiliary moments as printed (instead of corrected) for half of them
        if g.random() < 0.5:
            p = dataclasses.replace(p, am=1)
    return Instance(p, np.ascontiguousarray(phi0, dtype=np.float64), steps)
