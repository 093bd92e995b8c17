"""ctypes binding of liblbmhpde.so (include/lbmhpde.h).

Argument marshalling only: every step of the time step runs in the HIP
kernels of the library.  PyTorch, when present, supplies device memory and
the current stream.  There is no CPU fallback: if the library has not been
built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

from .workloads import Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmhpde.so")

OK, INVALID_ARG, UNSUPPORTED, SINGULAR_TAU, OUT_OF_MEMORY, DEVICE, NONFINITE, BUSY, TIMEOUT = range(9)
PATH_AUTO, PATH_STREAM, PATH_RESIDENT, PATH_TILED, PATH_SLAB = 0, 1, 2, 3, 4
BC_PERIODIC, BC_DIRICHLET_EQ, BC_DIRICHLET_NEE = 0, 1, 2


class LbmDesc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("am", ctypes.c_int32),
        ("alpha", ctypes.c_double * 7),
        ("pi_deg", ctypes.c_int32 * 7),
        ("pi_coef", (ctypes.c_double * 5) * 7),
        ("n", ctypes.c_int64),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("bc", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("pi_terms", ctypes.c_int32 * 7),
        ("pi_pad_", ctypes.c_int32),
        ("pi_gexp", (ctypes.c_double * 4) * 7),
        ("pi_gcoef", (ctypes.c_double * 4) * 7),
    ]


WAVE_SECH, WAVE_TANH, WAVE_LOGISTIC, WAVE_COS = 1, 2, 3, 4


class LbmWave(ctypes.Structure):
    """phi*(x, t) = a + b h(z)^p + d h(z)^r, z = k (x - xc - c t)
    (include/lbmhpde.h, lbm_wave)."""
    _fields_ = [
        ("shape", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("a", ctypes.c_double),
        ("b", ctypes.c_double),
        ("p", ctypes.c_double),
        ("d", ctypes.c_double),
        ("r", ctypes.c_double),
        ("k", ctypes.c_double),
        ("xc", ctypes.c_double),
        ("c", ctypes.c_double),
        ("x_first", ctypes.c_double),
        ("t0", ctypes.c_double),
    ]


WAVE_SHAPES = {"sech": WAVE_SECH, "tanh": WAVE_TANH, "logistic": WAVE_LOGISTIC, "cos": WAVE_COS}


def make_wave(shape, a: float, b: float, p: float, k: float, xc: float, c: float, x_first: float,
              t0: float = 0.0, d: float = 0.0, r: float = 0.0) -> LbmWave:
    """An LbmWave; `shape` is an lbm_wave_shape value or its name ("sech", "tanh",
    "logistic", "cos")."""
    code = WAVE_SHAPES[shape] if isinstance(shape, str) else int(shape)
    return LbmWave(code, 0, float(a), float(b), float(p), float(d), float(r), float(k), float(xc), float(c),
                   float(x_first), float(t0))


class LbmTuning(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int32),
        ("tile_steps", ctypes.c_int32),
        ("tile_wgs", ctypes.c_int32),
        ("res_chunks", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("best_node_updates_per_s", ctypes.c_double),
        ("default_node_updates_per_s", ctypes.c_double),
    ]


class LBMError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


_lib = None


def library() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -m paper_0907_1720_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    DP = ctypes.POINTER(LbmDesc)
    sig = {
        "lbm_status_str": (ctypes.c_char_p, [I32]),
        "lbm_version": (ctypes.c_char_p, []),
        "lbm_row_stride": (I64, [I64]),
        "lbm_validate": (I32, [DP]),
        "lbm_coefficients": (I32, [DP, P, I32, P, P]),
        "lbm_coefficients_general": (I32, [DP, P, P, I32, P, P, P]),
        "lbm_required_bytes": (I32, [DP, P]),
        "lbm_stability": (I32, [DP, D, D, I64, P, P]),
        "lbm_create": (I32, [DP, P, P, SZ, P]),
        "lbm_load_phi": (I32, [P, P, I32]),
        "lbm_advance": (I32, [P, I64]),
        "lbm_advance_noalloc": (I32, [DP, P, I64, P, P]),
        "lbm_advance_bounded": (I32, [P, I64, P, I32]),
        "lbm_advance_bounded_wave": (I32, [P, I64, P, I32]),
        "lbm_wave_rows": (I32, [P, I64, P, I32, P]),
        "lbm_read_phi": (I32, [P, P, I32]),
        "lbm_sum_phi": (I32, [P, P]),
        "lbm_state_bytes": (I32, [P, P]),
        "lbm_save_f": (I32, [P, P, SZ]),
        "lbm_load_f": (I32, [P, P, SZ]),
        "lbm_set_path": (I32, [P, I32]),
        "lbm_set_tiling": (I32, [P, I32, I32]),
        "lbm_last_advance_ms": (I32, [P, P]),
        "lbm_destroy": (I32, [P]),
        "lbm_batch_create": (I32, [DP, I32, P, P]),
        "lbm_batch_load_phi": (I32, [P, P]),
        "lbm_batch_advance": (I32, [P, P]),
        "lbm_batch_advance_bounded": (I32, [P, I64, P, I32]),
        "lbm_batch_advance_bounded_wave": (I32, [P, I64, P, I32]),
        "lbm_batch_read_phi": (I32, [P, I32, P, P]),
        "lbm_batch_last_advance_ms": (I32, [P, P]),
        "lbm_batch_set_path": (I32, [P, I32]),
        "lbm_batch_set_tiling": (I32, [P, I32, I32]),
        "lbm_batch_set_resident": (I32, [P, I32, I32]),
        "lbm_batch_set_lanes": (I32, [P, I32]),
        "lbm_batch_autotune": (I32, [P, I64, P]),
        "lbm_batch_test_stall": (I32, [P, I32, I64]),
        "lbm_batch_destroy": (I32, [P]),
        "lbm_server_create": (I32, [P, SZ, I32, I64, I32, P]),
        "lbm_server_submit": (I32, [P, DP, P, I64, P]),
        "lbm_server_step": (I32, [P, P, P, P]),
        "lbm_server_poll": (I32, [P, I64, P, I64, P]),
        "lbm_server_pump": (I32, [P, P, P, P, P]),
        "lbm_server_timing": (I32, [P, I64, P, P]),
        "lbm_server_stats": (I32, [P, P, P, P]),
        "lbm_server_destroy": (I32, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_str(s: int) -> str:
    try:
        return library().lbm_status_str(int(s)).decode()
    except ImportError:
        return "status"


def _check(status: int, what: str):
    if status != OK:
        raise LBMError(status, what)


def make_desc(p: Problem) -> LbmDesc:
    d = LbmDesc()
    d.m = int(p.m)
    d.q = int(p.q)
    d.scheme = int(p.scheme)
    d.am = int(p.am)
    for k in range(7):
        d.alpha[k] = float(p.alpha[k]) if k < len(p.alpha) else 0.0
        coeffs = p.pi[k] if k < len(p.pi) else ()
        if k == 0 or len(coeffs) == 0:
            d.pi_deg[k] = -1
        else:
            if len(coeffs) > 5:
                raise ValueError("Pi_k of degree > 4")
            d.pi_deg[k] = len(coeffs) - 1
            for i, c in enumerate(coeffs):
                d.pi_coef[k][i] = float(c)
    gpi = getattr(p, "gpi", ())
    for k in range(1, 7):
        terms = gpi[k] if k < len(gpi) else ()
        if len(terms) == 0:
            continue
        if len(terms) > 4:
            raise ValueError("at most 4 terms per non-polynomial Pi_k")
        d.pi_terms[k] = len(terms)
        for i, (e, c) in enumerate(terms):
            d.pi_gexp[k][i] = float(e)
            d.pi_gcoef[k][i] = float(c)
    d.n = int(p.n)
    d.dx, d.dt, d.tau = float(p.dx), float(p.dt), float(p.tau)
    d.bc = int(getattr(p, "bc", 0))
    d.prec = int(p.prec)
    return d


def validate(p: Problem) -> int:
    return library().lbm_validate(ctypes.byref(make_desc(p)))


def coefficients(p: Problem) -> np.ndarray:
    """Host-built equilibrium polynomials G, shape (q, D + 1): f_eq_j = sum_d G[j, d] phi^d."""
    buf = np.zeros(7 * 20, dtype=np.float64)
    q, D = ctypes.c_int32(), ctypes.c_int32()
    _check(library().lbm_coefficients(ctypes.byref(make_desc(p)), buf.ctypes.data, buf.size,
                                      ctypes.byref(q), ctypes.byref(D)), "lbm_coefficients")
    return buf[: q.value * (D.value + 1)].reshape(q.value, D.value + 1).copy()


def coefficients_general(p: Problem):
    """(nu, G) with f_eq_j(phi) = sum_c phi^nu[c] sum_d G[c, j, d] phi^d (every model)."""
    nu = np.zeros(4, dtype=np.float64)
    buf = np.zeros(4 * 7 * 20, dtype=np.float64)
    F, q, D = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(library().lbm_coefficients_general(ctypes.byref(make_desc(p)), nu.ctypes.data, buf.ctypes.data, buf.size,
                                              ctypes.byref(F), ctypes.byref(q), ctypes.byref(D)),
           "lbm_coefficients_general")
    n = F.value * q.value * (D.value + 1)
    return nu[: F.value].copy(), buf[:n].reshape(F.value, q.value, D.value + 1).copy()


def stability(p: Problem, phi_min: float, phi_max: float, steps: int):
    """(growth per step, amplification over `steps`) of the linearised scheme."""
    g, a = ctypes.c_double(), ctypes.c_double()
    _check(library().lbm_stability(ctypes.byref(make_desc(p)), float(phi_min), float(phi_max), int(steps),
                                   ctypes.byref(g), ctypes.byref(a)), "lbm_stability")
    return g.value, a.value


def advance_noalloc(p: Problem, phi0, steps: int, phi, stream: Optional[int] = None, allow_nonfinite: bool = False):
    """lbm_advance_noalloc: phi := phi after `steps` steps from phi0 (device
    tensors of p.n doubles, e.g. torch CUDA tensors), allocating nothing."""
    for t in (phi0, phi):
        if not (hasattr(t, "data_ptr") and getattr(t, "is_cuda", False)):
            raise ValueError("phi0 and phi must be device tensors")
        if t.numel() != p.n or t.element_size() != 8:
            raise ValueError(f"expected {p.n} doubles")
    d = make_desc(p)
    st = _current_stream() if stream is None else int(stream)
    s = library().lbm_advance_noalloc(ctypes.byref(d), int(phi0.data_ptr()), int(steps), int(phi.data_ptr()), st)
    if not (allow_nonfinite and s == NONFINITE):
        _check(s, "lbm_advance_noalloc")
    return s


def _current_stream() -> int:
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


class Solver:
    """One periodic problem on the GPU (lbm_create ... lbm_destroy)."""

    def __init__(self, p: Problem, stream: Optional[int] = None, dev_buf=None):
        lib = library()
        self.problem = p
        self._desc = make_desc(p)
        self.stream = _current_stream() if stream is None else int(stream)
        h = ctypes.c_void_p()
        buf_ptr, buf_bytes = None, 0
        if dev_buf is not None:   # e.g. a torch CUDA tensor that outlives the solver
            buf_ptr, buf_bytes = int(dev_buf.data_ptr()), int(dev_buf.numel() * dev_buf.element_size())
            self._keep = dev_buf
        _check(lib.lbm_create(ctypes.byref(self._desc), self.stream, buf_ptr, buf_bytes, ctypes.byref(h)),
               "lbm_create")
        self._h = h

    @staticmethod
    def required_bytes(p: Problem) -> int:
        n = ctypes.c_size_t()
        _check(library().lbm_required_bytes(ctypes.byref(make_desc(p)), ctypes.byref(n)), "lbm_required_bytes")
        return n.value

    def load_phi(self, phi):
        if hasattr(phi, "data_ptr") and getattr(phi, "is_cuda", False):
            _check(library().lbm_load_phi(self._h, int(phi.data_ptr()), 1), "lbm_load_phi")
        else:
            a = np.ascontiguousarray(phi, dtype=np.float64)
            assert a.size == self.problem.n
            _check(library().lbm_load_phi(self._h, a.ctypes.data, 0), "lbm_load_phi")

    def advance(self, steps: int):
        _check(library().lbm_advance(self._h, int(steps)), "lbm_advance")

    def advance_bounded(self, phib, layers: int = 0):
        """Bounded problem: len(phib) steps; phib[s] = exact phi at the outer
        `layers` nodes of each end (left then right) after step s + 1."""
        a = np.ascontiguousarray(phib, dtype=np.float64)
        steps = a.shape[0] if a.ndim == 2 else 0
        if a.ndim != 2 or (steps and a.shape[1] % 2):
            raise ValueError("phib must be (steps, 2 * layers)")
        lay = a.shape[1] // 2 if steps else int(layers)
        if layers and steps and lay != layers:
            raise ValueError("phib width is not 2 * layers")
        _check(library().lbm_advance_bounded(self._h, steps, a.ctypes.data, lay), "lbm_advance_bounded")

    def advance_bounded_wave(self, wave: LbmWave, steps: int, layers: int = 0):
        """Bounded problem: `steps` steps with the outer layers reset from the
        travelling wave `wave`, evaluated on the device."""
        _check(library().lbm_advance_bounded_wave(self._h, int(steps), ctypes.byref(wave), int(layers)),
               "lbm_advance_bounded_wave")

    def wave_rows(self, wave: LbmWave, steps: int, layers: int = 0) -> np.ndarray:
        """The (steps, 2 layers) boundary rows advance_bounded_wave would use."""
        lay = int(layers) if layers else self.problem.lattice() // 2
        out = np.empty((int(steps), 2 * lay), dtype=np.float64)
        _check(library().lbm_wave_rows(self._h, int(steps), ctypes.byref(wave), lay, out.ctypes.data),
               "lbm_wave_rows")
        return out

    def read_phi(self, out=None, allow_nonfinite: bool = False) -> np.ndarray:
        if out is not None and hasattr(out, "data_ptr"):
            s = library().lbm_read_phi(self._h, int(out.data_ptr()), 1)
            res = out
        else:
            res = np.empty(self.problem.n, dtype=np.float64)
            s = library().lbm_read_phi(self._h, res.ctypes.data, 0)
        if not (allow_nonfinite and s == NONFINITE):
            _check(s, "lbm_read_phi")
        return res

    def sum_phi(self) -> float:
        t = ctypes.c_double()
        _check(library().lbm_sum_phi(self._h, ctypes.byref(t)), "lbm_sum_phi")
        return t.value

    def save(self) -> bytes:
        n = ctypes.c_size_t()
        _check(library().lbm_state_bytes(self._h, ctypes.byref(n)), "lbm_state_bytes")
        buf = ctypes.create_string_buffer(n.value)
        _check(library().lbm_save_f(self._h, buf, n.value), "lbm_save_f")
        return buf.raw

    def load(self, blob: bytes):
        _check(library().lbm_load_f(self._h, blob, len(blob)), "lbm_load_f")

    def set_path(self, path: int):
        _check(library().lbm_set_path(self._h, int(path)), "lbm_set_path")

    def set_tiling(self, steps_per_launch: int = 0, wgs_per_cu: int = 0):
        _check(library().lbm_set_tiling(self._h, int(steps_per_launch), int(wgs_per_cu)), "lbm_set_tiling")

    def last_advance_ms(self) -> float:
        ms = ctypes.c_float()
        _check(library().lbm_last_advance_ms(self._h, ctypes.byref(ms)), "lbm_last_advance_ms")
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            library().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems advanced together (lbm_batch_*)."""

    def __init__(self, problems: Sequence[Problem], stream: Optional[int] = None):
        lib = library()
        self.problems = list(problems)
        arr = (LbmDesc * len(self.problems))(*[make_desc(p) for p in self.problems])
        self._descs = arr
        self.stream = _current_stream() if stream is None else int(stream)
        h = ctypes.c_void_p()
        _check(lib.lbm_batch_create(arr, len(self.problems), self.stream, ctypes.byref(h)), "lbm_batch_create")
        self._h = h

    def load_phi(self, phis: Sequence[np.ndarray]):
        if len(phis) != len(self.problems):
            raise ValueError(f"{len(phis)} initial states for {len(self.problems)} instances")
        keep = [np.ascontiguousarray(p, dtype=np.float64) for p in phis]
        for a, p in zip(keep, self.problems):
            if a.size != p.n:
                raise ValueError(f"initial state of {a.size} values for {p.n} nodes")
        ptrs = (ctypes.c_void_p * len(keep))(*[a.ctypes.data for a in keep])
        _check(library().lbm_batch_load_phi(self._h, ptrs), "lbm_batch_load_phi")

    def advance(self, steps):
        if np.isscalar(steps):
            steps = [int(steps)] * len(self.problems)
        s = np.ascontiguousarray(steps, dtype=np.int64)
        assert s.size == len(self.problems)
        _check(library().lbm_batch_advance(self._h, s.ctypes.data), "lbm_batch_advance")

    def advance_bounded(self, phibs, layers: int = 0):
        """Every instance advances len(rows) steps; bounded instance i resets its
        outer layers after step s from phibs[i][s] (left layers, then right);
        phibs[i] is None for periodic instances."""
        if len(phibs) != len(self.problems):
            raise ValueError(f"{len(phibs)} boundary row sets for {len(self.problems)} instances")
        arrs, steps = [], None
        for i, a in enumerate(phibs):
            if a is None:
                arrs.append(None)
                continue
            a = np.ascontiguousarray(a, dtype=np.float64)
            if a.ndim != 2 or a.shape[1] % 2:
                raise ValueError("phib rows must be (steps, 2 * layers)")
            if steps is not None and a.shape[0] != steps:
                raise ValueError("every bounded instance needs the same number of rows")
            steps = a.shape[0]
            if layers and a.shape[1] != 2 * layers:
                raise ValueError("phib width is not 2 * layers")
            layers = a.shape[1] // 2
            arrs.append(a)
        if steps is None:
            raise ValueError("no bounded instance")
        ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data if a is not None else None for a in arrs])
        _check(library().lbm_batch_advance_bounded(self._h, int(steps), ctypes.cast(ptrs, ctypes.c_void_p), int(layers)),
               "lbm_batch_advance_bounded")

    def advance_bounded_wave(self, waves, steps: int, layers: int = 0):
        """Every instance advances `steps` steps; bounded instance i resets its
        outer layers from waves[i] (an LbmWave evaluated on the device; None
        for periodic instances)."""
        if len(waves) != len(self.problems):
            raise ValueError(f"{len(waves)} waves for {len(self.problems)} instances")
        arr = (LbmWave * len(waves))()
        for i, w in enumerate(waves):
            if w is not None:
                arr[i] = w
        _check(library().lbm_batch_advance_bounded_wave(self._h, int(steps), ctypes.cast(arr, ctypes.c_void_p),
                                                        int(layers)), "lbm_batch_advance_bounded_wave")

    def read_phi(self, i: int):
        """(phi, status) of instance i; status is OK, NONFINITE or TIMEOUT for that instance."""
        out = np.empty(self.problems[i].n, dtype=np.float64)
        st = ctypes.c_int32()
        _check(library().lbm_batch_read_phi(self._h, int(i), out.ctypes.data, ctypes.byref(st)),
               "lbm_batch_read_phi")
        return out, st.value

    def set_path(self, path: int):
        _check(library().lbm_batch_set_path(self._h, int(path)), "lbm_batch_set_path")

    def set_tiling(self, steps_per_launch: int = 0, wgs_per_cu: int = 0):
        _check(library().lbm_batch_set_tiling(self._h, int(steps_per_launch), int(wgs_per_cu)),
               "lbm_batch_set_tiling")

    def set_resident(self, max_workgroups: int = 0, chunks: int = 0):
        _check(library().lbm_batch_set_resident(self._h, int(max_workgroups), int(chunks)),
               "lbm_batch_set_resident")

    def set_lanes(self, lanes: int = 0):
        """Streams one advance spreads its launches over (0 = one per hardware queue, at most 16)."""
        _check(library().lbm_batch_set_lanes(self._h, int(lanes)), "lbm_batch_set_lanes")

    def test_stall(self, what: int, wait_us: int = 0):
        """Forces a bounded device wait to give up (test hook; 0, 0 restores)."""
        _check(library().lbm_batch_test_stall(self._h, int(what), int(wait_us)), "lbm_batch_test_stall")

    def autotune(self, probe_steps: int) -> dict:
        """Times planner settings on a copy of the batch and keeps the fastest."""
        t = LbmTuning()
        _check(library().lbm_batch_autotune(self._h, int(probe_steps), ctypes.byref(t)), "lbm_batch_autotune")
        return {k: getattr(t, k) for k, _ in LbmTuning._fields_ if k != "pad_"}

    def apply_tuning(self, t: dict):
        """Sets the planner settings of an earlier autotune result."""
        self.set_path(t["path"])
        self.set_tiling(t["tile_steps"], t["tile_wgs"])
        self.set_resident(0, t["res_chunks"])

    def last_advance_ms(self) -> float:
        ms = ctypes.c_float()
        _check(library().lbm_batch_last_advance_ms(self._h, ctypes.byref(ms)), "lbm_batch_last_advance_ms")
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            library().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching of solve requests (lbm_server_*)."""

    def __init__(self, budget_bytes: int, max_slots: int = 4096, max_n: int = 16384,
                 block_steps: int = 1000, stream: Optional[int] = None):
        self.stream = _current_stream() if stream is None else int(stream)
        h = ctypes.c_void_p()
        _check(library().lbm_server_create(self.stream, int(budget_bytes), int(max_slots), int(max_n),
                                           int(block_steps), ctypes.byref(h)), "lbm_server_create")
        self._h = h
        self._n = {}

    def submit(self, p: Problem, phi0, steps: int) -> int:
        a = np.ascontiguousarray(phi0, dtype=np.float64)
        assert a.size == p.n
        d = make_desc(p)
        rid = ctypes.c_int64()
        _check(library().lbm_server_submit(self._h, ctypes.byref(d), a.ctypes.data, int(steps), ctypes.byref(rid)),
               "lbm_server_submit")
        self._n[rid.value] = p.n
        return rid.value

    def step(self):
        """One scheduling round; returns (active, queued, retired)."""
        a, q, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(library().lbm_server_step(self._h, ctypes.byref(a), ctypes.byref(q), ctypes.byref(r)),
               "lbm_server_step")
        return a.value, q.value, r.value

    def pump(self):
        """Non-blocking round management; returns (running, active, queued, retired)."""
        r, a, q, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(library().lbm_server_pump(self._h, ctypes.byref(r), ctypes.byref(a), ctypes.byref(q),
                                         ctypes.byref(t)), "lbm_server_pump")
        return r.value, a.value, q.value, t.value

    def timing(self, rid: int):
        """(queue seconds, service seconds) of a retired request, else None."""
        qs, ss = ctypes.c_double(), ctypes.c_double()
        s = library().lbm_server_timing(self._h, int(rid), ctypes.byref(qs), ctypes.byref(ss))
        if s == BUSY:
            return None
        _check(s, "lbm_server_timing")
        return qs.value, ss.value

    def poll(self, rid: int):
        """(phi, status) once request rid has finished, else None."""
        n = self._n[rid]
        out = np.empty(n, dtype=np.float64)
        st = ctypes.c_int32()
        s = library().lbm_server_poll(self._h, int(rid), out.ctypes.data, n, ctypes.byref(st))
        if s == BUSY:
            return None
        _check(s, "lbm_server_poll")
        return out, st.value

    def stats(self):
        nu, ms, free = ctypes.c_double(), ctypes.c_double(), ctypes.c_size_t()
        _check(library().lbm_server_stats(self._h, ctypes.byref(nu), ctypes.byref(ms), ctypes.byref(free)),
               "lbm_server_stats")
        return nu.value, ms.value, free.value

    def close(self):
        if getattr(self, "_h", None):
            library().lbm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
