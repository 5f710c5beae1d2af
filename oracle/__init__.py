"""Python binding of the CPU oracle (plain serial FP64 C, ``at_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2204_01133_amd``) never imports it and shares no code with it; the
two meet only in the seeded workloads of ``at_workloads``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "at_oracle.c")
_HDR = os.path.join(_HERE, "at_oracle.h")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None

PDE_IDS = {"adv_diff": 0, "adr_logistic": 1, "burgers": 2, "euler": 3, "reactive_euler": 4,
           "reactive_ns": 5}
SCHEME_IDS = {"fd2": 0, "fd4": 1, "fd8": 2, "weno5": 3, "weno5i": 4}
MODE_IDS = {"sync": 0, "as": 1, "at": 2}
FORM_IDS = {"flux": 0, "chain": 1}
RK_IDS = {"fe": 0, "rk2": 1, "ssprk3": 2, "rk4": 3}
GRAN_IDS = {"per_pe": 0, "per_pe_side": 1, "per_boundary": 2}
BC_IDS = {"periodic": 0, "nscbc": 1}

ERRORS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "stale: delay beyond kmax",
          -4: "out of range"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')}) {what}")
        self.code = code


class OrcProblem(ctypes.Structure):
    _fields_ = [
        ("pde", ctypes.c_int32), ("scheme", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("rk", ctypes.c_int32), ("granularity", ctypes.c_int32), ("kmax", ctypes.c_int32),
        ("n", ctypes.c_int64), ("p", ctypes.c_int32), ("n_cdf", ctypes.c_int32),
        ("at_levels", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("form", ctypes.c_int32), ("pad_form", ctypes.c_int32),
        ("cdf", ctypes.c_uint64 * 16),
        ("x0", ctypes.c_double), ("lx", ctypes.c_double), ("dt", ctypes.c_double),
        ("c", ctypes.c_double), ("alpha", ctypes.c_double), ("r", ctypes.c_double),
        ("gamma", ctypes.c_double), ("q", ctypes.c_double), ("ea", ctypes.c_double),
        ("b", ctypes.c_double), ("mu", ctypes.c_double), ("pr", ctypes.c_double),
        ("le", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("problem_id", ctypes.c_int64),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (serial, FP64, no floating-point contraction)."""
    with _lock:
        if not force and os.path.exists(_LIB_PATH) and \
                os.path.getmtime(_LIB_PATH) >= max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
            return _LIB_PATH
        os.makedirs(_BUILD, exist_ok=True)
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
        return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        _lib = load(build())
    return _lib


def load(path: str):
    """Load an oracle library built from at_oracle.c (the tests also load copies of
    it with a planted mistake, to show that a pin catches that mistake)."""
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.orc_create.argtypes = [P(OrcProblem), P(ctypes.c_double), P(ctypes.c_void_p)]
    L.orc_free.argtypes = [ctypes.c_void_p]
    L.orc_free.restype = None
    L.orc_set_history.argtypes = [ctypes.c_void_p, ctypes.c_int, P(ctypes.c_double), ctypes.c_int64]
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_current_step.argtypes = [ctypes.c_void_p]
    L.orc_current_step.restype = ctypes.c_int64
    L.orc_get_state.argtypes = [ctypes.c_void_p, P(ctypes.c_double)]
    L.orc_get_stage_level.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, P(ctypes.c_double)]
    L.orc_get_delays.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, P(ctypes.c_uint8),
                                 P(ctypes.c_uint8)]
    L.orc_set_override.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, P(ctypes.c_uint8)]
    L.orc_get_fluxes.argtypes = [ctypes.c_void_p, ctypes.c_int, P(ctypes.c_double)]
    L.orc_mix64.argtypes = [ctypes.c_uint64]
    L.orc_mix64.restype = ctypes.c_uint64
    L.orc_draw.argtypes = [P(OrcProblem), ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    L.orc_extrap_weights.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_double)]
    L.orc_rhs_sync.argtypes = [P(OrcProblem), P(ctypes.c_double), P(ctypes.c_double)]
    L.orc_lodi.argtypes = [P(OrcProblem), ctypes.c_int, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double),
                           P(ctypes.c_double)]
    L.orc_weno_interp.argtypes = [ctypes.c_double, P(ctypes.c_double), P(ctypes.c_double)]
    L.orc_weno_interp.restype = ctypes.c_double
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def to_struct(pr) -> OrcProblem:
    """Marshal an at_workloads.Problem into the oracle's descriptor."""
    s = OrcProblem()
    s.pde = PDE_IDS[pr.pde]
    s.scheme = SCHEME_IDS[pr.scheme]
    s.mode = MODE_IDS[pr.mode]
    s.rk = RK_IDS[pr.rk]
    s.granularity = GRAN_IDS[pr.granularity]
    s.kmax = pr.kmax
    s.n = pr.n
    s.p = pr.p
    s.n_cdf = len(pr.cdf)
    s.at_levels = int(pr.at_levels)
    s.bc = BC_IDS[getattr(pr, "bc", "periodic")]
    s.form = FORM_IDS[getattr(pr, "form", "flux")]
    for i, v in enumerate(pr.cdf):
        s.cdf[i] = int(v)
    for name in ("x0", "lx", "dt", "c", "alpha", "r", "gamma", "q", "ea", "b", "mu", "pr", "le",
                 "weno_eps"):
        setattr(s, name, float(getattr(pr, name)))
    s.seed = int(pr.seed) & ((1 << 64) - 1)
    s.problem_id = int(pr.problem_id)
    return s


def _check(code: int, what: str = ""):
    if code != 0:
        raise OracleError(code, what)


class Oracle:
    """One oracle run of one problem (FP64, serial)."""

    def __init__(self, pr, q0: Optional[np.ndarray] = None):
        self.pr = pr
        self._s = to_struct(pr)
        self.nf = pr.nf
        q = np.ascontiguousarray(pr.q0 if q0 is None else q0, dtype=np.float64)
        assert q.shape == (self.nf, pr.n)
        h = ctypes.c_void_p()
        _check(lib().orc_create(ctypes.byref(self._s), _dptr(q), ctypes.byref(h)), "create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def step_index(self) -> int:
        return int(lib().orc_current_step(self._h))

    def step(self, n_steps: int = 1) -> "Oracle":
        _check(lib().orc_step(self._h, int(n_steps)), "step")
        return self

    def state(self) -> np.ndarray:
        out = np.empty((self.nf, self.pr.n), dtype=np.float64)
        _check(lib().orc_get_state(self._h, _dptr(out)))
        return out

    def stage_level(self, m: int, s: int) -> np.ndarray:
        out = np.empty((self.nf, self.pr.n), dtype=np.float64)
        _check(lib().orc_get_stage_level(self._h, int(m), int(s), _dptr(out)))
        return out

    def set_history(self, levels: np.ndarray, n_current: int):
        lv = np.ascontiguousarray(levels, dtype=np.float64)
        assert lv.shape[1:] == (self.nf, self.pr.n)
        _check(lib().orc_set_history(self._h, lv.shape[0], _dptr(lv), int(n_current)), "history")

    def delays(self, step0: int, n_steps: int) -> Tuple[np.ndarray, np.ndarray]:
        d = np.empty((n_steps, self.pr.p, 2), dtype=np.uint8)
        e = np.empty_like(d)
        _check(lib().orc_get_delays(self._h, int(step0), int(n_steps), _u8ptr(d), _u8ptr(e)))
        return d, e

    def set_override(self, step0: int, sched: np.ndarray):
        s = np.ascontiguousarray(sched, dtype=np.uint8)
        assert s.ndim == 3 and s.shape[1:] == (self.pr.p, 2)
        _check(lib().orc_set_override(self._h, int(step0), s.shape[0], _u8ptr(s)), "override")

    def fluxes(self, pe: int) -> np.ndarray:
        lo = (pe * self.pr.n) // self.pr.p
        hi = ((pe + 1) * self.pr.n) // self.pr.p
        out = np.empty((hi - lo + 1, self.nf), dtype=np.float64)
        _check(lib().orc_get_fluxes(self._h, int(pe), _dptr(out)))
        return out


def run(pr, steps: Optional[int] = None) -> np.ndarray:
    """Run a problem for `steps` (default pr.steps) and return the final state."""
    with Oracle(pr) as o:
        o.step(pr.steps if steps is None else steps)
        return o.state()


def mix64(z: int) -> int:
    return int(lib().orc_mix64(ctypes.c_uint64(z & ((1 << 64) - 1))))


def draw(pr, step: int, idx: int, side: int) -> int:
    s = to_struct(pr)
    return int(lib().orc_draw(ctypes.byref(s), int(step), int(idx), int(side)))


def extrap_weights(J: int, k: int) -> np.ndarray:
    w = np.empty(J, dtype=np.float64)
    _check(lib().orc_extrap_weights(int(J), int(k), _dptr(w)))
    return w


def rhs_sync(pr, q: np.ndarray) -> np.ndarray:
    s = to_struct(pr)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(pr.nf, pr.n)
    out = np.empty_like(q)
    _check(lib().orc_rhs_sync(ctypes.byref(s), _dptr(q), _dptr(out)))
    return out


def weno_interp(eps: float, v) -> Tuple[float, np.ndarray]:
    """WENO5 interpolation form: value at the right edge of v[2] from v[0..4], and the
    three smoothness indicators."""
    a = np.ascontiguousarray(v, dtype=np.float64)
    assert a.shape == (5,)
    beta = np.empty(3)
    val = lib().orc_weno_interp(float(eps), _dptr(a), _dptr(beta))
    return float(val), beta


def lodi(pr, side: int, drop: bool, prim, dprim) -> np.ndarray:
    """Convective time derivatives of (rho, rho u, rho E, rho Y) at an end point in the
    characteristic form (non-periodic ends)."""
    s = to_struct(pr)
    a = np.ascontiguousarray(prim, dtype=np.float64)
    d = np.ascontiguousarray(dprim, dtype=np.float64)
    out = np.empty(4)
    _check(lib().orc_lodi(ctypes.byref(s), int(side), int(bool(drop)), _dptr(a), _dptr(d), _dptr(out)))
    return out
