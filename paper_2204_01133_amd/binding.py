"""ctypes binding of libat (include/at.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libat.so.  PyTorch supplies the device workspace (one uint8 tensor) and the
HIP stream.  If the library is not built, or no GPU is visible, the binding
raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(os.environ.get("AT_BUILD_DIR") or os.path.join(_HERE, "_build"), "libat.so")

PDE_IDS = {"adv_diff": 0, "adr_logistic": 1, "burgers": 2, "euler": 3, "reactive_euler": 4,
           "reactive_ns": 5}
FORM_IDS = {"flux": 0, "chain": 1}
SCHEME_IDS = {"fd2": 0, "fd4": 1, "fd8": 2, "weno5": 3, "weno5i": 4}
MODE_IDS = {"sync": 0, "as": 1, "at": 2}
RK_IDS = {"fe": 0, "rk2": 1, "ssprk3": 2, "rk4": 3}
GRAN_IDS = {"per_pe": 0, "per_pe_side": 1, "per_boundary": 2}
PREC_IDS = {"fp64": 0, "fp32c": 1, "fp32": 2}
BC_IDS = {"periodic": 0, "nscbc": 1}

AT_OK, AT_EINVAL, AT_EUNSUPPORTED, AT_ESTATE, AT_EHIP, AT_ESTALE, AT_ERANGE = 0, -1, -2, -3, -4, -5, -6
Q_STEP, Q_NUM_TILES, Q_NUM_GROUPS, Q_TOTAL_POINTS, Q_STATE_BYTES, Q_STAGES, Q_LDS_BYTES, \
    Q_STRIP_BYTES, Q_NUM_PES = range(9)


class AtProblemDesc(ctypes.Structure):
    _fields_ = [
        ("pde", ctypes.c_int32), ("scheme", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("rk", ctypes.c_int32), ("granularity", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("kmax", ctypes.c_int32), ("at_levels", ctypes.c_int32), ("n_cdf", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("n", ctypes.c_int64), ("p", ctypes.c_int32), ("form", ctypes.c_int32),
        ("cdf", ctypes.c_uint64 * 16),
        ("x0", ctypes.c_double), ("lx", ctypes.c_double), ("dt", ctypes.c_double),
        ("c", ctypes.c_double), ("alpha", ctypes.c_double), ("r", ctypes.c_double),
        ("gamma", ctypes.c_double), ("q", ctypes.c_double), ("ea", ctypes.c_double),
        ("b", ctypes.c_double), ("mu", ctypes.c_double), ("pr", ctypes.c_double),
        ("le", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("problem_id", ctypes.c_int64),
    ]


class AtRunOpts(ctypes.Structure):
    _fields_ = [
        ("tile_points", ctypes.c_int32), ("persistent", ctypes.c_int32),
        ("grid_per_cu", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
        ("xcd_remap", ctypes.c_int32), ("log_steps", ctypes.c_int32),
        ("override_steps", ctypes.c_int32), ("stage_api", ctypes.c_int32),
        ("lds_budget", ctypes.c_int32), ("tile_class", ctypes.c_int32), ("halo_lds", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 5),
    ]


class ATError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libat error {code}: {msg}")
        self.code = code


def describe(pr) -> AtProblemDesc:
    """Marshal a problem (at_workloads.Problem or any object with those fields)."""
    d = AtProblemDesc()
    d.pde = PDE_IDS[pr.pde]
    d.scheme = SCHEME_IDS[pr.scheme]
    d.mode = MODE_IDS[pr.mode]
    d.rk = RK_IDS[pr.rk]
    d.granularity = GRAN_IDS[pr.granularity]
    d.precision = PREC_IDS[pr.precision]
    d.kmax = pr.kmax
    d.at_levels = pr.at_levels
    d.n_cdf = len(pr.cdf)
    d.bc = BC_IDS[getattr(pr, "bc", "periodic")]
    d.form = FORM_IDS[getattr(pr, "form", "flux")]
    for i, v in enumerate(pr.cdf):
        d.cdf[i] = int(v)
    d.n = pr.n
    d.p = pr.p
    for name in ("x0", "lx", "dt", "c", "alpha", "r", "gamma", "q", "ea", "b", "mu", "pr", "le",
                 "weno_eps"):
        setattr(d, name, float(getattr(pr, name)))
    d.seed = int(pr.seed) & ((1 << 64) - 1)
    d.problem_id = int(pr.problem_id)
    return d


def make_opts(**kw) -> AtRunOpts:
    """Run options by field name of at_run_opts; an unknown name raises."""
    o = AtRunOpts()
    known = {name for name, _ in AtRunOpts._fields_ if name != "reserved"}
    for k, v in kw.items():
        if k not in known:
            raise TypeError(f"unknown run option {k!r} (known: {', '.join(sorted(known))})")
        setattr(o, k, int(v))
    return o


_lib = None


def load_library():
    """Load libat.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libat.so not built ({LIB_PATH}); run python -m paper_2204_01133_amd.build")
    from . import build as _build
    try:
        with open(_build.STAMP) as fh:
            stamp = fh.read().strip()
    except OSError:
        stamp = None
    if stamp != _build.source_hash():
        raise RuntimeError(f"libat.so ({LIB_PATH}) was not built from the current sources "
                           f"(stamp {stamp}, sources {_build.source_hash()}); rebuild with "
                           "python -m paper_2204_01133_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.at_init.argtypes = [P(AtProblemDesc), ctypes.c_int, P(AtRunOpts), P(vp), P(ctypes.c_size_t)]
    L.at_bind.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.at_bind_scratch.argtypes = [vp, vp]
    L.at_set_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
    L.at_reset.argtypes = [vp]
    L.at_rk_stage.argtypes = [vp, ctypes.c_int]
    L.at_step.argtypes = [vp, ctypes.c_int]
    L.at_batch_step.argtypes = [vp, ctypes.c_int]
    L.at_get_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
    L.at_get_delays.argtypes = [vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int, vp, vp]
    L.at_set_delay_override.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int64, ctypes.c_int]
    L.at_sync.argtypes = [vp]
    L.at_query.argtypes = [vp, ctypes.c_int, P(ctypes.c_int64)]
    L.at_stream.argtypes = [vp]
    L.at_stream.restype = vp
    L.at_strerror.argtypes = [ctypes.c_int]
    L.at_strerror.restype = ctypes.c_char_p
    L.at_last_error.argtypes = [vp]
    L.at_last_error.restype = ctypes.c_char_p
    L.at_free.argtypes = [vp]
    L.at_free.restype = None
    _lib = L
    return L


EXPORTED = ["at_init", "at_bind", "at_bind_scratch", "at_set_state", "at_reset", "at_rk_stage", "at_step",
            "at_batch_step", "at_get_state", "at_get_delays", "at_set_delay_override", "at_sync",
            "at_query", "at_stream", "at_strerror", "at_last_error", "at_free"]


class ATSolver:
    """Many independent periodic problems advanced by libat on one GPU.

    problems: sequence of at_workloads.Problem-like objects (their q0 is used
    as the level-0 state unless set_state is called).  opts: at_run_opts keys.
    scratch: bind the library's own device scratch (at_bind_scratch) instead of
    a workspace allocated here; for workloads whose workspace fits it.
    tuned: path of an autotuner cache; the run options it holds for this workload
    and device are used (opts given here override them).
    """

    def __init__(self, problems: Sequence, device: str = "cuda:0", stream=None, set_initial: bool = True,
                 scratch: bool = False, tuned: Optional[str] = None, **opts):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("ATSolver needs a GPU (HIP device); there is no CPU path")
        if tuned is not None:
            from .autotune import cached_opts
            opts = dict(cached_opts(problems, tuned), **opts)
        self.run_opts = dict(opts)           # the run options in effect (tuned ones included)
        self.torch = torch
        self.L = load_library()
        self.problems = list(problems)
        self.device = torch.device(device)
        arr = (AtProblemDesc * len(self.problems))(*[describe(p) for p in self.problems])
        self._descs = arr
        self._opts = make_opts(**opts)
        h = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        with torch.cuda.device(self.device):
            self._check(self.L.at_init(arr, len(self.problems), ctypes.byref(self._opts), ctypes.byref(h),
                                       ctypes.byref(nbytes)), None)
            self._h = h
            self.workspace_bytes = int(nbytes.value)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if scratch:
                self.ws = None
                self._check(self.L.at_bind_scratch(self._h, ctypes.c_void_p(self.stream.cuda_stream)))
                if set_initial:
                    for b, pr in enumerate(self.problems):
                        self.set_state(b, pr.q0)
                return
            self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            # the workspace is used on the solver's stream: its memory is not handed to
            # another tensor before that stream's pending work is done
            if self.stream != torch.cuda.current_stream(self.device):
                self.ws.record_stream(self.stream)
            base = self.ws.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            self._check(self.L.at_bind(self._h, ctypes.c_void_p(self._ws_ptr), self.workspace_bytes,
                                       ctypes.c_void_p(self.stream.cuda_stream)))
            if set_initial:
                for b, pr in enumerate(self.problems):
                    self.set_state(b, pr.q0)

    # -- helpers ---------------------------------------------------------------
    def _check(self, rc: int, h="self"):
        if rc != 0:
            handle = self._h if h == "self" else None
            # without a context (a failed at_init), the planner's message of this thread
            msg = self.L.at_last_error(handle).decode() or self.L.at_strerror(rc).decode()
            raise ATError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self.L.at_sync(self._h)             # no launch in flight on the workspace
            self.L.at_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API -------------------------------------------------------------------
    def set_state(self, b: int, q):
        torch = self.torch
        if isinstance(q, torch.Tensor) and q.is_cuda:
            # q (and its converted copy) are written on the caller's current stream and
            # read by the library on the solver's stream: order the two, and keep their
            # memory from being reused before the solver's stream has read it
            cur = torch.cuda.current_stream(self.device)
            t = q.to(dtype=torch.float64).contiguous()
            if self.stream != cur:
                self.stream.wait_stream(cur)
            self._check(self.L.at_set_state(self._h, b, ctypes.c_void_p(t.data_ptr()), 1))
            if self.stream != cur:
                t.record_stream(self.stream)
                q.record_stream(self.stream)
        else:
            a = np.ascontiguousarray(q, dtype=np.float64)
            self._check(self.L.at_set_state(self._h, b, a.ctypes.data_as(ctypes.c_void_p), 0))

    def reset(self):
        self._check(self.L.at_reset(self._h))

    def step(self, n: int = 1):
        self._check(self.L.at_step(self._h, int(n)))

    def batch_step(self, n: int = 1):
        self._check(self.L.at_batch_step(self._h, int(n)))

    def rk_stage(self, s: int):
        self._check(self.L.at_rk_stage(self._h, int(s)))

    def sync(self):
        self._check(self.L.at_sync(self._h))

    def state(self, b: int) -> np.ndarray:
        pr = self.problems[b]
        out = np.empty((pr.nf, pr.n), dtype=np.float64)
        self._check(self.L.at_get_state(self._h, b, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def state_device(self, b: int):
        """The state as a device tensor, ready for work on the caller's current stream
        (which is made to wait for the solver's stream)."""
        torch = self.torch
        pr = self.problems[b]
        cur = torch.cuda.current_stream(self.device)
        out = torch.empty((pr.nf, pr.n), dtype=torch.float64, device=self.device)
        if self.stream != cur:
            self.stream.wait_stream(cur)        # out's memory is free on the solver's stream too
        self._check(self.L.at_get_state(self._h, b, ctypes.c_void_p(out.data_ptr()), 1))
        if self.stream != cur:
            out.record_stream(self.stream)
            cur.wait_stream(self.stream)
        return out

    def delays(self, b: int, step0: int, n_steps: int) -> Tuple[np.ndarray, np.ndarray]:
        P = self.problems[b].p
        d = np.empty((n_steps, P, 2), dtype=np.uint8)
        e = np.empty_like(d)
        self._check(self.L.at_get_delays(self._h, b, int(step0), int(n_steps),
                                         d.ctypes.data_as(ctypes.c_void_p), e.ctypes.data_as(ctypes.c_void_p)))
        return d, e

    def set_override(self, b: int, sched: Optional[np.ndarray], step0: int = 0):
        if sched is None:
            self._check(self.L.at_set_delay_override(self._h, b, None, 0, 0))
            return
        s = np.ascontiguousarray(sched, dtype=np.uint8)
        self._check(self.L.at_set_delay_override(self._h, b, s.ctypes.data_as(ctypes.c_void_p), int(step0),
                                                 s.shape[0]))

    def query(self, key: int) -> int:
        v = ctypes.c_int64()
        self._check(self.L.at_query(self._h, key, ctypes.byref(v)))
        return int(v.value)
