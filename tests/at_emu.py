"""ctypes wrapper of libat_emu.so: the CPU emulation of libat's tile kernels.

Test infrastructure of the HIP path: it runs the kernels' own tile code on the
host with bounds checks, using the same planner and workspace layout.  It is
not the oracle (it shares the kernels' code by design) and the product never
loads it.
"""
import ctypes
import os

import numpy as np

from paper_2204_01133_amd import binding

EMU_PATH = os.path.join(os.path.dirname(binding.LIB_PATH), "libat_emu.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(EMU_PATH):
            from paper_2204_01133_amd import build as B
            B.build_emu()
        L = ctypes.CDLL(EMU_PATH)
        vp = ctypes.c_void_p
        P = ctypes.POINTER
        L.emu_init.argtypes = [P(binding.AtProblemDesc), ctypes.c_int, P(binding.AtRunOpts), P(vp)]
        L.emu_error.argtypes = [vp]
        L.emu_error.restype = ctypes.c_char_p
        L.emu_free.argtypes = [vp]
        L.emu_free.restype = None
        L.emu_set_state.argtypes = [vp, ctypes.c_int, vp]
        L.emu_get_state.argtypes = [vp, ctypes.c_int, vp]
        L.emu_step.argtypes = [vp, ctypes.c_int]
        L.emu_rk_stage.argtypes = [vp, ctypes.c_int]
        L.emu_get_delays.argtypes = [vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int, vp, vp]
        L.emu_set_override.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int64, ctypes.c_int]
        L.emu_query.argtypes = [vp, ctypes.c_int]
        L.emu_query.restype = ctypes.c_int64
        _lib = L
    return _lib


class EmuError(RuntimeError):
    pass


class Emu:
    def __init__(self, problems, **opts):
        self.problems = list(problems)
        L = lib()
        arr = (binding.AtProblemDesc * len(self.problems))(*[binding.describe(p) for p in self.problems])
        self._opts = binding.make_opts(**opts)
        h = ctypes.c_void_p()
        rc = L.emu_init(arr, len(self.problems), ctypes.byref(self._opts), ctypes.byref(h))
        self._h = h
        self._chk(rc)
        for b, pr in enumerate(self.problems):
            self.set_state(b, pr.q0)

    def _chk(self, rc):
        if rc != 0:
            raise EmuError(f"emu error {rc}: {lib().emu_error(self._h).decode()}")

    def close(self):
        if self._h:
            lib().emu_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, b, q):
        a = np.ascontiguousarray(q, dtype=np.float64)
        self._chk(lib().emu_set_state(self._h, b, a.ctypes.data_as(ctypes.c_void_p)))

    def step(self, n=1):
        self._chk(lib().emu_step(self._h, int(n)))

    def rk_stage(self, s):
        self._chk(lib().emu_rk_stage(self._h, int(s)))

    def state(self, b):
        pr = self.problems[b]
        out = np.empty((pr.nf, pr.n), dtype=np.float64)
        self._chk(lib().emu_get_state(self._h, b, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def delays(self, b, step0, n):
        P = self.problems[b].p
        d = np.empty((n, P, 2), dtype=np.uint8)
        e = np.empty_like(d)
        self._chk(lib().emu_get_delays(self._h, b, int(step0), int(n), d.ctypes.data_as(ctypes.c_void_p),
                                       e.ctypes.data_as(ctypes.c_void_p)))
        return d, e

    def set_override(self, b, sched, step0=0):
        s = np.ascontiguousarray(sched, dtype=np.uint8)
        self._chk(lib().emu_set_override(self._h, b, s.ctypes.data_as(ctypes.c_void_p), int(step0), s.shape[0]))

    def query(self, key):
        return int(lib().emu_query(self._h, key))
