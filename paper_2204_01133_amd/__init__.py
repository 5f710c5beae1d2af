"""MI355X (gfx950) implementation of the asynchrony-tolerant multi-stage
Runge-Kutta hot path of Kumari et al., arXiv:2204.01133.

The compute path is libat.so (hand-written HIP kernels behind the C ABI of
include/at.h); :mod:`paper_2204_01133_amd.binding` marshals arguments to it.
"""
from .binding import ATError, ATSolver, describe, load_library, make_opts  # noqa: F401

__all__ = ["ATSolver", "ATError", "describe", "load_library", "make_opts"]
