"""The oracle's WENO interpolation form (Sec. 3, eqs. interpS, fullSten, omg, betaS; the AT
form through the two-level extrapolated halo of eq. stenF) as a scheme for the flux
derivative of eq. wender.  The candidate coefficients, weights and smoothness indicators
are pinned in test_oracle_weno_design.py; here the scheme as a whole: interface values
interpolated at fifth order and differenced give a second-order derivative (the reason
the paper's simulations use the reconstruction form), AT keeps the synchronous error,
and shocks stay captured (exact Riemann solution of Sod)."""
import numpy as np

import at_workloads as W
import oracle
from test_oracle_convergence import order, sod_periodic_exact


def test_linear_advection_orders():
    ns = [64, 128, 256]
    errs = {"sync": [], "at": []}
    for mode in errs:
        for n in ns:
            pr = W.advection_e1(n, p=4, mode=mode, delay="half").replace(scheme="weno5i")
            u = oracle.run(pr)[0]
            errs[mode].append(np.abs(u - np.sin(np.pi * (pr.x() - 5.0)) ** 4).mean())
    assert 1.8 < order(errs["sync"])[-1] < 2.2, errs
    assert 1.8 < order(errs["at"])[-1] < 2.2, errs
    assert abs(errs["at"][-1] - errs["sync"][-1]) < 0.01 * errs["sync"][-1], errs
    # the reconstruction form is far more accurate at the same resolution
    pr = W.advection_e1(ns[-1], p=4, mode="sync")
    e5 = np.abs(oracle.run(pr)[0] - np.sin(np.pi * (pr.x() - 5.0)) ** 4).mean()
    assert e5 < 0.05 * errs["sync"][-1]


def test_sod_against_exact_riemann():
    t_end = 0.1
    errs = {"sync": [], "at": []}
    for n in (256, 512):
        base = W.euler_sod_c4(n=n, p=8, kmax=2).replace(scheme="weno5i")
        steps = int(round(t_end / base.dt))
        base = base.replace(dt=t_end / steps, steps=steps)
        ex = sod_periodic_exact(base.x(), t_end)
        for mode in errs:
            q = oracle.run(base.replace(mode=mode))
            assert np.isfinite(q).all() and q[0].min() > 0
            errs[mode].append(np.abs(q[0] - ex[0]).mean())
    assert errs["sync"][0] > errs["sync"][1] and errs["at"][0] > errs["at"][1], errs
    assert errs["sync"][1] < 0.01, errs
    for a, s in zip(errs["at"], errs["sync"]):
        assert abs(a - s) < 0.3 * s, errs
