"""Pins of the oracle's time integration and of the reductions the paper states.

* Synchronous FD + RK (eq. rk1): von Neumann closed form.  A Fourier mode is
  multiplied per step by the stability polynomial of the RK scheme (the
  truncated exponential for these tableaus) at z = dt * symbol of the stencil;
  the symbol is built here from weights re-derived by a Vandermonde solve.
* Zero delay (Sec. 2.2 after eq. at1; Sec. 2.3 after eq. rkat2; Sec. 3 after
  eqs. atRecon / beta2AT2): AT and AS with every delay 0 are bitwise the
  synchronous scheme.
* Conservation on periodic domains (flux-difference / central forms telescope)
  in synchronous mode; fixed points u = 0, u = 1 of the logistic problem for
  any delays (extrapolation weights sum to 1).
"""
import math

import numpy as np
import pytest

import at_workloads as W
import oracle
from test_oracle_stencils import fd_weights


def symbol(order, theta, deriv):
    offs, w = fd_weights(order, deriv)
    return np.sum(w[None, :] * np.exp(1j * np.outer(theta, offs)), axis=1)


@pytest.mark.parametrize("scheme,order", [("fd2", 2), ("fd4", 4), ("fd8", 8)])
@pytest.mark.parametrize("rk,S", [("fe", 1), ("rk2", 2), ("ssprk3", 3), ("rk4", 4)])
def test_sync_fourier_closed_form(scheme, order, rk, S):
    n, m, steps = 64, 3, 40
    c, alpha = 1.0, 2e-3
    pr = W.adv_diff_c1(n=n, p=4, mode="sync", steps=steps, c=c, alpha=alpha, scheme=scheme,
                       rk=rk, cfl=0.1, kmax=0)
    x = pr.x()
    ph = 0.3
    pr = pr.replace(q0=np.sin(2 * np.pi * m * x + ph)[None])
    u = oracle.run(pr)[0]
    dx = pr.dx
    theta = np.array([2 * np.pi * m * dx])
    lam = -c * symbol(order, theta, 1)[0] / dx + alpha * symbol(order, theta, 2)[0] / dx ** 2
    z = pr.dt * lam
    G = sum(z ** j / math.factorial(j) for j in range(S + 1))
    want = np.imag(G ** steps * np.exp(1j * (2 * np.pi * m * x + ph)))
    np.testing.assert_allclose(u, want, atol=2e-13)


def _zero_override(pr, steps):
    return np.zeros((steps, pr.p, 2), dtype=np.uint8)


@pytest.mark.parametrize("make", [
    lambda: W.adv_diff_c1(n=128, p=8, kmax=3, steps=20),
    lambda: W.batched_adr_c3(n_problems=1, n_min=256, n_max=256)[0].replace(steps=20),
    lambda: W.euler_sod_c4(n=256, p=8, steps=20),
    lambda: W.euler_sod_c4(n=256, p=8, steps=20).replace(scheme="weno5i"),
    lambda: W.burgers_sweep(64, p=8),
    lambda: W.reactive_ns_c2(n=256, p=8, steps=10),
    lambda: W.reactive_ns_c2(n=256, p=8, steps=10).replace(form="chain"),
    lambda: W.detonation_c5(n=512, p=8, steps=10, precision="fp64"),
])
@pytest.mark.parametrize("mode", ["at", "as"])
def test_zero_delay_is_bitwise_synchronous(make, mode):
    pr = make().replace(mode=mode)
    steps = min(pr.steps, 20)
    o = oracle.Oracle(pr)
    o.set_override(0, _zero_override(pr, steps))
    o.step(steps)
    a = o.state()
    s = oracle.run(pr.replace(mode="sync"), steps)
    assert np.array_equal(a, s)


def test_sync_independent_of_pe_count():
    base = W.euler_sod_c4(n=256, p=1, steps=30, mode="sync")
    ref = oracle.run(base)
    for p in (2, 7, 256):
        assert np.array_equal(oracle.run(base.replace(p=p)), ref)


def test_sync_conservation():
    pr = W.adv_diff_c1(n=256, p=8, mode="sync", steps=200)
    u0 = pr.q0.sum()
    u = oracle.run(pr)
    assert abs(u.sum() - u0) < 1e-11
    pe = W.euler_sod_c4(n=512, p=8, mode="sync", steps=100)
    q = oracle.run(pe)
    np.testing.assert_allclose(q.sum(axis=1), pe.q0.sum(axis=1), rtol=1e-13, atol=1e-11)


def test_at_breaks_telescoping_but_drift_is_small():
    # AT: two PEs evaluate the same interface differently, so the sum drifts by
    # O(truncation error) -- expected, and it shrinks with resolution.
    drift = []
    for n in (128, 256):
        pr = W.euler_sod_c4(n=n, p=8, steps=int(40 * n / 128), kmax=2)
        q = oracle.run(pr)
        drift.append(abs(q[0].sum() - pr.q0[0].sum()) / n)
    assert 0 < drift[1] < drift[0]


@pytest.mark.parametrize("value", [0.0, 1.0])
def test_logistic_fixed_points_under_delays(value):
    pr = W.batched_adr_c3(n_problems=1, n_min=512, n_max=512)[0]
    pr = pr.replace(q0=np.full((1, pr.n), value), steps=50)
    u = oracle.run(pr)
    assert np.abs(u - value).max() < 1e-12
