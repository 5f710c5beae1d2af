"""Pins of the oracle's spatial schemes against what the paper prints.

* Central FD weights: polynomial exactness (Taylor constraints, the same
  construction as eq. geDer with a single level) -- weights are re-derived here
  by a Vandermonde solve, not copied from the oracle.
* AT weights: Lagrange extrapolation, exact small integers, and the delay
  polynomials of Table A (App. A).
* Table A (App. A): the (1,4) and (2,4) AT schemes, left and right boundary,
  for delays 0..4, through one real forward-Euler step of the oracle.
* eq. at1 (Sec. 2.2): 2nd-order AT first derivative (printed without the 1/2
  of the central difference; the oracle follows the consistent reading).
* AT-WENO (Sec. 3 eqs. atRecon, beta2AT0-2; App. B eqs. atReconR, atReconRm,
  atReconM, beta2AT0-1 and beta2AT2R): the printed candidate reconstructions
  and AT smoothness indicators with ideal weights {1/10, 3/5, 3/10} (eq. idRec)
  and nonlinear weights of eq. omg reproduce the oracle's interface fluxes.
"""
import math

import numpy as np
import pytest

import at_workloads as W
import oracle


# --------------------------------------------------------------------------
# central finite differences
# --------------------------------------------------------------------------
def fd_weights(order, deriv):
    """Central weights on offsets -H..H from the Taylor (Vandermonde) system."""
    H = order // 2
    offs = np.arange(-H, H + 1, dtype=float)
    A = np.vander(offs, increasing=True).T           # rows: powers 0..2H
    rhs = np.zeros(2 * H + 1)
    rhs[deriv] = math.factorial(deriv)
    return offs, np.linalg.solve(A, rhs)


@pytest.mark.parametrize("scheme,order", [("fd2", 2), ("fd4", 4), ("fd8", 8)])
def test_fd_polynomial_exactness(scheme, order):
    H = order // 2
    n = 64
    for deg in range(order + 2):
        x = np.arange(n, dtype=float) + 0.5
        u = ((x - 30.0) / 7.0) ** deg
        d1 = deg * ((x - 30.0) / 7.0) ** max(deg - 1, 0) / 7.0 if deg else 0 * x
        d2 = deg * (deg - 1) * ((x - 30.0) / 7.0) ** max(deg - 2, 0) / 49.0 if deg > 1 else 0 * x
        for c, a, want in [(1.0, 0.0, -d1), (0.0, 1.0, d2)]:
            if (a == 0 and deg > order) or (c == 0 and deg > order + 1):
                continue
            pr = W.Problem(pde="adv_diff", scheme=scheme, n=n, p=1, dt=1.0, q0=u[None], mode="sync",
                           rk="fe", c=c, alpha=a, lx=float(n))
            k = oracle.rhs_sync(pr, u)[0]
            sl = slice(H, n - H)
            np.testing.assert_allclose(k[sl], want[sl], rtol=1e-9, atol=1e-9 * (1 + abs(want).max()))


# --------------------------------------------------------------------------
# Lagrange extrapolation weights
# --------------------------------------------------------------------------
def test_extrapolation_weights_small_integers():
    known = {
        (2, 0): [1, 0], (2, 1): [2, -1], (2, 4): [5, -4],
        (3, 0): [1, 0, 0], (3, 1): [3, -3, 1], (3, 2): [6, -8, 3], (3, 3): [10, -15, 6],
        (3, 4): [15, -24, 10], (5, 4): [70, -224, 280, -160, 35],
    }
    for (J, k), w in known.items():
        assert oracle.extrap_weights(J, k).tolist() == [float(v) for v in w]


@pytest.mark.parametrize("J", [1, 2, 3, 4, 5])
def test_extrapolation_exact_on_polynomials(J):
    rng = np.random.default_rng(J)
    for k in range(6):
        w = oracle.extrap_weights(J, k)
        assert abs(w.sum() - 1.0) < 1e-14
        for deg in range(J):
            coef = rng.normal(size=deg + 1)
            t = -(k + np.arange(J, dtype=float))
            vals = np.polyval(coef, t)
            assert abs(w @ vals - np.polyval(coef, 0.0)) < 1e-9 * (1 + abs(vals).max()) * 10 ** J


def test_table_a_delay_polynomials():
    # Table A: level n-k weighted by (k^2+3k+2)/2, n-k-1 by -(k^2+2k), n-k-2 by (k^2+k)/2
    for k in range(8):
        w = oracle.extrap_weights(3, k)
        assert w.tolist() == [(k * k + 3 * k + 2) / 2, -(k * k + 2 * k), (k * k + k) / 2]


# --------------------------------------------------------------------------
# helpers: one forward-Euler step from a given random history
# --------------------------------------------------------------------------
def one_step_from_history(pr, hist, n_cur, kL, kR):
    """hist[l] = level n_cur - (len-1) + l.  PE 1's left side gets delay kL,
    PE 0's right side gets kR (P = 2).  Returns (K = u^{n+1} - u^n with dt = 1)."""
    o = oracle.Oracle(pr)
    o.set_history(hist, n_cur)
    sched = np.zeros((1, pr.p, 2), dtype=np.uint8)
    sched[0, 1, 0] = kL
    sched[0, 0, 1] = kR
    sched[0, 0, 0] = 1
    sched[0, 1, 1] = 2
    o.set_override(n_cur, sched)
    o.step(1)
    return o, (o.state() - hist[-1])[0]


def test_table_a_at_schemes_through_oracle_step():
    n, J, kmax = 16, 3, 4
    rng = np.random.default_rng(11)
    D = kmax + J
    hist = rng.uniform(-1, 1, size=(D, 1, n))
    n_cur = D - 1
    U = lambda lvl, j: hist[lvl - (n_cur - (D - 1)), 0, j % n]  # noqa: E731
    for kind in ("d1", "d2"):
        c, a = (1.0, 0.0) if kind == "d1" else (0.0, 1.0)
        pr = W.Problem(pde="adv_diff", scheme="fd4", n=n, p=2, dt=1.0, q0=hist[-1], mode="at",
                       rk="fe", kmax=kmax, c=c, alpha=a, lx=float(n))
        for k in range(kmax + 1):
            _, K = one_step_from_history(pr, hist, n_cur, k, k)
            nn = n_cur
            co = [(k * k + 3 * k + 2) / 2, -(k * k + 2 * k), (k * k + k) / 2]
            # left boundary point j = 8 (PE 1), delayed j-1, j-2
            j = 8
            if kind == "d2":
                want = sum(co[l] * (-U(nn, j + 2) + 16 * U(nn, j + 1) - 30 * U(nn, j)
                                    + 16 * U(nn - k - l, j - 1) - U(nn - k - l, j - 2)) / 12.0
                           for l in range(3))
            else:
                want = -sum(co[l] * (-U(nn, j + 2) + 8 * U(nn, j + 1) - 8 * U(nn - k - l, j - 1)
                                     + U(nn - k - l, j - 2)) / 12.0 for l in range(3))
            assert abs(K[j] - want) < 1e-11 * (1 + abs(want)), (kind, k, "left")
            # right boundary point j = 7 (PE 0), delayed j+1, j+2
            j = 7
            if kind == "d2":
                want = sum(co[l] * (-U(nn - k - l, j + 2) + 16 * U(nn - k - l, j + 1) - 30 * U(nn, j)
                                    + 16 * U(nn, j - 1) - U(nn, j - 2)) / 12.0 for l in range(3))
            else:
                want = -sum(co[l] * (-U(nn - k - l, j + 2) + 8 * U(nn - k - l, j + 1)
                                     - 8 * U(nn, j - 1) + U(nn, j - 2)) / 12.0 for l in range(3))
            assert abs(K[j] - want) < 1e-11 * (1 + abs(want)), (kind, k, "right")


def test_eq_at1_second_order_at_first_derivative():
    # eq. at1 prints (k u_{j-1}^{n-k-1} - (k+1) u_{j-1}^{n-k} + u_{j+1}) / dx; this is twice
    # the central difference (u_{j+1} - u~_{j-1}) / (2 dx) on the extrapolated buffer value
    # u~ = (k+1) u^{n-k} - k u^{n-k-1}, i.e. the print drops the 1/2 (read as a typo).
    n, kmax = 16, 4
    rng = np.random.default_rng(5)
    D = kmax + 2
    hist = rng.uniform(-1, 1, size=(D, 1, n))
    n_cur = D - 1
    pr = W.Problem(pde="adv_diff", scheme="fd2", n=n, p=2, dt=1.0, q0=hist[-1], mode="at", rk="fe",
                   kmax=kmax, c=1.0, alpha=0.0, lx=float(n))
    for k in range(kmax + 1):
        _, K = one_step_from_history(pr, hist, n_cur, k, k)
        j = 8
        U = lambda lvl, jj: hist[lvl - (n_cur - (D - 1)), 0, jj]  # noqa: E731
        printed = k * U(n_cur - k - 1, j - 1) - (k + 1) * U(n_cur - k, j - 1) + U(n_cur, j + 1)
        assert abs(K[j] - (-printed / 2.0)) < 1e-12


# --------------------------------------------------------------------------
# AT-WENO: printed reconstructions and smoothness indicators
# --------------------------------------------------------------------------
EPS = 1e-6


def _omega_combine(u, beta, gam):
    a = [g / (EPS + b) ** 2 for g, b in zip(gam, beta)]
    return sum(ai * ui for ai, ui in zip(a, u)) / sum(a)


def _beta_sync(v0, v1, v2):
    # eq. betaS, first line (stencil {j-2, j-1, j} in its printed variables)
    return (4 * v0 ** 2 + (11 * v2 - 19 * v1) * v0 + 25 * v1 ** 2 + 10 * v2 ** 2 - 31 * v1 * v2) / 3.0


def _beta_sync2(uj, uj1, uj2):
    # eq. beta2AT2 (= beta^(2) of eq. betaS)
    return (10 * uj ** 2 - 31 * uj1 * uj + 25 * uj1 ** 2 + 4 * uj2 ** 2 + (11 * uj - 19 * uj1) * uj2) / 3.0


def left_paper(k, A, a, B, b, u0, u1, u2):
    """Left PE boundary, j = boundary point.  A = u_{j-2}^{n-k}, a = u_{j-2}^{n-k-1},
    B = u_{j-1}^{n-k}, b = u_{j-1}^{n-k-1}, u0 = u_j^n, u1 = u_{j+1}^n, u2 = u_{j+2}^n."""
    # eq. atRecon (reconstruction at j+1/2)
    rp = [-k * a / 3 + 7 * k * b / 6 + (2 * k + 2) * A / 6 + (-7 * k - 7) * B / 6 + 11 * u0 / 6,
          k * b / 6 + (-k - 1) * B / 6 + 5 * u0 / 6 + u1 / 3,
          u0 / 3 + 5 * u1 / 6 - u2 / 6]
    # eq. atReconM (reconstruction at j-1/2)
    rm = [k * a / 6 - 5 * k * b / 6 + (-k - 1) * A / 6 + (5 * k + 5) * B / 6 + u0 / 3,
          -k * b / 3 + (2 * k + 2) * B / 6 + 5 * u0 / 6 - u1 / 6,
          11 * u0 / 6 - 7 * u1 / 6 + u2 / 3]
    # eqs. beta2AT0, beta2AT1, beta2AT2
    b0 = (4 * A ** 2 + 25 * B ** 2
          + k ** 2 * (4 * a ** 2 + 4 * A ** 2 + 19 * A * (b - B) + 25 * (b - B) ** 2
                      + a * (19 * (B - b) - 8 * A))
          - 31 * u0 * B + 10 * u0 ** 2 + A * (11 * u0 - 19 * B)
          + k * (8 * A ** 2 + (19 * b - 38 * B + 11 * u0) * A + a * (-8 * A + 19 * B - 11 * u0)
                 - (b - B) * (50 * B - 31 * u0))) / 3.0
    b1 = (4 * k ** 2 * (b - B) ** 2 + 4 * B ** 2 + 13 * u0 ** 2 + 4 * u1 ** 2 + (5 * u1 - 13 * u0) * B
          - 13 * u0 * u1 - k * (b - B) * (8 * B - 13 * u0 + 5 * u1)) / 3.0
    b2 = _beta_sync2(u0, u1, u2)
    return rp, rm, [b0, b1, b2]


def right_paper(k, C, c, Dv, d, um2, um1, u0):
    """Right PE boundary, j = boundary point.  C = u_{j+1}^{n-k}, c = u_{j+1}^{n-k-1},
    Dv = u_{j+2}^{n-k}, d = u_{j+2}^{n-k-1}; um2, um1, u0 = u_{j-2}, u_{j-1}, u_j at n."""
    # eq. atReconR (at j+1/2)
    rp = [um2 / 3 - 7 * um1 / 6 + 11 * u0 / 6,
          -k * c / 3 + (2 * k + 2) * C / 6 - um1 / 6 + 5 * u0 / 6,
          -5 * k * c / 6 + k * d / 6 + (5 * k + 5) * C / 6 + (-k - 1) * Dv / 6 + u0 / 3]
    # eq. atReconRm (at j-1/2)
    rm = [-um2 / 6 + 5 * um1 / 6 + u0 / 3,
          k * c / 6 + (-k - 1) * C / 6 + um1 / 3 + 5 * u0 / 6,
          7 * k * c / 6 - k * d / 3 + (-7 * k - 7) * C / 6 + (2 * k + 2) * Dv / 6 + 11 * u0 / 6]
    # App. B: beta2AT0 (synchronous), beta2AT1, beta2AT2R
    b0 = _beta_sync(um2, um1, u0)
    e = k * c - (k + 1) * C
    b1 = (um1 * (-5 * k * c + 5 * (k + 1) * C - 13 * u0) + 4 * e ** 2 + 13 * u0 * e
          + 4 * um1 ** 2 + 13 * u0 ** 2) / 3.0
    b2 = (k ** 2 * (25 * c ** 2 + (19 * (Dv - d) - 50 * C) * c + 25 * C ** 2 + 4 * (d - Dv) ** 2
                    + 19 * C * (d - Dv))
          + k * (50 * C ** 2 + 19 * (d - 2 * Dv) * C + 8 * Dv * (Dv - d) + c * (19 * Dv - 50 * C))
          + 25 * C ** 2 + 4 * Dv ** 2 - 19 * C * Dv
          + u0 * (-31 * C + 11 * Dv + k * (31 * c - 31 * C - 11 * d + 11 * Dv)) + 10 * u0 ** 2) / 3.0
    return rp, rm, [b0, b1, b2]


GAM_P = (0.1, 0.6, 0.3)      # eq. idRec, left-biased (C+)
GAM_M = (0.3, 0.6, 0.1)      # its mirror for the right-biased (C-) reconstruction


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_at_weno_printed_formulas(k):
    n, kmax = 16, 4
    D = kmax + 2
    rng = np.random.default_rng(100 + k)
    hist = rng.uniform(0.2, 1.0, size=(D, 1, n))
    n_cur = D - 1
    U = lambda lvl, j: hist[lvl - (n_cur - (D - 1)), 0, j % n]  # noqa: E731
    nn = n_cur
    for c in (1.0, -1.0):
        pr = W.Problem(pde="adv_diff", scheme="weno5", n=n, p=2, dt=1.0, q0=hist[-1], mode="at",
                       rk="fe", kmax=kmax, c=c, alpha=0.0, lx=float(n))
        o, _ = one_step_from_history(pr, hist, n_cur, k, k)
        f0, f1 = o.fluxes(0), o.fluxes(1)
        # left boundary of PE 1: j = 8
        j = 8
        rp, rm, beta = left_paper(k, U(nn - k, j - 2), U(nn - k - 1, j - 2), U(nn - k, j - 1),
                                  U(nn - k - 1, j - 1), U(nn, j), U(nn, j + 1), U(nn, j + 2))
        # right boundary of PE 0: j = 7
        jr = 7
        rpR, rmR, betaR = right_paper(k, U(nn - k, jr + 1), U(nn - k - 1, jr + 1), U(nn - k, jr + 2),
                                      U(nn - k - 1, jr + 2), U(nn, jr - 2), U(nn, jr - 1), U(nn, jr))
        if c > 0:   # C+ = u, C- = 0: flux = left-biased WENO of u
            got_l, want_l = f1[1, 0], _omega_combine(rp, beta, GAM_P)        # j + 1/2
            got_r, want_r = f0[-1, 0], _omega_combine(rpR, betaR, GAM_P)     # j + 1/2
        else:       # C+ = 0, C- = -u: flux = -(right-biased WENO of u)
            got_l, want_l = f1[0, 0], -_omega_combine(rm, beta, GAM_M)       # j - 1/2
            got_r, want_r = f0[-2, 0], -_omega_combine(rmR, betaR, GAM_M)    # j - 1/2
        assert abs(got_l - want_l) < 1e-12, (k, c, "left", got_l, want_l)
        assert abs(got_r - want_r) < 1e-12, (k, c, "right", got_r, want_r)


def test_weno_ideal_weights_give_fifth_order_stencil():
    # Smooth data: WENO tends to the linear 5th-order combination (2,-13,47,27,-3)/60
    # (ideal weights of eq. idRec).  Use a tiny-amplitude linear profile (all beta
    # ~ 0 so the nonlinear weights equal the ideal ones).
    n = 16
    x = np.arange(n) + 0.5
    u = 1.0 + 1e-9 * x
    pr = W.Problem(pde="adv_diff", scheme="weno5", n=n, p=1, dt=1.0, q0=u[None], mode="at", rk="fe",
                   kmax=0, c=1.0, lx=float(n))
    o = oracle.Oracle(pr)
    o.step(1)
    f = o.fluxes(0)[:, 0]
    for i in range(3, 12):
        lin = (2 * u[i - 2] - 13 * u[i - 1] + 47 * u[i] + 27 * u[i + 1] - 3 * u[i + 2]) / 60.0
        assert abs(f[i + 1] - lin) < 1e-14
