"""Pin of the oracle's spatial right-hand sides against the continuous PDEs.

For smooth periodic fields, the synchronous discrete RHS (central FD of order
2/4/8 or LLF-WENO5) must converge to the exact continuous RHS at the scheme's
order.  The exact RHS is derived here symbolically (sympy) from the
conservative flux form of each PDE (Sec. 4, eq. ge, in one dimension, with the
one-step-chemistry closure: R = 1, E = T/(gamma-1) + u^2/2 + q Y, constant mu,
kappa = mu c_p / Pr, rho D = mu / (Pr Le), fuel enthalpy q carried by the
diffusive flux).  The oracle instead evaluates the expanded, non-conservative
form of the viscous terms and the flux-split WENO reconstruction, so a dropped
term, a wrong sign or coefficient, or a swapped operand in any field's RHS
leaves an O(1) residual that does not shrink under refinement.
"""
import numpy as np
import pytest
import sympy as sp

import at_workloads as W
import oracle

X = sp.symbols("x", real=True)
TWO_PI = 2 * sp.pi

# smooth, periodic on [0, 1), no constant states (every derivative is exercised)
RHO = 1 + sp.Rational(1, 5) * sp.sin(TWO_PI * X)
U = sp.Rational(1, 10) + sp.Rational(3, 10) * sp.cos(TWO_PI * X)
T = 1 + sp.Rational(1, 10) * sp.sin(2 * TWO_PI * X + sp.Rational(3, 10))
Y = sp.Rational(1, 2) + sp.Rational(3, 10) * sp.cos(TWO_PI * X + sp.Rational(7, 10))
S1 = sp.Rational(1, 2) + sp.Rational(1, 5) * sp.sin(TWO_PI * X) \
    + sp.Rational(1, 10) * sp.cos(3 * TWO_PI * X + 1)

GAMMA, QH, EA, B, MU, PR, LE = 1.4, 0.5, 2.0, 1.5, 0.01, 0.72, 1.3
C, ALPHA, R = 0.7, 3e-3, 2.5


def _exact(pde, alpha=ALPHA):
    """Conserved fields and the exact RHS d(q)/dt as sympy expressions."""
    g = sp.Float(GAMMA)
    d = lambda e: sp.diff(e, X)  # noqa: E731
    if pde in ("adv_diff", "adr_logistic"):
        rhs = -C * d(S1) + alpha * d(d(S1))
        if pde == "adr_logistic":
            rhs += R * S1 * (1 - S1)
        return [S1], [rhs]
    if pde == "burgers":
        return [S1], [-d(S1 ** 2 / 2)]
    p = RHO * T
    if pde == "euler":
        rhoE = p / (g - 1) + RHO * U ** 2 / 2
        q = [RHO, RHO * U, rhoE]
        flux = [RHO * U, RHO * U ** 2 + p, (rhoE + p) * U]
        return q, [-d(f) for f in flux]
    rhoE = RHO * (T / (g - 1) + U ** 2 / 2 + QH * Y)
    q = [RHO, RHO * U, rhoE, RHO * Y]
    omega = -B * RHO * Y * sp.exp(-EA / T)
    flux = [RHO * U, RHO * U ** 2 + p, (rhoE + p) * U, RHO * U * Y]
    if pde == "reactive_ns":
        kappa = MU * g / ((g - 1) * PR)
        rhoD = MU / (PR * LE)
        tau = sp.Rational(4, 3) * MU * d(U)
        heat = -kappa * d(T) - QH * rhoD * d(Y)
        flux = [flux[0], flux[1] - tau, flux[2] - U * tau + heat, flux[3] - rhoD * d(Y)]
    rhs = [-d(f) for f in flux]
    rhs[3] += omega
    return q, rhs


def _alpha(scheme):
    return 0.0 if scheme == "weno5" else ALPHA     # WENO carries no diffusion term


def _problem(pde, scheme, n):
    nf = W.nfields(pde)
    return W.Problem(pde=pde, scheme=scheme, n=n, p=4, dt=1e-3, q0=np.zeros((nf, n)),
                     mode="sync", rk="rk4", c=C, alpha=_alpha(scheme), r=R, gamma=GAMMA, q=QH, ea=EA,
                     b=B, mu=MU, pr=PR, le=LE)


def _residual(pde, scheme, n):
    q, rhs = _exact(pde, _alpha(scheme))
    x = (np.arange(n) + 0.5) / n
    lam = [sp.lambdify(X, e, "numpy") for e in q]
    lrh = [sp.lambdify(X, e, "numpy") for e in rhs]
    state = np.stack([np.broadcast_to(f(x), (n,)) for f in lam]).astype(np.float64)
    want = np.stack([np.broadcast_to(f(x), (n,)) for f in lrh]).astype(np.float64)
    got = oracle.rhs_sync(_problem(pde, scheme, n), state)
    return np.abs(got - want).max(axis=1) / np.abs(want).max(axis=1)


CASES = [
    # pde, scheme, coarse N, expected order (lower bound used), max residual at 2N
    ("adv_diff", "fd2", 256, 2, 1e-3),
    ("adv_diff", "fd4", 256, 4, 1e-6),
    ("adr_logistic", "fd8", 128, 8, 1e-9),
    ("adr_logistic", "weno5", 256, 4, 1e-5),
    ("burgers", "weno5", 256, 4, 1e-5),
    ("euler", "weno5", 256, 4, 1e-5),
    ("reactive_euler", "weno5", 256, 4, 1e-5),
    ("reactive_ns", "fd4", 256, 4, 1e-6),
    ("reactive_ns", "fd8", 128, 8, 1e-9),
]


@pytest.mark.parametrize("pde,scheme,n,order,tol", CASES)
def test_rhs_converges_to_continuous_pde(pde, scheme, n, order, tol):
    e1 = _residual(pde, scheme, n)
    e2 = _residual(pde, scheme, 2 * n)
    assert np.all(e2 < tol), (pde, scheme, e1, e2)
    # observed order per field (skip fields already at rounding level)
    for a, b in zip(e1, e2):
        if b > 1e-12:
            assert np.log2(a / b) > order - 0.6, (pde, scheme, e1, e2)


def test_planted_sign_error_is_caught():
    """The residual measure separates a correct RHS from one with a flipped term:
    flip the sign of the heat-conduction contribution in the exact RHS and the
    residual stays O(1) under refinement."""
    q, rhs = _exact("reactive_ns")
    g = GAMMA
    kappa = MU * g / ((g - 1) * PR)
    wrong = rhs[2] - 2 * kappa * sp.diff(T, X, 2)
    n = 256
    x = (np.arange(n) + 0.5) / n
    state = np.stack([sp.lambdify(X, e, "numpy")(x) for e in q])
    got = oracle.rhs_sync(_problem("reactive_ns", "fd8", n), state)
    w = sp.lambdify(X, wrong, "numpy")(x)
    assert np.abs(got[2] - w).max() / np.abs(w).max() > 1e-3
