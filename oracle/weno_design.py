"""Construction of AT-WENO candidate stencils, ideal weights and smoothness indicators
from Taylor-series constraints, in exact rational arithmetic (Sec. 3 of Kumari et al.,
arXiv:2204.01133: the interpolation form, eqs. interpS, fullSten, omg, betaS, the
four-point stochastic stencils of eqs. atS0, atS1, the ideal-weight sets of eq. idw and
eq. gammAT2, the negative-weight splitting of eq. splitGam, the smoothness indicators of
eqs. bet1, beta, betaAT0-2, the five-point stencil of eq. stenF and the reconstruction
form of eq. recon).

TEST INFRASTRUCTURE ONLY (part of the oracle): the product path never imports it.

Conventions.  A stencil point is (x, t): x in grid spacings relative to point j, t in
time steps relative to level n (a delayed level n - k is t = -k).  The approximated
value is u at (x*, 0), x* = 1/2 (the edge j + 1/2).  A Taylor term (p, q) is the
coefficient of dx^p dt^q d^p/dx^p d^q/dt^q u / (p! q!); a linear approximation
sum_m c_m u(x_m, t_m) matches term (p, q) when sum_m c_m (x_m - x*)^p t_m^q = [p = q = 0]
(for cell averages, the p-th power is averaged over the cell of x_m).  The delay scaling
dt ~ dx^r decides which terms are low order: r = 2 gives {1, dt, dx, dx^2} for third order.
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial
from typing import Dict, List, Sequence, Tuple

Point = Tuple[Fraction, Fraction]
Term = Tuple[int, int]

HALF = Fraction(1, 2)
# third order under dt ~ dx^2 (Sec. 3): the terms 1, dt, dx, dx^2
TERMS_R2 = ((0, 0), (0, 1), (1, 0), (2, 0))
# the five-point stencil of eq. stenF also removes the dt dx term
TERMS_R2_DTDX = ((0, 0), (0, 1), (1, 0), (2, 0), (1, 1))
TERMS_SYNC3 = ((0, 0), (1, 0), (2, 0))


def _frac(v) -> Fraction:
    return v if isinstance(v, Fraction) else Fraction(v)


def solve(A: List[List[Fraction]], rhs: List[Fraction]) -> List[Fraction]:
    """Exact solution of a square linear system (Gauss-Jordan with pivot search)."""
    n = len(A)
    M = [list(map(_frac, row)) + [_frac(rhs[i])] for i, row in enumerate(A)]
    for c in range(n):
        piv = next((r for r in range(c, n) if M[r][c] != 0), None)
        if piv is None:
            raise ValueError("singular constraint system")
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def moment(x, t, p: int, q: int, target=HALF, average: bool = False) -> Fraction:
    """Taylor weight of term (p, q) for a point at (x, t): (x - x*)^p t^q / (p! q!), the
    x-power averaged over the cell [x - 1/2, x + 1/2] for a cell average."""
    x, t = _frac(x), _frac(t)
    if average:
        lo, hi = x - HALF - target, x + HALF - target
        xp = (hi ** (p + 1) - lo ** (p + 1)) / (p + 1)
    else:
        xp = (x - target) ** p
    return xp * t ** q / (factorial(p) * factorial(q))


def stencil_coefficients(points: Sequence[Point], terms: Sequence[Term], target=HALF,
                         average: bool = False) -> List[Fraction]:
    """Coefficients c_m of the approximation of u(x*, 0) that matches the given terms
    (as many terms as points)."""
    if len(points) != len(terms):
        raise ValueError("the constraints must be as many as the points")
    A = [[moment(x, t, p, q, target, average) for (x, t) in points] for (p, q) in terms]
    rhs = [Fraction(1) if (p, q) == (0, 0) else Fraction(0) for (p, q) in terms]
    return solve(A, rhs)


def truncation(points: Sequence[Point], coeffs: Sequence[Fraction], term: Term, target=HALF,
               average: bool = False) -> Fraction:
    """Coefficient of Taylor term `term` in the error of sum_m c_m u(x_m, t_m) - u(x*, 0)."""
    p, q = term
    s = sum(_frac(c) * moment(x, t, p, q, target, average) for c, (x, t) in zip(coeffs, points))
    return s - (1 if (p, q) == (0, 0) else 0)


def ideal_weights(candidates: Sequence[Tuple[Sequence[Point], Sequence[Fraction]]],
                  removed: Sequence[Term], target=HALF, average: bool = False) -> List[Fraction]:
    """Ideal (linear) weights gamma_i of the candidate approximations (eq. idw): they sum
    to one and remove the given further truncation terms of the combination."""
    A = [[Fraction(1)] * len(candidates)]
    A += [[truncation(pts, c, term, target, average) for pts, c in candidates] for term in removed]
    return solve(A, [Fraction(1)] + [Fraction(0)] * len(removed))


def combined(candidates, gammas) -> Dict[Point, Fraction]:
    """The full stencil sum_i gamma_i (candidate i): coefficient per point."""
    out: Dict[Point, Fraction] = {}
    for (pts, c), g in zip(candidates, gammas):
        for pt, cm in zip(pts, c):
            key = (_frac(pt[0]), _frac(pt[1]))
            out[key] = out.get(key, Fraction(0)) + g * cm
    return out


def split_weights(gammas: Sequence[Fraction], theta=3):
    """Negative-weight splitting (eq. splitGam, after Shi, Hu & Shu): gamma~+ = (gamma +
    theta |gamma|) / 2, gamma~- = gamma~+ - gamma, sigma+- = sum gamma~+-, gamma+- =
    gamma~+- / sigma+- (reading: each sign normalised by its own sum; the printed index
    of sigma and numerator of gamma-+ are garbled).  Returns (gamma+, gamma-, sigma+,
    sigma-); gamma = sigma+ gamma+ - sigma- gamma-."""
    theta = _frac(theta)
    gp = [(_frac(g) + theta * abs(_frac(g))) / 2 for g in gammas]
    gm = [a - _frac(g) for a, g in zip(gp, gammas)]
    sp, sm = sum(gp), sum(gm)
    return [a / sp for a in gp], [a / sm for a in gm], sp, sm


# Simpson's 3/8 rule on the cell [x_j - 1/2, x_j + 1/2] (eq. beta; reading: nodes -1/2,
# -1/6, 1/6, 1/2 with weights 1, 3, 3, 1 over 8, exact for the cubic integrands here)
SIMPSON38 = ((Fraction(-1, 2), Fraction(1, 8)), (Fraction(-1, 6), Fraction(3, 8)),
             (Fraction(1, 6), Fraction(3, 8)), (Fraction(1, 2), Fraction(1, 8)))


def fit_polynomial(points: Sequence[Point], values: Sequence, terms: Sequence[Term]) -> Dict[Term, Fraction]:
    """The space-time polynomial sum_(p,q) a_pq x^p t^q (x relative to point j) through
    the stencil's values."""
    A = [[_frac(x) ** p * _frac(t) ** q for (p, q) in terms] for (x, t) in points]
    return dict(zip(terms, solve(A, list(values))))


def smoothness(points: Sequence[Point], values: Sequence, terms: Sequence[Term], order: int = 2) -> Fraction:
    """Smoothness indicator of a candidate (eq. bet1 with dx = 1): sum over l = 1..order of
    the integral over cell j of (d^l/dx^l P)^2 at t = 0, P the candidate's polynomial,
    integrated by Simpson's 3/8 rule (eq. beta)."""
    a = fit_polynomial(points, values, terms)

    def deriv(l: int, x: Fraction) -> Fraction:
        s = Fraction(0)
        for (p, q), c in a.items():
            if q == 0 and p >= l:
                s += c * Fraction(factorial(p), factorial(p - l)) * x ** (p - l)
        return s

    return sum(w * sum(deriv(l, x) ** 2 for l in range(1, order + 1)) for x, w in SIMPSON38)


# ---- the candidate stencils of Sec. 3 (left PE boundary at point j, delay k) ----------
def sync_candidates() -> List[List[Point]]:
    """S(0..2) = {j-2, j-1, j}, {j-1, j, j+1}, {j, j+1, j+2} at level n (eq. interpS)."""
    return [[(Fraction(i - 2 + m), Fraction(0)) for m in range(3)] for i in range(3)]


def four_point_candidates(k, variant: int) -> List[List[Point]]:
    """The four-point stochastic stencils of Sec. 3 for delay k: variant 0 is eqs. atS0,
    atS1 with S(2) synchronous (ideal weights 0, 1/2, 1/2); variant 1 moves u_j of S(1)
    to the delayed level (-3/2, -5/2, 5); variant 2 gives S(2) the same structure
    (eq. gammAT2: 3/8, 5/4, -5/8)."""
    k = _frac(k)
    s0 = [(Fraction(-2), -k - 1), (Fraction(-2), -k), (Fraction(-1), -k), (Fraction(0), Fraction(0))]
    if variant == 0:
        s1 = [(Fraction(-1), -k - 1), (Fraction(-1), -k), (Fraction(0), Fraction(0)), (Fraction(1), Fraction(0))]
    else:
        s1 = [(Fraction(-1), -k - 1), (Fraction(-1), -k), (Fraction(0), -k), (Fraction(1), Fraction(0))]
    if variant == 2:
        s2 = [(Fraction(0), -k - 1), (Fraction(0), -k), (Fraction(1), -k), (Fraction(2), Fraction(0))]
    else:
        s2 = [(Fraction(0), Fraction(0)), (Fraction(1), Fraction(0)), (Fraction(2), Fraction(0))]
    return [s0, s1, s2]


def five_point_candidates(k) -> List[List[Point]]:
    """The stencil of eq. stenF: both levels n-k, n-k-1 at the delayed points of S(0) and
    S(1) (the latter also u_j at n-k), S(2) synchronous."""
    k = _frac(k)
    s0 = [(Fraction(-2), -k - 1), (Fraction(-2), -k), (Fraction(-1), -k - 1), (Fraction(-1), -k),
          (Fraction(0), Fraction(0))]
    s1 = [(Fraction(-1), -k - 1), (Fraction(-1), -k), (Fraction(0), -k), (Fraction(0), Fraction(0)),
          (Fraction(1), Fraction(0))]
    s2 = [(Fraction(0), Fraction(0)), (Fraction(1), Fraction(0)), (Fraction(2), Fraction(0))]
    return [s0, s1, s2]


def terms_for(points: Sequence[Point], five_point: bool = False) -> Sequence[Term]:
    if len(points) == 3:
        return TERMS_SYNC3
    return TERMS_R2_DTDX if five_point else TERMS_R2


def candidate_set(kind: str, k, average: bool = False):
    """[(points, coefficients)] of a candidate family: "sync", "four0", "four1", "four2",
    "five" (interpolation unless average: cell-average reconstruction, eq. recon)."""
    if kind == "sync":
        stencils, five = sync_candidates(), False
    elif kind.startswith("four"):
        stencils, five = four_point_candidates(k, int(kind[-1])), False
    elif kind == "five":
        stencils, five = five_point_candidates(k), True
    else:
        raise ValueError(kind)
    return [(s, stencil_coefficients(s, terms_for(s, five), average=average)) for s in stencils]


def family_weights(kind: str, k, average: bool = False) -> List[Fraction]:
    """Ideal weights of a candidate family.  Four-point families: the dt dx and dx^3 terms
    of the combination removed (a fourth-order full stencil); these weights do not depend
    on the delay, and at k = 0 (where the dt dx terms vanish) the family keeps the weights
    of k = 1, as the paper applies them.  Synchronous and five-point families (no dt dx
    term in any candidate): dx^3 and dx^4 removed (fifth order at k = 0)."""
    if kind.startswith("four"):
        cands = candidate_set(kind, max(_frac(k), Fraction(1)), average)
        return ideal_weights(cands, [(1, 1), (3, 0)], average=average)
    return ideal_weights(candidate_set(kind, k, average), [(3, 0), (4, 0)], average=average)


def weno_value(candidates, values_per_candidate, gammas, eps, betas=None, theta=3) -> float:
    """Nonlinear WENO combination (eq. omg) of the candidate values with ideal weights
    gammas; with a negative ideal weight, the split form of eq. fullSplit (weights of
    each sign normalised separately, recombined as sigma+ u+ - sigma- u-).  betas: the
    candidates' smoothness indicators (default: from the stencils, eq. bet1)."""
    vals = []
    for (pts, c), v in zip(candidates, values_per_candidate):
        vals.append(sum(float(cm) * float(x) for cm, x in zip(c, v)))
    if betas is None:
        betas = [float(smoothness(pts, [_frac(x) for x in v], terms_for(pts, len(pts) == 5)))
                 for (pts, _), v in zip(candidates, values_per_candidate)]
    g = [float(x) for x in gammas]
    if min(g) >= 0:
        a = [gi / (eps + b) ** 2 for gi, b in zip(g, betas)]
        return sum(ai * vi for ai, vi in zip(a, vals)) / sum(a)
    gp, gm, sp, sm = split_weights([_frac(x) for x in gammas], theta)
    ap = [float(x) / (eps + b) ** 2 for x, b in zip(gp, betas)]
    am = [float(x) / (eps + b) ** 2 for x, b in zip(gm, betas)]
    up = sum(a * v for a, v in zip(ap, vals)) / sum(ap)
    um = sum(a * v for a, v in zip(am, vals)) / sum(am)
    return float(sp) * up - float(sm) * um
