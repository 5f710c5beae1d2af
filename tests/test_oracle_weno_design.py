"""Pins of the AT-WENO stencil design and of the oracle's WENO interpolation form against
what Sec. 3 of the paper prints: the candidate interpolants (eqs. interpS, atS0, atS1,
stenF, recon), the ideal-weight sets (eqs. fullSten, idw, gammAT2, and the reconstruction
weights 1/10, 6/10, 3/10), the smoothness indicators (eqs. betaS, betaAT0-2), the
negative-weight splitting (eq. splitGam), and the statements the section makes about
them (a four-point full stencil skips u_{j+1} at zero delay and is fourth order; the
five-point stencil recovers the synchronous fifth-order interpolant).  The oracle's
construction (oracle/weno_design.py) solves Taylor constraints; the printed values are
typed here from the paper, so a wrong constraint, point or sign in the construction
fails one of them."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import weno_design as D

KS = (1, 2, 3, 4)


def test_interpolation_candidates_and_weights():
    # eq. interpS
    cands = D.candidate_set("sync", 0)
    assert [c for _, c in cands] == [[Fr(3, 8), Fr(-5, 4), Fr(15, 8)], [Fr(-1, 8), Fr(3, 4), Fr(3, 8)],
                                     [Fr(3, 8), Fr(3, 4), Fr(-1, 8)]]
    # ideal weights and the fifth-order five-point interpolant that follows
    g = D.family_weights("sync", 0)
    assert g == [Fr(1, 16), Fr(5, 8), Fr(5, 16)]
    full = D.combined(cands, g)
    assert [full[(Fr(x), Fr(0))] for x in range(-2, 3)] == [Fr(3, 128), Fr(-5, 32), Fr(45, 64), Fr(15, 32),
                                                           Fr(-5, 128)]
    assert D.truncation(list(full), list(full.values()), (5, 0)) != 0     # exactly fifth order


@pytest.mark.parametrize("k", KS)
def test_four_point_candidates(k):
    kk = Fr(k)
    (s0, c0), (s1, c1), _ = D.candidate_set("four0", k)
    # eq. atS0: {u_{j-2}^{n-k-1}, u_{j-2}^{n-k}, u_{j-1}^{n-k}, u_j^n}
    assert c0 == [Fr(7, 8) * kk, (3 - 7 * kk) / 8, Fr(-5, 4), Fr(15, 8)]
    # eq. atS1: {u_{j-1}^{n-k-1}, u_{j-1}^{n-k}, u_j^n, u_{j+1}^n}
    assert c1 == [kk / 8, (-kk - 1) / 8, Fr(3, 4), Fr(3, 8)]
    # leading truncation terms TE = exact - approximation (the paper's sign): the dt dx term
    # of atS0 depends on the delay (eq. teATS0: -5/4 k, and 5/16 dx^3), that of atS1 does not
    # (-1/16 dx^3 only)
    def te(s, c, term):
        return -D.truncation(s, c, term)
    assert te(s0, c0, (1, 1)) == Fr(-5, 4) * kk
    assert te(s0, c0, (3, 0)) == Fr(5, 16)
    assert te(s1, c1, (1, 1)) == 0
    assert te(s1, c1, (3, 0)) == Fr(-1, 16)


@pytest.mark.parametrize("k", KS)
def test_four_point_ideal_weights_are_not_convex(k):
    assert D.family_weights("four0", k) == [0, Fr(1, 2), Fr(1, 2)]
    assert D.family_weights("four1", k) == [Fr(-3, 2), Fr(-5, 2), 5]
    assert D.family_weights("four2", k) == [Fr(3, 8), Fr(5, 4), Fr(-5, 8)]     # eq. gammAT2


def test_four_point_stencil_at_zero_delay_skips_a_point():
    """With the weights of eq. gammAT2, the zero-delay full stencil uses only j-2, j-1, j,
    j+2 and is fourth order (its dx^4 term is not removed)."""
    cands = D.candidate_set("four2", 0)
    full = D.combined(cands, D.family_weights("four2", 0))
    nz = sorted(int(x) for (x, t), c in full.items() if c != 0)
    assert nz == [-2, -1, 0, 2]
    pts = list(full)
    assert D.truncation(pts, [full[p] for p in pts], (3, 0)) == 0
    assert D.truncation(pts, [full[p] for p in pts], (4, 0)) != 0


@pytest.mark.parametrize("k", KS)
def test_five_point_stencil(k):
    """eq. stenF: convex weights 1/16, 5/8, 5/16 (those of the synchronous stencils) and,
    at the delayed points, the synchronous coefficients applied to the two-level linear
    extrapolation (k + 1) u^{n-k} - k u^{n-k-1}."""
    kk = Fr(k)
    cands = D.candidate_set("five", k)
    (s0, c0), (s1, c1), (s2, c2) = cands
    # points: u_{j-2}^{n-k-1}, u_{j-2}^{n-k}, u_{j-1}^{n-k-1}, u_{j-1}^{n-k}, u_j^n
    assert c0 == [Fr(-3, 8) * kk, Fr(3, 8) * (kk + 1), Fr(5, 4) * kk, Fr(-5, 4) * (kk + 1), Fr(15, 8)]
    # points: u_{j-1}^{n-k-1}, u_{j-1}^{n-k}, u_j^{n-k}, u_j^n, u_{j+1}^n
    assert c1 == [kk / 8, (-kk - 1) / 8, 0, Fr(3, 4), Fr(3, 8)]
    assert c2 == [Fr(3, 8), Fr(3, 4), Fr(-1, 8)]
    assert D.family_weights("five", k) == [Fr(1, 16), Fr(5, 8), Fr(5, 16)]
    # the oracle's two-level extrapolation weights give the same coefficients
    w = oracle.extrap_weights(2, k)
    assert np.allclose(w, [k + 1, -k])
    assert float(c0[1]) == pytest.approx(3 / 8 * w[0]) and float(c0[0]) == pytest.approx(3 / 8 * w[1])


@pytest.mark.parametrize("k", (0, 1, 2, 3))
def test_reconstruction_candidates(k):
    """eq. recon (cell averages): coefficients for i = 0, 1, 2; at k = 0 the Jiang-Shu
    candidates, with ideal weights 1/10, 6/10, 3/10."""
    kk = Fr(k)
    for i in range(3):
        pts = [(Fr(i - 2), -kk - 1), (Fr(i - 2), -kk), (Fr(i - 1), -kk), (Fr(i), Fr(0))]
        c = D.stencil_coefficients(pts, D.TERMS_R2, average=True)
        assert c == [Fr(3 * i * i - 12 * i + 5, 6) * kk, Fr(-3 * i * i * k + 12 * i * k - 5 * k + 3 * i * i - 6 * i + 2, 6),
                     Fr(-6 * i * i + 18 * i - 7, 6), Fr(3 * i * i - 12 * i + 11, 6)]
    assert D.family_weights("sync", 0, average=True) == [Fr(1, 10), Fr(3, 5), Fr(3, 10)]


def _rand_vals(rng, n):
    return [Fr(int(x), int(d)) for x, d in zip(rng.integers(-20, 21, n), rng.integers(1, 7, n))]


def test_smoothness_indicators_synchronous():
    """eq. betaS (the printed quadratic forms) equals eq. bet1 evaluated for the candidate
    polynomials by Simpson's 3/8 rule."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b, c, d, e = _rand_vals(rng, 5)      # u_{j-2} .. u_{j+2}
        printed = [(4 * a * a + (11 * c - 19 * b) * a + 25 * b * b + 10 * c * c - 31 * b * c) / 3,
                   (4 * b * b + (5 * d - 13 * c) * b + 13 * c * c + 4 * d * d - 13 * c * d) / 3,
                   (10 * c * c + (11 * e - 31 * d) * c + 25 * d * d + 4 * e * e - 19 * d * e) / 3]
        vals = [[a, b, c], [b, c, d], [c, d, e]]
        got = [D.smoothness(p, v, D.TERMS_SYNC3) for p, v in zip(D.sync_candidates(), vals)]
        assert got == printed


@pytest.mark.parametrize("k", (1, 2, 3))
def test_smoothness_indicators_asynchronous(k):
    """eqs. betaAT0-2 (the four-point stencils of eq. gammAT2) from the candidates'
    space-time polynomials."""
    rng = np.random.default_rng(k)
    kk = Fr(k)
    stencils = D.four_point_candidates(k, 2)
    for _ in range(10):
        # A = u^{n-k} of the outer delayed point, B = its u^{n-k-1}, C the inner delayed
        # point at n-k, D the synchronous point, for each candidate (its own points)
        vals = [_rand_vals(rng, 4) for _ in range(3)]
        got = [D.smoothness(p, v, D.TERMS_R2) for p, v in zip(stencils, vals)]
        pr = []
        for (c2, c1a, c1b, c1c, c1d, c0), (B, A, C, Dv) in zip(
                [(10, -11, 4, 20, 31, (-19, 25, -31, 10)), (4, -5, 4, 8, 13, (-13, 13, -13, 4)),
                 (4, -11, 10, 8, 19, (-31, 25, -19, 4))], vals):
            p1, p2, p3, p4 = c0
            # the printed forms: (c2 k^2 + c1a k + c1b) A^2 + (-2 c2 k^2 B + k (-c1a B + c1d C - c1c D)
            #   + p1 C + (-c1a) D) A + c2 k^2 B^2 + p2 C^2 + p3 D C + k B (c1c D - c1d C) + p4 D^2
            pr.append(((c2 * kk ** 2 + c1a * kk + c1b) * A * A
                       + (-2 * c2 * kk ** 2 * B + kk * (-c1a * B + c1d * C - c1c * Dv) + p1 * C - c1a * Dv) * A
                       + c2 * kk ** 2 * B * B + p2 * C * C + p3 * Dv * C + kk * B * (c1c * Dv - c1d * C) + p4 * Dv * Dv) / 3)
        assert got == pr


def test_smoothness_indicators_asynchronous_reduce_at_zero_delay():
    rng = np.random.default_rng(7)
    for _ in range(10):
        B, A, C, Dv = _rand_vals(rng, 4)
        s4 = D.four_point_candidates(0, 2)[0]          # the older level of u_{j-2} is unused
        s3 = D.sync_candidates()[0]
        assert D.smoothness(s4, [B, A, C, Dv], D.TERMS_R2) == D.smoothness(s3, [A, C, Dv], D.TERMS_SYNC3)


def test_smoothness_indicators_asynchronous_printed_beta0():
    """eq. betaAT0 typed term by term as printed (k = 2)."""
    k = Fr(2)
    A, B, C, Dv = Fr(3, 2), Fr(-1, 3), Fr(5, 4), Fr(2, 7)    # A = u_{j-2}^{n-k}, B = u_{j-2}^{n-k-1}, C = u_{j-1}^{n-k}, D = u_j^n
    printed = ((10 * k * k - 11 * k + 4) * A * A
               + (-20 * k * k * B + k * (11 * B + 31 * C - 20 * Dv) - 19 * C + 11 * Dv) * A
               + 10 * k * k * B * B + 25 * C * C - 31 * Dv * C + k * B * (20 * Dv - 31 * C) + 10 * Dv * Dv) / 3
    s0 = D.four_point_candidates(2, 2)[0]
    assert D.smoothness(s0, [B, A, C, Dv], D.TERMS_R2) == printed


@pytest.mark.parametrize("kind", ["four1", "four2"])
def test_negative_weight_splitting(kind):
    g = D.family_weights(kind, 1)
    gp, gm, sp, sm = D.split_weights(g, theta=3)
    assert all(x >= 0 for x in gp + gm)
    assert sum(gp) == 1 and sum(gm) == 1 and sp - sm == 1
    assert [sp * a - sm * b for a, b in zip(gp, gm)] == g


def test_non_convex_weights_need_splitting():
    """The motivation of Sec. 3 for the convex five-point stencil: the weights of eq.
    gammAT2 put straight into eq. omg can make the normalising sum vanish (values without
    bound on ordinary data); split (eq. fullSplit) they stay bounded; the five-point
    family needs no splitting."""
    rng = np.random.default_rng(0)
    cands4 = D.candidate_set("four2", 1)
    g4 = D.family_weights("four2", 1)
    cands5 = D.candidate_set("five", 1)
    g5 = D.family_weights("five", 1)
    worst_raw = worst_split = worst_five = 0.0
    for _ in range(2000):
        pts = {}
        for p, _ in cands4 + cands5:
            for pt in p:
                pts.setdefault(pt, Fr(float(rng.normal())).limit_denominator(10 ** 6))
        span = max(pts.values()) - min(pts.values())
        v4 = [[pts[pt] for pt in p] for p, _ in cands4]
        betas = [float(D.smoothness(p, v, D.TERMS_R2 if len(p) == 4 else D.TERMS_SYNC3)) for (p, _), v in zip(cands4, v4)]
        cv = [sum(float(c) * float(x) for c, x in zip(cc, v)) for (p, cc), v in zip(cands4, v4)]
        a = [float(gi) / (1e-6 + b) ** 2 for gi, b in zip(g4, betas)]
        raw = sum(x * y for x, y in zip(a, cv)) / sum(a)
        split = D.weno_value(cands4, v4, g4, 1e-6, betas)
        five = D.weno_value(cands5, [[pts[pt] for pt in p] for p, _ in cands5], g5, 1e-6)
        worst_raw = max(worst_raw, abs(raw) / float(span))
        worst_split = max(worst_split, abs(split) / float(span))
        worst_five = max(worst_five, abs(five) / float(span))
    assert worst_raw > 100.0
    assert worst_split < 3.0 and worst_five < 3.0


# ---- the oracle's WENO interpolation form (C) ----------------------------------------
def test_oracle_interpolation_linear_limit_and_betas():
    """With eps far above every beta the weights are the ideal ones, so the oracle's value
    is the printed five-point interpolant; its betas are eq. bet1's."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = rng.normal(size=5)
        val, beta = oracle.weno_interp(1e30, v)
        assert val == pytest.approx(np.dot([3 / 128, -5 / 32, 45 / 64, 15 / 32, -5 / 128], v), rel=1e-13, abs=1e-14)
        vf = [Fr(float(x)) for x in v]
        want = [float(D.smoothness(p, vals, D.TERMS_SYNC3))
                for p, vals in zip(D.sync_candidates(), [vf[0:3], vf[1:4], vf[2:5]])]
        assert np.allclose(beta, want, rtol=1e-12, atol=1e-13)


def test_oracle_interpolation_is_essentially_non_oscillatory():
    """A jump between v3 and v4: the weight of the one candidate that avoids it (stencil
    {j-2, j-1, j}) tends to 1, so the value is that candidate's interpolant."""
    v = np.array([0.1, 0.2, 0.3, 5.0, 5.1])
    val, _ = oracle.weno_interp(1e-12, v)
    assert val == pytest.approx(3 / 8 * 0.1 - 5 / 4 * 0.2 + 15 / 8 * 0.3, abs=1e-3)


def test_oracle_interpolation_order():
    """Interpolation of a smooth function half a cell right of j: fifth order."""
    errs = []
    hs = [0.1 / 2 ** i for i in range(5)]
    for h in hs:
        x = 0.3 + h * np.arange(-2, 3)
        val, _ = oracle.weno_interp(1e-40, np.sin(x))
        errs.append(abs(val - math.sin(0.3 + 0.5 * h)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders[1:]) > 4.7, orders
