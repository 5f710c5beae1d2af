"""Pins of the oracle's chain-rule form of the reacting Navier-Stokes right-hand side (Sec.
4 after eq. convEq: the derivatives of the convective products expanded by the chain rule
into derivatives of the primitives, so that the AT halo carries primitives; Sec. 6 on the
memory-compute trade-off against differentiating the fluxes themselves).

* Both forms converge to the exact right-hand side of smooth periodic fields at the
  order of the interior stencil (derivatives of the closed-form fields; a dropped or
  wrong chain-rule term leaves an O(1) error).
* The forms are different discretisations: the flux form telescopes on a periodic
  domain (all sums conserved to rounding); the chain-rule form keeps mass (skew
  symmetry of the central stencil) but not momentum.
* AT keeps the synchronous accuracy in both forms.
"""
import math

import numpy as np
import pytest

import at_workloads as W
import oracle

GAMMA, QH, EA, B, MU, PR, LE = 1.4, 5.0, 8.0, 3.0, 2e-3, 0.72, 1.0


def _fields(x):
    """Smooth periodic primitives and their first and second derivatives (closed form)."""
    tp = 2 * math.pi
    rho = 1.0 + 0.2 * np.sin(tp * x)
    rx = 0.2 * tp * np.cos(tp * x)
    u = 0.3 * np.cos(tp * x)
    ux = -0.3 * tp * np.sin(tp * x)
    uxx = -0.3 * tp * tp * np.cos(tp * x)
    T = 1.5 + 0.4 * np.sin(2 * tp * x)
    Tx = 0.4 * 2 * tp * np.cos(2 * tp * x)
    Txx = -0.4 * (2 * tp) ** 2 * np.sin(2 * tp * x)
    Y = 0.5 + 0.3 * np.cos(tp * x + 0.3)
    Yx = -0.3 * tp * np.sin(tp * x + 0.3)
    Yxx = -0.3 * tp * tp * np.cos(tp * x + 0.3)
    return rho, rx, u, ux, uxx, T, Tx, Txx, Y, Yx, Yxx


def _exact_rhs(x):
    """The right-hand side of the one-step-chemistry NS equations for the closed-form
    fields: -(C)_x + viscous terms + source, C = (rho u, rho u^2 + p, u (rho E + p),
    rho u Y), p = rho T, rho E = p/(gamma-1) + rho u^2/2 + q rho Y."""
    rho, rx, u, ux, uxx, T, Tx, Txx, Y, Yx, Yxx = _fields(x)
    p, px = rho * T, rx * T + rho * Tx
    rE = p / (GAMMA - 1) + 0.5 * rho * u * u + QH * rho * Y
    rEx = px / (GAMMA - 1) + 0.5 * (rx * u * u + 2 * rho * u * ux) + QH * (rx * Y + rho * Yx)
    kappa = MU * GAMMA / ((GAMMA - 1) * PR)
    rhoD = MU / (PR * LE)
    K = np.empty((4, x.size))
    K[0] = -(rx * u + rho * ux)
    K[1] = -(rx * u * u + 2 * rho * u * ux + px) + 4 / 3 * MU * uxx
    K[2] = -(ux * (rE + p) + u * (rEx + px)) + 4 / 3 * MU * (ux * ux + u * uxx) + kappa * Txx + QH * rhoD * Yxx
    K[3] = -(rx * u * Y + rho * ux * Y + rho * u * Yx) + rhoD * Yxx - B * rho * Y * np.exp(-EA / T)
    return K


def _problem(n, form, scheme="fd8", p=8, mode="sync", kmax=2, steps=10):
    x = (np.arange(n) + 0.5) / n
    rho, _, u, _, _, T, _, _, Y, _, _ = _fields(x)
    q0 = W.reactive_conserved(rho, u, T, Y, GAMMA, QH)
    return W.Problem(pde="reactive_ns", scheme=scheme, n=n, p=p, dt=0.05 / n, q0=q0, mode=mode, rk="rk4",
                     kmax=kmax, gamma=GAMMA, q=QH, ea=EA, b=B, mu=MU, pr=PR, le=LE, steps=steps, form=form)


@pytest.mark.parametrize("scheme,expect", [("fd4", 4), ("fd8", 8)])
def test_both_forms_converge_to_the_exact_rhs(scheme, expect):
    errs = {"flux": [], "chain": []}
    ns = (32, 64, 128) if scheme == "fd8" else (64, 128, 256)
    for n in ns:
        x = (np.arange(n) + 0.5) / n
        ex = _exact_rhs(x)
        for form in errs:
            pr = _problem(n, form, scheme)
            errs[form].append(np.abs(oracle.rhs_sync(pr, pr.q0) - ex).max())
    for form, e in errs.items():
        o = math.log2(e[-2] / e[-1])
        assert expect - 0.5 < o < expect + 1.5, (form, e)
    # different discretisations of the same operator
    assert errs["chain"][-1] != errs["flux"][-1]


def test_planted_chain_rule_error_is_caught():
    """The exact-RHS comparison detects a dropped term: the rho_x u Y term of the species
    flux, written into the expected values, leaves an O(1) mismatch."""
    n = 128
    x = (np.arange(n) + 0.5) / n
    ex = _exact_rhs(x)
    rho, rx, u, ux, uxx, T, Tx, Txx, Y, Yx, Yxx = _fields(x)
    wrong = ex.copy()
    wrong[3] += rx * u * Y                      # as if the term were missing
    got = oracle.rhs_sync(_problem(n, "chain"), _problem(n, "chain").q0)
    assert np.abs(got - ex).max() < 1e-6
    assert np.abs(got - wrong).max() > 0.1


def test_momentum_telescopes_in_the_flux_form_only():
    """The flux form's differences telescope on a periodic domain (sums conserved to
    rounding).  In the chain-rule form, mass still is conserved (with an antisymmetric
    central stencil, sum_j (D rho)_j u_j = -sum_j rho_j (D u)_j), but momentum is not:
    D(u^2) differs from 2 u D(u) by the truncation error."""
    n = 128
    drift = {}
    for form in ("flux", "chain"):
        pr = _problem(n, form, steps=200)
        q = oracle.run(pr)
        drift[form] = [abs(q[f].sum() - pr.q0[f].sum()) / np.abs(pr.q0[f]).sum() for f in range(2)]
    assert drift["flux"][0] < 1e-14 and drift["chain"][0] < 1e-14, drift
    assert drift["flux"][1] < 1e-15, drift
    assert drift["chain"][1] > 1e4 * max(drift["flux"][1], 1e-17), drift


def test_at_keeps_the_synchronous_accuracy_in_both_forms():
    """Flame workload: in both forms the AT run stays close to the synchronous one (far
    closer than AS), by nearly the same amount."""
    base = W.reactive_ns_c2(n=512, p=8, kmax=2, steps=100)
    q = {}
    for form in ("flux", "chain"):
        for mode in ("sync", "at", "as"):
            q[form, mode] = oracle.run(base.replace(form=form, mode=mode))
    scale = np.abs(q["flux", "sync"]).max(axis=1)

    def dev(form, mode):
        return (np.abs(q[form, mode] - q[form, "sync"]).max(axis=1) / scale).max()
    for form in ("flux", "chain"):
        assert dev(form, "at") < 0.01 * dev(form, "as"), form
    assert abs(dev("chain", "at") - dev("flux", "at")) < 0.2 * dev("flux", "at")
    assert (np.abs(q["chain", "sync"] - q["flux", "sync"]).max(axis=1) / scale).max() > 0
