"""Pin of the local Lax-Friedrichs wave speed of the WENO flux (Sec. 3, eq. Csplit).

At a jump between two constant states, each with at least three points on either
side of the interface, the WENO5 reconstruction of each split flux puts all but a
(eps / beta)^2 ~ 1e-12 share of its weight on the candidate stencil that lies
entirely on its upwind side.  The interface flux of the method then reduces to the
textbook Rusanov flux (Toro, Riemann Solvers and Numerical Methods for Fluid
Dynamics, Sec. 10.5.1):

    F = (C(q_L) + C(q_R)) / 2 - alpha (q_R - q_L) / 2,
    alpha = max(|u_L| + c_L, |u_R| + c_R),  c = sqrt(gamma p / rho).

A periodic slab has two such jumps, one with each state on the left, so an alpha
taken from one point of the interface fails at one of them; a sound speed without
gamma fails at both.  The flux and sound speed below are the textbook Euler ones,
written from the primitive variables; the test plants both mistakes in copies of
the oracle and shows that the pin catches each.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import at_workloads as W
import oracle

GAMMA = 1.4
N = 16
SLAB = slice(4, 12)          # state A on points 4..11, state B on the others


def _slab(a, b):
    """(F, N) array: column a on the slab, b elsewhere."""
    out = np.repeat(np.asarray(b, float)[:, None], N, axis=1)
    out[:, SLAB] = np.asarray(a, float)[:, None]
    return out


def _euler_case():
    # primitives (rho, u, p) of the two states: every conserved field jumps
    A = (1.0, 0.35, 2.0)
    B = (0.2, -0.6, 0.1)
    q0 = _slab(W.euler_conserved(*A, GAMMA), W.euler_conserved(*B, GAMMA))

    def flux_and_speed(rho, u, p):
        E = p / (GAMMA - 1.0) + 0.5 * rho * u * u
        C = np.array([rho * u, rho * u * u + p, u * (E + p)])
        return C, abs(u) + np.sqrt(GAMMA * p / rho)

    pr = W.Problem(pde="euler", scheme="weno5", n=N, p=1, dt=1e-6, q0=q0, mode="at", rk="fe", kmax=0,
                   gamma=GAMMA)
    return pr, A, B, flux_and_speed, lambda rho, u, p: W.euler_conserved(rho, u, p, GAMMA)


def _reactive_case():
    q = 2.0
    # primitives (rho, u, p, Y); temperature T = p / rho (R = 1)
    A = (1.0, 0.35, 2.0, 0.05)
    B = (0.2, -0.6, 0.1, 0.9)

    def cons(rho, u, p, Y):
        return W.reactive_conserved(rho, u, p / rho, Y, GAMMA, q)

    def flux_and_speed(rho, u, p, Y):
        E = p / (rho * (GAMMA - 1.0)) + 0.5 * u * u + q * Y        # total energy per mass
        C = np.array([rho * u, rho * u * u + p, u * (rho * E + p), rho * Y * u])
        return C, abs(u) + np.sqrt(GAMMA * p / rho)

    q0 = _slab(cons(*A), cons(*B))
    pr = W.Problem(pde="reactive_euler", scheme="weno5", n=N, p=1, dt=1e-6, q0=q0, mode="at", rk="fe",
                   kmax=0, gamma=GAMMA, q=q, ea=20.0, b=0.0)
    return pr, A, B, flux_and_speed, cons


def _burgers_case():
    A, B = (0.3,), (-1.2,)

    def flux_and_speed(u):
        return np.array([0.5 * u * u]), abs(u)

    pr = W.Problem(pde="burgers", scheme="weno5", n=N, p=1, dt=1e-6, q0=_slab(A, B), mode="at", rk="fe",
                   kmax=0)
    return pr, A, B, flux_and_speed, lambda u: np.array([u])


CASES = {"euler": _euler_case, "reactive_euler": _reactive_case, "burgers": _burgers_case}


def _rusanov(flux_and_speed, cons, left, right):
    CL, sL = flux_and_speed(*left)
    CR, sR = flux_and_speed(*right)
    alpha = max(sL, sR)
    return 0.5 * (CL + CR) - 0.5 * alpha * (np.asarray(cons(*right)) - np.asarray(cons(*left)))


def _pin_error(make):
    """Largest deviation of the oracle's two jump fluxes from Rusanov's, relative to the
    flux scale."""
    pr, A, B, fs, cons = make()
    with oracle.Oracle(pr) as o:
        o.step(1)                  # forward Euler: the one right-hand side is that of q0
        fl = o.fluxes(0)           # interface ii lies between own points ii-1 and ii
    want_ba = _rusanov(fs, cons, B, A)      # interface 3 | 4
    want_ab = _rusanov(fs, cons, A, B)      # interface 11 | 12
    scale = max(np.abs(want_ab).max(), np.abs(want_ba).max())
    return max(np.abs(fl[SLAB.start] - want_ba).max(), np.abs(fl[SLAB.stop] - want_ab).max()) / scale


@pytest.mark.parametrize("name", sorted(CASES))
def test_jump_flux_is_rusanov(name):
    # what remains is the weight the WENO weights leave on the candidates that cross the
    # jump, about (eps / beta)^2 of the split flux's jump: 1e-12 to 1e-9 of the flux scale
    # for these states (the smallest split-flux jump, in rho Y, sets the largest)
    assert _pin_error(CASES[name]) < 1e-8


# mistakes planted in copies of the oracle: (text in at_oracle.c, replacement)
PLANTED = {
    "sound_speed_without_gamma": [("sqrt(pb->gamma * p / q[0])", "sqrt(p / q[0])"),
                                  ("sqrt(pb->gamma * T)", "sqrt(T)")],
    "alpha_from_left_point": [("double al = lam[i] > lam[i + 1] ? lam[i] : lam[i + 1];",
                               "double al = lam[i];")],
    "alpha_from_right_point": [("double al = lam[i] > lam[i + 1] ? lam[i] : lam[i + 1];",
                                "double al = lam[i + 1];")],
}


@pytest.fixture
def planted(tmp_path, monkeypatch):
    src_dir = os.path.dirname(oracle._SRC)

    def build(name):
        text = open(oracle._SRC).read()
        for old, new in PLANTED[name]:
            assert text.count(old) == 1, old
            text = text.replace(old, new)
        d = tmp_path / name
        d.mkdir()
        (d / "at_oracle.c").write_text(text)
        shutil.copy(os.path.join(src_dir, "at_oracle.h"), d / "at_oracle.h")
        lib = str(d / "liboracle.so")
        subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", lib,
                        str(d / "at_oracle.c"), "-lm"], check=True)
        monkeypatch.setattr(oracle, "_lib", oracle.load(lib))
    return build


@pytest.mark.parametrize("mistake", sorted(PLANTED))
def test_planted_wave_speed_mistakes_are_caught(planted, mistake):
    planted(mistake)
    worst = max(_pin_error(CASES[n]) for n in ("euler", "reactive_euler"))
    assert worst > 1e-3, (mistake, worst)
