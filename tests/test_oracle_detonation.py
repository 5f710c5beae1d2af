"""Pin of the oracle's reacting Euler composition over many steps (Sec. 4, eq. ge with
one-step chemistry; the AT-WENO5 scheme of Sec. 3): a detonation started by a
high-pressure driver settles to the Chapman-Jouguet speed, which depends only on the
heat release, gamma and the state ahead (not on the kinetics):

    D_CJ = sqrt(c0^2 + (gamma^2 - 1) q / 2) + sqrt((gamma^2 - 1) q / 2),  c0^2 = gamma p0 / rho0.

The front (the first unburnt point ahead of the driver) is tracked between two times
after the start-up: 0.983 D_CJ with and without delays, 0.976 D_CJ in the WENO
interpolation form (N 512; one grid point over the interval is 0.7 % of D_CJ).  Copies
of the oracle with a plausible thermodynamic mistake (the flux pressure without the
chemical energy: 0.67 D_CJ; the energy flux without the pressure work: 0.73 D_CJ) fail.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import at_workloads as W
import oracle

GAMMA, QH, EA, B = 1.4, 50.0, 10.0, 2000.0
D_CJ = math.sqrt(GAMMA + (GAMMA ** 2 - 1) * QH / 2) + math.sqrt((GAMMA ** 2 - 1) * QH / 2)


def _problem(n, mode="sync", kmax=0, scheme="weno5"):
    """Unit periodic tube at rest (rho = p = T = 1, Y = 1) with a driver at x < 0.02 (p 84,
    burnt); the driver also sends a detonation to the left, which wraps round, so the
    right-running front is followed until it has crossed less than half the tube."""
    x = (np.arange(n) + 0.5) / n
    driver = x < 0.02
    rho = np.ones(n)
    p = np.where(driver, 4.0 * (1.0 + (GAMMA - 1.0) * QH), 1.0)
    Y = np.where(driver, 0.0, 1.0)
    q0 = W.reactive_conserved(rho, np.zeros(n), p / rho, Y, GAMMA, QH)
    dt = 0.4 / n / 16.0
    return W.Problem(pde="reactive_euler", scheme=scheme, n=n, p=8, dt=dt, q0=q0, mode=mode, rk="ssprk3",
                     kmax=kmax, gamma=GAMMA, q=QH, ea=EA, b=B, steps=10)


def front_speed(pr, t1=0.015, t2=0.045, run=None):
    """Speed of the right-running front between t1 and t2 (None if there is no front:
    the gas ahead has burnt everywhere).  run: (step(k), state()) of another solver of
    the same problem (default: the oracle)."""
    if run is None:
        o = oracle.Oracle(pr)
        run = (o.step, o.state)
    step, state = run
    pos, t = [], 0.0
    for ts in (t1, t2):
        k = int(round((ts - t) / pr.dt))
        step(k)
        t += k * pr.dt
        q = state()
        Y = q[3] / q[0]
        i0 = int(0.02 * pr.n) + 1
        ahead = np.nonzero(Y[i0:] > 0.5)[0]
        if ahead.size == 0:
            return None
        pos.append((i0 + ahead.min()) / pr.n)
    return (pos[1] - pos[0]) / (t2 - t1)


@pytest.mark.parametrize("mode,kmax", [("sync", 0), ("at", 4)])
def test_detonation_runs_at_the_chapman_jouguet_speed(mode, kmax):
    d = front_speed(_problem(512, mode, kmax))
    assert abs(d / D_CJ - 1.0) < 0.03, (d, D_CJ)


def test_interpolation_form_runs_at_the_chapman_jouguet_speed():
    d = front_speed(_problem(512, "at", 4, scheme="weno5i"))
    assert abs(d / D_CJ - 1.0) < 0.03, (d, D_CJ)


PLANTED = {
    "flux_pressure_without_chemical_energy": [
        ("        double p = rho * T;\n        C[0] = q[1]; C[1] = q[1] * u + p; C[2] = u * (q[2] + p); C[3] = q[3] * u; return;",
         "        double p = (pb->gamma - 1.0) * (q[2] - 0.5 * q[1] * u);\n"
         "        C[0] = q[1]; C[1] = q[1] * u + p; C[2] = u * (q[2] + p); C[3] = q[3] * u; return;")],
    "energy_flux_without_pressure_work": [
        ("C[0] = q[1]; C[1] = q[1] * u + p; C[2] = u * (q[2] + p); C[3] = q[3] * u; return;",
         "C[0] = q[1]; C[1] = q[1] * u + p; C[2] = u * q[2]; C[3] = q[3] * u; return;")],
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
def test_planted_thermodynamic_mistakes_are_caught(planted, mistake):
    planted(mistake)
    d = front_speed(_problem(512))
    assert d is None or abs(d / D_CJ - 1.0) > 0.1, (mistake, d, D_CJ)
