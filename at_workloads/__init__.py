"""Seeded synthetic workloads for the asynchrony-tolerant (AT) solver.

This module is the ONLY code shared by the HIP library's tests/bench and the
CPU oracle.  It holds problem descriptions and initial conditions (inputs),
never any arithmetic of the method itself: no stencils, no extrapolation
weights, no Runge-Kutta tableaus, no delay draws.  Each side turns a
:class:`Problem` into its own descriptor and runs the method with its own code.

Every generator is seeded and reproducible.  The shapes follow the paper's
one-dimensional periodic test problems (Sec. 3 order tests, Sec. 5 reacting
cases) scaled to the sizes of the benchmark configurations:

* ``adv_diff_c1``     - advection-diffusion, 1024 points, 8 PEs, FD4 + AT
* ``reactive_ns_c2``  - one-step-chemistry premixed flame, 8192 points, 64 PEs, FD8 + AT
* ``batched_adr_c3``  - 4096 advection-diffusion-logistic problems of uneven size
* ``euler_sod_c4``    - Euler shock tube, 65536 points, 256 PEs, AT-WENO5
* ``burgers_sweep``   - inviscid Burgers order sweep (Sec. 3, Table wenoNLin)
* ``advection_e1``    - linear advection order sweep (Sec. 3, Table wenoLin)
* ``detonation_c5``   - reactive Euler detonation, 2^20 points, 4096 PEs
* ``detonation_batch_c5`` - 256 detonation tubes of uneven length

The delay distribution is given either as "uniform on {0..kmax}" or by the
paper's probability sets (Sec. 5, Table dels), converted here to integer
cumulative thresholds on a 32-bit scale (an input format, not part of the
method): ``cdf[i] = round(2**32 * sum(p[0..i]))`` for i < kmax.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

PDES = ("adv_diff", "adr_logistic", "burgers", "euler", "reactive_euler", "reactive_ns")
SCHEMES = ("fd2", "fd4", "fd8", "weno5", "weno5i")
MODES = ("sync", "as", "at")
RKS = ("fe", "rk2", "ssprk3", "rk4")
GRANULARITIES = ("per_pe", "per_pe_side", "per_boundary")
PRECISIONS = ("fp64", "fp32c", "fp32")
BCS = ("periodic", "nscbc")
# reactive NS: AT on the convective fluxes ("flux") or, by the chain rule, on the primitives ("chain")
FORMS = ("flux", "chain")

# Probability sets of Table dels (Sec. 5): [p0 p1 p2].
DELAY_SETS = {
    "set1": (0.8, 0.1, 0.1),
    "set2": (0.6, 0.3, 0.1),
    "set3": (0.4, 0.5, 0.1),
    "set4": (1.0, 0.0, 0.0),
    # Order-test probabilities of Tables wenoLin / wenoNLin.
    "half": (0.5, 0.5),
    "third": (1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0),
}


def nfields(pde: str) -> int:
    return {"adv_diff": 1, "adr_logistic": 1, "burgers": 1, "euler": 3,
            "reactive_euler": 4, "reactive_ns": 4}[pde]


def delay_cdf(p: Sequence[float]) -> Tuple[int, ...]:
    """Integer cumulative thresholds (32-bit scale) for probabilities p[0..kmax]."""
    p = [float(v) for v in p]
    if any(v < 0 for v in p) or abs(sum(p) - 1.0) > 1e-9:
        raise ValueError("delay probabilities must be >= 0 and sum to 1")
    out, acc = [], 0.0
    for v in p[:-1]:
        acc += v
        out.append(min(1 << 32, int(round(acc * 4294967296.0))))
    return tuple(out)


@dataclasses.dataclass
class Problem:
    """One periodic 1D problem: PDE, grid, PE split, scheme, delay model, IC."""
    pde: str
    scheme: str
    n: int
    p: int
    dt: float
    q0: np.ndarray                    # (F, N) float64 initial state, SoA
    mode: str = "at"
    rk: str = "rk4"
    kmax: int = 0
    cdf: Tuple[int, ...] = ()         # () -> uniform on {0..kmax}
    granularity: str = "per_pe"
    at_levels: int = 0                # J time levels of the AT extrapolation (0: scheme default)
    bc: str = "periodic"              # "periodic", or "nscbc": two ends with non-reflecting conditions
    form: str = "flux"                # reactive NS: "flux" or "chain" (chain rule on the primitives)
    x0: float = 0.0
    lx: float = 1.0
    c: float = 0.0
    alpha: float = 0.0
    r: float = 0.0
    gamma: float = 1.4
    q: float = 0.0
    ea: float = 0.0
    b: float = 0.0
    mu: float = 0.0
    pr: float = 0.72
    le: float = 1.0
    weno_eps: float = 1e-6
    seed: int = 1
    problem_id: int = 0
    precision: str = "fp64"
    steps: int = 1                    # number of steps the workload is run for
    name: str = ""

    def __post_init__(self):
        assert self.pde in PDES and self.scheme in SCHEMES and self.mode in MODES
        assert self.rk in RKS and self.granularity in GRANULARITIES
        assert self.precision in PRECISIONS and self.bc in BCS and self.form in FORMS
        self.q0 = np.ascontiguousarray(self.q0, dtype=np.float64).reshape(nfields(self.pde), self.n)
        if self.cdf:
            assert len(self.cdf) == self.kmax, "cdf needs kmax thresholds"

    @property
    def nf(self) -> int:
        return nfields(self.pde)

    @property
    def dx(self) -> float:
        return self.lx / self.n

    def x(self) -> np.ndarray:
        """Cell-centred periodic grid x_j = x0 + (j + 1/2) dx."""
        return self.x0 + (np.arange(self.n, dtype=np.float64) + 0.5) * self.dx

    def replace(self, **kw) -> "Problem":
        d = dataclasses.asdict(self)
        d.update(kw)
        if "q0" not in kw:
            d["q0"] = self.q0.copy()
        return Problem(**d)


# ----------------------------------------------------------------------------
# helpers to build initial conditions (inputs only)
# ----------------------------------------------------------------------------

def at_stable_cfl(kmax: int) -> float:
    """CFL number at which central FD + the 3-level AT halo + RK4 stays stable
    for delays up to kmax.

    Measured with the oracle on advection, diffusion and mixed problems down
    to 16 points per PE over 8000 steps (the paper tested delays up to 2 at
    unstated CFL): kmax 0 -> 0.4, 1 -> 0.3, 2 -> 0.25, 3 -> 0.12, 4 -> 0.08.
    """
    return {0: 0.4, 1: 0.3, 2: 0.25, 3: 0.12, 4: 0.08}.get(kmax, 0.05)


def _grid(n: int, x0: float, lx: float) -> np.ndarray:
    return x0 + (np.arange(n, dtype=np.float64) + 0.5) * (lx / n)


def euler_conserved(rho, u, p, gamma):
    """Conserved Euler state (rho, rho u, rho E) from primitives (input set-up)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def reactive_conserved(rho, u, T, Y, gamma, q):
    """Conserved (rho, rho u, rho E, rho Y) with E = T/(gamma-1) + u^2/2 + q Y, R = 1."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    E = T / (gamma - 1.0) + 0.5 * u * u + q * Y
    return np.stack([rho, rho * u, rho * E, rho * Y])


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def adv_diff_c1(seed: int = 1, n: int = 1024, p: int = 8, kmax: int = 3, mode: str = "at",
                steps: int = 1000, c: float = 1.0, alpha: float = 1e-3, scheme: str = "fd4",
                rk: str = "rk4", cfl: Optional[float] = None, precision: str = "fp64",
                granularity: str = "per_pe", cdf: Tuple[int, ...] = ()) -> Problem:
    """u_t + c u_x = alpha u_xx on [0,1), u0 = sin 2 pi x + 0.5 sin 6 pi x.

    dt = cfl * min(dx/|c|, dx^2/alpha); cfl defaults to the AT-stable value for kmax.
    """
    if cfl is None:
        cfl = at_stable_cfl(kmax)
    x = _grid(n, 0.0, 1.0)
    dx = 1.0 / n
    lim = []
    if c != 0:
        lim.append(dx / abs(c))
    if alpha > 0:
        lim.append(dx * dx / alpha)
    dt = cfl * min(lim)
    u0 = np.sin(2 * np.pi * x) + 0.5 * np.sin(6 * np.pi * x)
    return Problem(pde="adv_diff", scheme=scheme, n=n, p=p, dt=dt, q0=u0[None], mode=mode, rk=rk,
                   kmax=kmax, cdf=cdf, granularity=granularity, c=c, alpha=alpha, seed=seed,
                   precision=precision, steps=steps, name="adv_diff_c1")


def adv_diff_exact(x: np.ndarray, t: float, c: float, alpha: float) -> np.ndarray:
    """Exact solution of u_t + c u_x = alpha u_xx for the C1 initial condition."""
    return (np.exp(-4 * np.pi ** 2 * alpha * t) * np.sin(2 * np.pi * (x - c * t))
            + 0.5 * np.exp(-36 * np.pi ** 2 * alpha * t) * np.sin(6 * np.pi * (x - c * t)))


def reactive_ns_c2(seed: int = 1, n: int = 8192, p: int = 64, kmax: int = 4, mode: str = "at",
                   steps: int = 2000, scheme: str = "fd8", precision: str = "fp64") -> Problem:
    """One-step-chemistry premixed flame (surrogate of the Sec. 5.4 flame), periodic.

    dt = cfl(kmax) dx / S_ref with S_ref = 1.25 sqrt(gamma T_ad) bounding |u| + c.
    """
    rng = np.random.default_rng(seed)
    gamma = 1.4
    q = float(rng.uniform(5.0, 7.0))
    ea = float(rng.uniform(30.0, 40.0))
    t_ad = 1.0 + q * (gamma - 1.0) / gamma
    x = _grid(n, 0.0, 1.0)
    dx = 1.0 / n
    delta = 16 * dx
    phi = 0.5 * (np.tanh((x - 0.4) / delta) - np.tanh((x - 0.6) / delta))
    T = 1.0 + (t_ad - 1.0) * phi
    Y = 1.0 - phi
    rho = 1.0 / T
    q0 = reactive_conserved(rho, np.zeros(n), T, Y, gamma, q)
    s_ref = 1.25 * math.sqrt(gamma * t_ad)
    dt = at_stable_cfl(kmax) * dx / s_ref
    b = 20.0 * math.exp(ea / t_ad)
    return Problem(pde="reactive_ns", scheme=scheme, n=n, p=p, dt=dt, q0=q0, mode=mode, rk="rk4",
                   kmax=kmax, gamma=gamma, q=q, ea=ea, b=b, mu=2e-5, pr=0.72, le=1.0, seed=seed,
                   precision=precision, steps=steps, name="reactive_ns_c2")


def acoustic_wave(n: int = 512, p: int = 8, kmax: int = 2, mode: str = "at", seed: int = 1,
                  amp: float = 1e-3, width: float = 300.0, x_peak: float = 0.35, u0: float = 0.0,
                  mu: float = 1e-5, t_end: Optional[float] = None, scheme: str = "fd4",
                  precision: str = "fp64", cdf: Tuple[int, ...] = ()) -> Problem:
    """Acoustic pulse in a gas at rest between two non-reflecting ends (the non-reacting
    case of Sec. 5.1, eq. acIC, non-dimensional): on [0, 1) with rho0 = T0 = p0 = 1 (R = 1),
    gamma 1.4, c0 = sqrt(gamma),
        u = u0 + A exp(-B (x - x0)^2),  p = p0 + rho0 c0 (u - u0),  rho = rho0 + rho0 (u - u0) / c0,
    a right-running simple wave of amplitude A = amp * c0.  No reaction (b = 0), uniform Y.
    dt = cfl(kmax) dx / (c0 + |u|max); t_end defaults to the time the pulse needs to
    reach x = 1.2 (past the right end)."""
    gamma = 1.4
    c0 = math.sqrt(gamma)
    x = _grid(n, 0.0, 1.0)
    dx = 1.0 / n
    A = amp * c0
    u = u0 + A * np.exp(-width * (x - x_peak) ** 2)
    pr_ = 1.0 + c0 * (u - u0)
    rho = 1.0 + (u - u0) / c0
    T = pr_ / rho
    q0 = reactive_conserved(rho, u, T, np.ones(n), gamma, 0.0)
    dt0 = at_stable_cfl(kmax) * dx / (c0 + abs(u0) + A)
    if t_end is None:
        t_end = (1.2 - x_peak) / (c0 + u0)
    steps = int(math.ceil(t_end / dt0 - 1e-9))
    dt = t_end / steps
    return Problem(pde="reactive_ns", scheme=scheme, n=n, p=p, dt=dt, q0=q0, mode=mode, rk="rk4", kmax=kmax,
                   cdf=cdf, gamma=gamma, q=0.0, ea=1.0, b=0.0, mu=mu, pr=0.72, le=1.0, seed=seed,
                   precision=precision, steps=steps, bc="nscbc", name="acoustic_wave")


def batched_adr_c3(seed: int = 1, n_problems: int = 4096, steps: int = 1000,
                   precision: str = "fp64", mode: str = "at", n_min: int = 256,
                   n_max: int = 8192) -> List[Problem]:
    """4096 independent advection-diffusion-logistic problems of uneven size.

    u_t + c u_x = alpha u_xx + r u (1 - u);  N log-uniform in [256, 8192];
    P log-uniform in [4, 128] clamped to N/16;  kmax uniform in {1..4};
    c ~ U[0.5, 2];  alpha log-uniform in [1e-4, 1e-2];  r ~ U[1, 10];
    dt = cfl(kmax) * min(dx/c, dx^2/alpha, 1/r) with cfl(kmax) = at_stable_cfl(kmax).
    """
    rng = np.random.default_rng(seed)
    out = []
    ratio = n_max / n_min
    for b in range(n_problems):
        n = int(round(n_min * ratio ** rng.uniform()))
        p = int(round(4 * 32 ** rng.uniform()))
        p = max(1, min(p, n // 16))
        kmax = int(rng.integers(1, 5))
        c = float(rng.uniform(0.5, 2.0))
        alpha = float(10 ** rng.uniform(-4.0, -2.0))
        r = float(rng.uniform(1.0, 10.0))
        m = int(rng.integers(2, 9))
        ph = float(rng.uniform(0.0, 2 * np.pi))
        x = _grid(n, 0.0, 1.0)
        dx = 1.0 / n
        cfl = at_stable_cfl(kmax)
        dt = cfl * min(dx / c, dx * dx / alpha, 1.0 / r)
        u0 = 0.5 + 0.3 * np.sin(2 * np.pi * x) + 0.1 * np.sin(2 * np.pi * m * x + ph)
        out.append(Problem(pde="adr_logistic", scheme="fd4", n=n, p=p, dt=dt, q0=u0[None], mode=mode,
                           rk="rk4", kmax=kmax, c=c, alpha=alpha, r=r, seed=seed, problem_id=b,
                           precision=precision, steps=steps, name="batched_adr_c3"))
    return out


def euler_sod_c4(seed: int = 1, n: int = 65536, p: int = 256, kmax: int = 4, mode: str = "at",
                 steps: int = 200, precision: str = "fp64", cdf: Tuple[int, ...] = ()) -> Problem:
    """Periodic Sod shock tube: (1,0,1) for x < 0.5, (0.125,0,0.1) otherwise."""
    gamma = 1.4
    x = _grid(n, 0.0, 1.0)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    pr = np.where(left, 1.0, 0.1)
    q0 = euler_conserved(rho, np.zeros(n), pr, gamma)
    dt = 0.4 * (1.0 / n) / 2.5
    return Problem(pde="euler", scheme="weno5", n=n, p=p, dt=dt, q0=q0, mode=mode, rk="ssprk3",
                   kmax=kmax, cdf=cdf, gamma=gamma, seed=seed, precision=precision, steps=steps,
                   name="euler_sod_c4")


def burgers_sweep(n: int, p: Optional[int] = 8, t_end: float = 0.15, mode: str = "at",
                  delay: str = "half", seed: int = 1, n_ref: int = 256, cfl: float = 0.4,
                  precision: str = "fp64") -> Problem:
    """Inviscid Burgers u_t + (u^2/2)_x = 0 on [-1,1), u0 = 0.5 + sin(pi x).

    dt = C dx^2 with C fixed so that the CFL number is `cfl` at N = n_ref
    (|u|max = 1.5), rounded down so that t_end / dt is an integer.
    `delay` is a key of DELAY_SETS or "uniformK" for uniform on {0..K}.
    """
    p = n if p is None else p
    lx = 2.0
    x = _grid(n, -1.0, lx)
    dx = lx / n
    dx_ref = lx / n_ref
    cc = cfl / (1.5 * dx_ref)
    dt0 = cc * dx * dx
    steps = int(math.ceil(t_end / dt0 - 1e-9))
    dt = t_end / steps
    kmax, cdf = _delay_spec(delay)
    u0 = 0.5 + np.sin(np.pi * x)
    return Problem(pde="burgers", scheme="weno5", n=n, p=p, dt=dt, q0=u0[None], mode=mode,
                   rk="ssprk3", kmax=kmax, cdf=cdf, x0=-1.0, lx=lx, seed=seed, steps=steps,
                   precision=precision, name="burgers_sweep")


def advection_e1(n: int, p: Optional[int] = 4, t_end: float = 1.0, mode: str = "at",
                 delay: str = "half", seed: int = 1, literal_ic: bool = False,
                 dt_coef: float = 0.64, precision: str = "fp64") -> Problem:
    """Linear advection u_t + 5 u_x = 0 on [-1,1), u0 = sin^4(pi x) (or sin^4(pi x + 0.25)).

    dt = dt_coef * dx^2 rounded down so that t_end / dt is an integer (Sec. 3 order test).
    """
    p = n if p is None else p
    lx = 2.0
    x = _grid(n, -1.0, lx)
    dx = lx / n
    steps = int(math.ceil(t_end / (dt_coef * dx * dx) - 1e-9))
    dt = t_end / steps
    kmax, cdf = _delay_spec(delay)
    ph = 0.25 if literal_ic else 0.0
    u0 = np.sin(np.pi * x + ph) ** 4
    return Problem(pde="adv_diff", scheme="weno5", n=n, p=p, dt=dt, q0=u0[None], mode=mode,
                   rk="ssprk3", kmax=kmax, cdf=cdf, x0=-1.0, lx=lx, c=5.0, alpha=0.0, seed=seed,
                   steps=steps, precision=precision, name="advection_e1")


def _delay_spec(delay: str) -> Tuple[int, Tuple[int, ...]]:
    if delay.startswith("uniform"):
        return int(delay[len("uniform"):]), ()
    probs = DELAY_SETS[delay]
    return len(probs) - 1, delay_cdf(probs)


def _detonation(n: int, p: int, ea: float, q: float, seed: int, problem_id: int, kmax: int,
                mode: str, steps: int, precision: str, name: str) -> Problem:
    gamma = 1.4
    x = _grid(n, 0.0, 1.0)
    dx = 1.0 / n
    driver = x < 0.02
    rho = np.ones(n)
    u = np.zeros(n)
    Y = np.where(driver, 0.0, 1.0)
    pr = np.where(driver, 4.0 * (1.0 + (gamma - 1.0) * q), 1.0)
    T = pr / rho
    q0 = reactive_conserved(rho, u, T, Y, gamma, q)
    s_ref = 16.0
    t_ref = 1.0 + (gamma - 1.0) * q
    b = (s_ref / (64.0 * dx)) * math.exp(ea / t_ref)
    dt = 0.4 * dx / s_ref
    return Problem(pde="reactive_euler", scheme="weno5", n=n, p=p, dt=dt, q0=q0, mode=mode,
                   rk="ssprk3", kmax=kmax, gamma=gamma, q=q, ea=ea, b=b, seed=seed,
                   problem_id=problem_id, precision=precision, steps=steps, name=name)


def detonation_c5(seed: int = 1, n: int = 1 << 20, p: int = 4096, kmax: int = 4, mode: str = "at",
                  steps: int = 200, precision: str = "fp32c") -> Problem:
    """Reactive Euler detonation, one-step Arrhenius, Ea ~ U[20,30], q ~ U[40,60]."""
    rng = np.random.default_rng(seed)
    ea = float(rng.uniform(20.0, 30.0))
    q = float(rng.uniform(40.0, 60.0))
    return _detonation(n, p, ea, q, seed, 0, kmax, mode, steps, precision, "detonation_c5")


def detonation_batch_c5(seed: int = 1, n_tubes: int = 256, kmax: int = 4, mode: str = "at",
                        steps: int = 200, precision: str = "fp32c", n_min: int = 16384,
                        n_max: int = 131072) -> List[Problem]:
    """256 detonation tubes, N ~ U{16384..131072}, P = ceil(N/256), per-tube Ea and q."""
    rng = np.random.default_rng(seed + 1000)
    out = []
    for b in range(n_tubes):
        n = int(rng.integers(n_min, n_max + 1))
        p = -(-n // 256)
        ea = float(rng.uniform(20.0, 30.0))
        q = float(rng.uniform(40.0, 60.0))
        out.append(_detonation(n, p, ea, q, seed, b, kmax, mode, steps, precision,
                               "detonation_batch_c5"))
    return out


def total_points(problems: Sequence[Problem]) -> int:
    return int(sum(pr.n for pr in problems))
