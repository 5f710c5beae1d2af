"""Parity cases shared by the emulator tests (CPU) and the GPU tests.

Sizes are small enough for the oracle to finish in seconds while spanning
several tiles, ragged PE splits (N not divisible by P), one-point PEs and
every kernel kind, precision, mode, RK scheme and delay granularity.
"""
import numpy as np

import at_workloads as W

# FP64 bar: norm-wise relative error per field (max |gpu - oracle| / scale)
TOL_FP64 = 1e-12
# FP32 forms: stated bounds per form (measured margins are ~10x below these)
TOL_FP32C = 2e-6
TOL_FP32 = 2e-5


def field_scale(pr, ref):
    """Per-field scale for norm-wise errors: max |q| of the field, and for
    momentum fields (near zero at rest) max(rho) times the wave-speed scale."""
    s = np.abs(ref).max(axis=1).astype(float)
    if pr.pde in ("euler", "reactive_euler", "reactive_ns"):
        rho = np.abs(ref[0]).max()
        E = np.abs(ref[2]).max() / max(rho, 1e-300)
        s[1] = max(s[1], rho * np.sqrt(max(E, 1e-300)))
    return np.maximum(s, 1e-300)


def norm_err(pr, got, ref):
    return (np.abs(got - ref).max(axis=1) / field_scale(pr, ref)).max()


# FP32 forms on the reacting WENO kind (detonation) beyond its first steps: the ignition at
# the front amplifies the FP32 rounding of the bulk flux arithmetic, in synchronous and AT
# runs alike (about 5e-6 within 50-100 steps at N 4096), whatever the state's compensation
TOL_FP32_REACTING = 2e-5


def tol(prec, pr=None):
    t = {"fp64": TOL_FP64, "fp32c": TOL_FP32C, "fp32": TOL_FP32}[prec]
    if prec != "fp64" and pr is not None and pr.pde == "reactive_euler":
        t = max(t, TOL_FP32_REACTING)
    return t


def single_cases():
    """(name, problem, steps) -- one problem per context."""
    out = [
        ("c1_fd4_at", W.adv_diff_c1(n=256, p=8, kmax=3), 40),
        ("c1_fd4_ragged", W.adv_diff_c1(n=250, p=7, kmax=3), 40),
        ("c1_fd8_at", W.adv_diff_c1(n=200, p=7, kmax=2, scheme="fd8"), 30),
        ("fd2_rk2_onept", W.adv_diff_c1(n=64, p=64, kmax=2, scheme="fd2", rk="rk2",
                                        granularity="per_pe_side"), 30),
        ("fd4_fe_p1", W.adv_diff_c1(n=96, p=1, kmax=2, rk="fe", cfl=0.1), 30),
        ("fd4_boundary", W.adv_diff_c1(n=256, p=8, kmax=3, granularity="per_boundary"), 40),
        ("fd4_set3", W.adv_diff_c1(n=256, p=8, kmax=2, cdf=W.delay_cdf(W.DELAY_SETS["set3"])), 40),
        ("fd4_as", W.adv_diff_c1(n=256, p=8, kmax=3, mode="as"), 40),
        ("fd4_sync", W.adv_diff_c1(n=256, p=8, kmax=3, mode="sync"), 40),
        ("fd4_bigpe", W.adv_diff_c1(n=8192, p=2, kmax=2), 10),
        ("burgers_p8", W.burgers_sweep(128, p=8, n_ref=128), 30),
        ("burgers_onept", W.burgers_sweep(64, p=None, n_ref=64), 20),
        ("advection_e1", W.advection_e1(64, p=4), 20),
        ("sod", W.euler_sod_c4(n=512, p=8), 30),
        ("sod_ragged_as", W.euler_sod_c4(n=500, p=9, mode="as"), 30),
        ("detonation", W.detonation_c5(n=1024, p=8, precision="fp64"), 20),
        # WENO interpolation form (Sec. 3, eqs. interpS, fullSten; AT halo of eq. stenF)
        ("sod_interp", W.euler_sod_c4(n=512, p=8).replace(scheme="weno5i"), 30),
        ("burgers_interp_as", W.burgers_sweep(128, p=8, n_ref=128, mode="as").replace(scheme="weno5i"), 20),
        ("advection_interp_ragged", W.advection_e1(60, p=7).replace(scheme="weno5i"), 20),
        ("detonation_interp", W.detonation_c5(n=1024, p=8, precision="fp64").replace(scheme="weno5i"), 20),
        ("flame", W.reactive_ns_c2(n=512, p=8), 20),
        ("flame_fd4_rk2", W.reactive_ns_c2(n=300, p=5, scheme="fd4").replace(rk="rk2"), 20),
        # chain-rule form of reactive NS (Sec. 4 after eq. convEq): AT on the primitives
        ("flame_chain", W.reactive_ns_c2(n=512, p=8).replace(form="chain"), 20),
        ("flame_chain_fd4_as_ragged", W.reactive_ns_c2(n=300, p=7, scheme="fd4", mode="as").replace(form="chain"), 20),
        # non-periodic ends with non-reflecting conditions (acoustic pulse, Sec. 5.1)
        ("acoustic_at", W.acoustic_wave(n=256, p=8, kmax=2), 60),
        ("acoustic_as_ragged", W.acoustic_wave(n=250, p=7, kmax=2, mode="as", x_peak=0.8), 40),
        ("acoustic_fd8_sync", W.acoustic_wave(n=320, p=4, kmax=2, mode="sync", scheme="fd8", x_peak=0.9), 30),
    ]
    return out


def batch_case():
    prs = W.batched_adr_c3(n_problems=8, n_min=256, n_max=2048, steps=30)
    return prs, 30


def with_precision(pr, prec):
    return pr.replace(precision=prec)
