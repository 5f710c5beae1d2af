"""Benchmark: grid-point RK-stage updates/s of the batched AT hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 4096
independent advection-diffusion-logistic problems, N log-uniform in
[256, 8192] (sum 9,402,907 points), 4-128 PEs each, delays uniform on
{0..kmax} with kmax in 1..4, 4th-order central FD with the 3-level AT halo
(Table A), classical RK4; synthetic seeded data (at_workloads.batched_adr_c3).

One "step" = one RK time step (all 4 stages, delay draws, strip ring update)
of all 4096 problems: one persistent/batched kernel launch, replayed from a
HIP graph.  Timed form: FP32 with compensated (hi+lo) state.  Reported beside
it: FP64 batched, FP32 batched with a 4-byte state, and FP64 plain (one launch
per problem) on the same data, with the error of each batched form against the
FP64 oracle on sampled problems.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20]
    python bench.py --config {c1,c2,c4,c5,c5batch} --steps 100   # other configurations
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import at_workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# a device copy of 4 GiB (beyond the last-level cache) measured 4782 GB/s read + write on MI355X
# (profiles/copy_bandwidth.md): the achievable streaming rate, reported beside the peak
COPY_GBS_MEASURED = 4782.0
# sources that decide the headline kernel's code and its tiles (the traffic record
# is used only while their hash matches the one it was measured with)
KERNEL_SOURCES = ["paper_2204_01133_amd/csrc/at_tile.hpp", "paper_2204_01133_amd/csrc/at_kernels.hpp",
                  "paper_2204_01133_amd/csrc/at_variants.hpp", "paper_2204_01133_amd/csrc/at_k_adr32.hip",
                  "paper_2204_01133_amd/csrc/at_plan.cpp", "paper_2204_01133_amd/csrc/at_plan.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c3_fp32c_traffic.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# default time levels of the AT halo extrapolation by scheme: 3 for the 4th- and 8th-order
# central schemes (Table A), 2 for 2nd order and AT-WENO (linear in time)
AT_LEVELS = {"fd2": 2, "fd4": 3, "fd8": 3, "weno5": 2, "weno5i": 2}


def algorithmic_bytes_per_step(prs, solver) -> dict:
    """State read+write of every point, plus the strip ring: every PE side
    writes one record of the current level and reads J records of delayed
    levels when its delay is non-zero (expected value for uniform delays).
    The problems of one call share the record size (same kind, scheme and form)."""
    from paper_2204_01133_amd import binding
    state = solver.query(binding.Q_STATE_BYTES)
    strip_w = solver.query(binding.Q_STRIP_BYTES)
    rec = strip_w / max(1, 2 * sum(p.p for p in prs))
    strip_r = 0.0
    for p in prs:
        assert not p.cdf and p.mode == "at", "expected uniform delays and the AT mode"
        J = p.at_levels or AT_LEVELS[p.scheme]
        strip_r += 2 * p.p * (p.kmax / (p.kmax + 1.0)) * J * rec
    return {"state": state, "strip_write": strip_w, "strip_read": strip_r,
            "total": state + strip_w + strip_r}


GRAPH_STEPS = 50
WARMUP_S = 0.25     # seconds of untimed stepping before each timed form


def graph_len(steps, graph_steps=GRAPH_STEPS):
    """Steps per captured graph for a timed run of `steps`: at most GRAPH_STEPS, and no
    more than the run, so that every timed step is replayed from a graph."""
    return max(1, min(graph_steps, steps)) if graph_steps > 0 else 0


def warmup_steps(warmup, steps, graph_steps=GRAPH_STEPS):
    """Untimed steps before the timed ones: at least one graph's worth when the timed
    steps replay a graph, so that capturing and instantiating it is not timed."""
    g = graph_len(steps, graph_steps)
    return max(warmup, g) if g > 0 else warmup


def time_form(prs, steps, warmup, method="batch_step", graph_steps=GRAPH_STEPS, **opts):
    """Seconds for `steps` steps (HIP events on the stream the tile kernels are launched
    on), after the untimed warm-up; returns (solver, seconds, wall seconds, graph length)."""
    import torch
    from paper_2204_01133_amd import ATSolver
    g = graph_len(steps, graph_steps) if method == "batch_step" else 0
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = ATSolver(prs, stream=st, graph_steps=g, **opts)
        run = getattr(s, method)
        run(warmup_steps(warmup, steps, g) if method == "batch_step" else warmup)
        torch.cuda.synchronize()
        # keep stepping (untimed) until the GPU has been busy for WARMUP_S, so that a short
        # timed run is not taken at the idle clock
        t_w = time.perf_counter()
        while method == "batch_step" and time.perf_counter() - t_w < WARMUP_S:
            run(max(g, 1))
            torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(st)
        run(steps)
        e1.record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
    return s, ms / 1000.0, wall, g


def states_after(prs, steps, graph_steps, idx):
    """States of problems idx after exactly `steps` batched steps of a fresh solver in the
    timed launch form (the timed solvers run extra untimed warm-up steps, so their step
    count is not the oracle's)."""
    from paper_2204_01133_amd import ATSolver
    s = ATSolver(prs, graph_steps=graph_steps)
    s.batch_step(steps)
    out = [s.state(i) for i in idx]
    s.close()
    return out


def _oracle_job(args):
    """One sampled problem on the oracle: its state after `keep` steps (for the errors of
    the GPU forms) and the CPU seconds of all `steps` steps (creation not included)."""
    pr, keep, steps = args
    import oracle
    with oracle.Oracle(pr.replace(precision="fp64")) as o:
        t = time.perf_counter()
        o.step(keep)
        out = o.state()
        if steps > keep:
            o.step(steps - keep)
        return out, time.perf_counter() - t


def _noop(_):
    return os.getpid()


def host_info():
    """Host CPU as seen by this process: logical CPUs, the ones it may run on, model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except Exception:
        allowed = os.cpu_count()
    return {"nproc": os.cpu_count(), "affinity": allowed, "model": model}


def oracle_sample(prs, idx, keep, steps, workers):
    """Run the sampled problems on the oracle in `workers` processes.  The pool is
    started and every worker has run a no-op before the clock starts, so the timed
    region is the oracle's own stepping (and the return of the states)."""
    import multiprocessing as mp
    jobs = [(prs[i], keep, steps) for i in idx]
    if workers > 1:
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            pool.map(_noop, range(4 * workers), chunksize=1)
            t0 = time.perf_counter()
            res = pool.map(_oracle_job, jobs, chunksize=1)
            wall = time.perf_counter() - t0
    else:
        t0 = time.perf_counter()
        res = [_oracle_job(j) for j in jobs]
        wall = time.perf_counter() - t0
    return [r[0] for r in res], wall, sum(r[1] for r in res)


def norm_err(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def field_errs(pr, got, ref):
    """Norm-wise relative error per field: max |got - ref| / scale of the field (max |ref|;
    for the momentum of the gas-dynamics problems, which is near zero at rest, at least
    max(rho) times the wave-speed scale sqrt(max E / max rho))."""
    sc = np.abs(ref).max(axis=1).astype(float)
    if pr.pde in ("euler", "reactive_euler", "reactive_ns"):
        rho = np.abs(ref[0]).max()
        sc[1] = max(sc[1], rho * np.sqrt(max(np.abs(ref[2]).max() / max(rho, 1e-300), 1e-300)))
    return (np.abs(got - ref).max(axis=1) / np.maximum(sc, 1e-300)).tolist()


# the other configurations (parity cases of the tests): timed here for the record, not
# bench lines of the headline metric
OTHER_CONFIGS = {
    "c1": ("advection-diffusion, N 1024, P 8, kmax 3, FD4 + AT, RK4", lambda: [W.adv_diff_c1()]),
    "c2": ("reactive NS flame, N 8192, P 64, kmax 4, FD8 + AT (J 3), RK4", lambda: [W.reactive_ns_c2()]),
    "c4": ("Euler Sod, N 65536, P 256, kmax 4, AT-WENO5 (J 2), SSP-RK3", lambda: [W.euler_sod_c4()]),
    "c5": ("reactive Euler detonation, N 2^20, P 4096, kmax 4, AT-WENO5, SSP-RK3",
           lambda: [W.detonation_c5()]),
    "c5batch": ("256 detonation tubes, N uniform [16384, 131072], AT-WENO5, SSP-RK3",
                lambda: W.detonation_batch_c5()),
}


# Algorithmic FLOPs per own point and RK stage of the WENO kinds, counted from the
# method's formulas (a division, square root or exp counts as one; the synchronous
# stages recomputed on the boundary windows, about 2 % more, are not counted):
#   per field: two WENO5 reconstructions of 69 (candidate values 16, smoothness
#   indicators 33, weights and their normalisation 20), the split values at the point
#   (6), the interface flux sum and difference (3), the stage state and update (5):
#   152;
#   per point, Euler: u, p, the flux vector and the wave speed (15);
#   reactive Euler: the same from the primitives (15) in the bulk precision, and the
#   temperature inversion with the Arrhenius rate (13) in FP64.
# (FP32 part, FP64 part) of the FP32 forms; the FP64 form does all of it in FP64.
WENO_FLOP = {"euler": (3 * 152 + 15, 0), "reactive_euler": (4 * 152 + 15, 13)}
VALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
# steps of the accuracy runs of the other configurations: their stated length, but 20
# for the single 2^20-point detonation (the serial oracle takes about 4 s per step)
ACC_STEPS = {"c5": 20}


def _ref_job(args):
    pr, steps = args
    import oracle
    return oracle.run(pr.replace(precision="fp64"), steps)


def run_other(name, steps, warmup, accuracy=True, workers=16, scheme=None, form=None):
    """Timing of both forms of another configuration, in the batched launch form with
    HIP graphs, and (accuracy) the error of each form against the oracle per field after
    the configuration's stated length, in the same launch form."""
    import multiprocessing as mp
    from paper_2204_01133_amd import binding
    desc, make = OTHER_CONFIGS[name]
    base = make()
    if scheme is not None:
        # the WENO configurations in the interpolation form (Sec. 3, eqs. interpS, fullSten)
        if any(p.scheme not in ("weno5", "weno5i") for p in base) or scheme not in ("weno5", "weno5i"):
            raise SystemExit(f"--scheme {scheme}: only the WENO configurations take another WENO form")
        base = [p.replace(scheme=scheme) for p in base]
        desc = desc.replace("AT-WENO5", "AT-WENO5 interpolation form" if scheme == "weno5i" else "AT-WENO5")
    if form is not None:
        # reactive NS: AT on the fluxes or, by the chain rule, on the primitives (Sec. 4)
        if any(p.pde != "reactive_ns" for p in base):
            raise SystemExit(f"--form {form}: only the reactive NS configuration has the chain-rule form")
        base = [p.replace(form=form) for p in base]
        desc += ", chain rule on the primitives" if form == "chain" else ", fluxes differentiated"
    pts = W.total_points(base)
    stages = {"rk4": 4, "ssprk3": 3, "rk2": 2, "fe": 1}[base[0].rk]
    acc_steps = ACC_STEPS.get(name, base[0].steps)
    ns = np.array([p.n for p in base])
    check = sorted({int(ns.argmin()), int(ns.argmax())})        # problems compared with the oracle
    pool = refs = None
    if accuracy:
        pool = mp.get_context("fork").Pool(min(workers, len(check)))
        refs = pool.map_async(_ref_job, [(base[b], acc_steps) for b in check])
    forms = {}
    warmup = warmup_steps(warmup, steps)
    g = graph_len(steps)
    for prec in ("fp32c", "fp64"):
        prs = [p.replace(precision=prec) for p in base]
        s, t, _, g = time_form(prs, steps, warmup)
        nbytes = algorithmic_bytes_per_step(prs, s)["total"]
        gbs = nbytes * steps / t / 1e9
        f = {"value": pts * stages * steps / t, "ms_per_step": t * 1000.0 / steps,
             "launches_per_step": s.query(binding.Q_NUM_GROUPS), "tiles": s.query(binding.Q_NUM_TILES),
             "algorithmic_bytes_per_step": nbytes, "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
        s.close()
        if base[0].pde in WENO_FLOP:
            f32, f64 = WENO_FLOP[base[0].pde]
            if prec == "fp64":
                f32, f64 = 0, f32 + f64
            ups = pts * stages / (t / steps)               # point-stage updates per second
            t32, t64 = ups * f32 / 1e12, ups * f64 / 1e12
            f["valu"] = {"bound": "alu", "flop_per_point_stage": {"f32": f32, "f64": f64},
                         "achieved_tflops": {"f32": t32, "f64": t64},
                         "peak_tflops": VALU_PEAK_TFLOPS,
                         "frac": t32 / VALU_PEAK_TFLOPS["f32"] + t64 / VALU_PEAK_TFLOPS["f64"]}
        forms[prec + "_batched"] = f
    if accuracy:
        ref = dict(zip(check, refs.get()))
        pool.close()
        for prec in ("fp32c", "fp64"):
            prs = [p.replace(precision=prec) for p in base]
            from paper_2204_01133_amd import ATSolver
            s = ATSolver(prs, graph_steps=graph_len(acc_steps))
            s.batch_step(acc_steps)
            errs = {int(b): field_errs(prs[b], s.state(b), ref[b]) for b in check}
            s.close()
            forms[prec + "_batched"]["accuracy"] = {
                "steps": acc_steps, "problems": {str(b): {"n": int(ns[b]), "max_norm_err_per_field": e}
                                                 for b, e in errs.items()},
                "max_norm_err_vs_oracle": max(max(e) for e in errs.values())}
    line = {"metric": "grid-point RK-stage updates/s", "unit": "grid-point RK-stage updates/s",
            "config": {"workload": desc, "problems": len(base), "total_points": pts, "stages": stages,
                       "form": f"at_batch_step, HIP graph of {g} steps"},
            "steps": steps, "warmup": warmup, "data": "synthetic", "forms": forms}
    print(json.dumps(line))


def main():
    global WARMUP_S
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline FP32 batched form (profiler runs)")
    ap.add_argument("--sample", type=int, default=128, help="problems in the oracle sample")
    ap.add_argument("--config", default="c3", choices=["c3"] + sorted(OTHER_CONFIGS),
                    help="c3 (default): the headline line; others: both forms, timing and accuracy")
    ap.add_argument("--no-accuracy", action="store_true", help="other configurations: timing only")
    ap.add_argument("--form", default=None, choices=["flux", "chain"],
                    help="reactive NS configuration: AT on the fluxes or on the primitives (chain rule)")
    ap.add_argument("--scheme", default=None, choices=["weno5", "weno5i"],
                    help="WENO configurations: reconstruction (weno5) or interpolation form (weno5i)")
    ap.add_argument("--warmup-s", type=float, default=WARMUP_S,
                    help="seconds of untimed stepping before each timed form (0 for profiler runs)")
    ap.add_argument("--cpu-steps", type=int, default=800,
                    help="steps of the oracle sample timed for cpu_baseline (at least the GPU's)")
    args = ap.parse_args()
    WARMUP_S = args.warmup_s
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the AT batch shards by "
              "problem across GPUs with no communication (one plan and ring per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible: libat has no CPU path", file=sys.stderr)
        sys.exit(1)

    # worker processes of the oracle: the host's CPUs this process may use, at most 16
    # (the CPU share of one GPU on a shared GPU host)
    info = host_info()
    workers = max(1, min(16, info["affinity"] or 1))

    if args.config != "c3":
        run_other(args.config, args.steps, args.warmup, accuracy=not args.no_accuracy, workers=workers,
                  scheme=args.scheme, form=args.form)
        return

    base = W.batched_adr_c3()
    S = 4
    total_pts = W.total_points(base)
    K, Wm = args.steps, warmup_steps(args.warmup, args.steps)

    # headline: FP32 compensated, batched + graph
    prs32 = [p.replace(precision="fp32c") for p in base]
    s32, t32, wall32, g32 = time_form(prs32, K, Wm)
    bytes32 = algorithmic_bytes_per_step(prs32, s32)
    from paper_2204_01133_amd import binding
    launches = s32.query(binding.Q_NUM_GROUPS)      # tile-kernel launches per batched step
    value = total_pts * S * K / t32
    ms_step = t32 * 1000.0 / K
    achieved = bytes32["total"] / (t32 / K) / 1e9

    if args.only_headline:
        line = {"metric": "grid-point RK-stage updates/s", "value": value, "ms_per_step": ms_step,
                "steps": K, "warmup": Wm, "hbm_gbs": achieved, "bytes_per_launch": bytes32["total"]}
        print(json.dumps(line))
        return

    # FP64 batched, FP64 plain (one launch per problem, fewer steps: launch bound)
    prs64 = [p.replace(precision="fp64") for p in base]
    s64, t64, _, g64 = time_form(prs64, K, Wm)
    bytes64 = algorithmic_bytes_per_step(prs64, s64)
    # FP32 batched with a 4-byte state (the low part is not kept across steps)
    prsf = [p.replace(precision="fp32") for p in base]
    sf, tf, _, gf = time_form(prsf, K, Wm)
    bytesf = algorithmic_bytes_per_step(prsf, sf)
    kp = max(2, min(20, K // 50))
    _, tplain, _, _ = time_form(prs64, kp, 2, method="step", graph_steps=0)

    # accuracy of both forms against the oracle (equal stated error), sampled problems
    idx = list(range(0, len(base), max(1, len(base) // args.sample)))[: args.sample]
    total_steps = K + Wm
    # the oracle runs the sample for at least cpu_steps steps (about 15 s of CPU), so that
    # its rate is not set by a short GPU run; the errors are taken at the GPU's step count
    cpu_steps = max(total_steps, args.cpu_steps)
    sample_pts = sum(base[i].n for i in idx)
    if args.no_cpu_baseline:
        err32 = err64 = errf = None
        cpu_rate, owall, ocpu = None, 0.0, 0.0
    else:
        refs, owall, ocpu = oracle_sample(base, idx, total_steps, cpu_steps, workers)
        err32 = max(norm_err(a, r) for a, r in zip(states_after(prs32, total_steps, g32, idx), refs))
        err64 = max(norm_err(a, r) for a, r in zip(states_after(prs64, total_steps, g64, idx), refs))
        errf = max(norm_err(a, r) for a, r in zip(states_after(prsf, total_steps, gf, idx), refs))
        cpu_rate = sample_pts * S * cpu_steps / owall

    traffic = None
    try:
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_hash") == kernel_hash():
            traffic = tr.get("bytes_per_launch")
    except (OSError, ValueError):
        traffic = None

    # one launch per step: the step time is the launch time of the one tile kernel
    # (plus the graph's inter-kernel gap); bytes and time per launch = per step
    line = {
        "metric": "grid-point RK-stage updates/s + % HBM roofline; FP32-batched vs FP64 at equal error",
        "value": value,
        "unit": "grid-point RK-stage updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched advection-diffusion-logistic, 4096 problems, N log-uniform "
                        "[256, 8192], P 4-128, kmax 1-4, FD4 + 3-level AT halo, RK4",
            "problems": len(base),
            "total_points": total_pts,
            "stages": S,
            "form": f"at_batch_step, FP32 compensated state, HIP graph of {g32} steps",
            "parallelism": "1 GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "frac_of_measured_copy": achieved / COPY_GBS_MEASURED,
            "bytes_per_launch": bytes32["total"],
            "avg_launch_us": t32 / K * 1e6,
            "launches_per_step": launches,
            "kernel": "at_tile_kernel<Cfg<0, 2, 4, true, 8>, true> (scalar FD, H=2, RK4, FP32C, 8 points/thread, whole-step form)",
        },
        "cpu_baseline": None if cpu_rate is None else {
            "value": cpu_rate,
            "unit": "grid-point RK-stage updates/s",
            "cores": workers,
            "per_core": sample_pts * S * cpu_steps / ocpu if ocpu > 0 else None,
            "kind": "oracle",
            "sample": f"{len(idx)} of {len(base)} problems (every {len(base) // len(idx)}th, "
                      f"{sample_pts} points), {cpu_steps} steps, FP64 serial C oracle, "
                      f"{workers} worker processes started before the clock, {ocpu:.1f} s CPU in "
                      f"{owall:.2f} s; per_core = updates per CPU-second of one process",
            "host": info,
        },
        "forms": {
            "fp32c_batched": {"value": value, "ms_per_step": ms_step, "max_norm_err_vs_oracle": err32,
                              "hbm_gbs": achieved},
            "fp64_batched": {"value": total_pts * S * K / t64, "ms_per_step": t64 * 1000.0 / K,
                             "max_norm_err_vs_oracle": err64,
                             "hbm_gbs": bytes64["total"] / (t64 / K) / 1e9},
            "fp32_batched": {"value": total_pts * S * K / tf, "ms_per_step": tf * 1000.0 / K,
                             "max_norm_err_vs_oracle": errf,
                             # the 4-byte state is rounded to FP32 once per step (at most 2^-24
                             # of the field's scale each time)
                             "stated_error_bound": max(2e-5, total_steps * 2.0 ** -24),
                             "hbm_gbs": bytesf["total"] / (tf / K) / 1e9},
            "fp64_plain": {"value": total_pts * S * kp / tplain, "ms_per_step": tplain * 1000.0 / kp,
                           "launches_per_step": len(base)},
            "stated_error_bound": 2e-6,
        },
        "wall_s_timed": wall32,
        "warmup_s_extra": WARMUP_S,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
