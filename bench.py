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
    python bench.py --config {c1,c2,c4,c5,c5batch} --steps 100   # other configurations, timing only
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
AT_LEVELS = {"fd2": 2, "fd4": 3, "fd8": 3, "weno5": 2}


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


def warmup_steps(warmup, steps, graph_steps=50):
    """Untimed steps before the timed ones: at least one graph's worth when the timed
    steps replay a graph, so that capturing and instantiating it is not timed."""
    return max(warmup, graph_steps) if 0 < graph_steps <= steps else warmup


def time_form(prs, steps, warmup, method="batch_step", graph_steps=50, **opts):
    import torch
    from paper_2204_01133_amd import ATSolver
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = ATSolver(prs, stream=st, graph_steps=graph_steps, **opts)
        run = getattr(s, method)
        run(warmup_steps(warmup, steps, graph_steps) if method == "batch_step" else warmup)
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
    return s, ms / 1000.0, wall


def _oracle_job(args):
    pr, steps = args
    import oracle
    t = time.perf_counter()
    with oracle.Oracle(pr.replace(precision="fp64")) as o:
        o.step(steps)
        out = o.state()
    return out, time.perf_counter() - t


def oracle_sample(prs, idx, steps, workers):
    import multiprocessing as mp
    jobs = [(prs[i], steps) for i in idx]
    t0 = time.perf_counter()
    if workers > 1:
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            res = pool.map(_oracle_job, jobs)
    else:
        res = [_oracle_job(j) for j in jobs]
    wall = time.perf_counter() - t0
    return [r[0] for r in res], wall, sum(r[1] for r in res)


def norm_err(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


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


def run_other(name, steps, warmup):
    desc, make = OTHER_CONFIGS[name]
    base = make()
    pts = W.total_points(base)
    stages = {"rk4": 4, "ssprk3": 3, "rk2": 2, "fe": 1}[base[0].rk]
    forms = {}
    warmup = warmup_steps(warmup, steps)
    for prec in ("fp32c", "fp64"):
        prs = [p.replace(precision=prec) for p in base]
        s, t, _ = time_form(prs, steps, warmup)
        from paper_2204_01133_amd import binding
        nbytes = algorithmic_bytes_per_step(prs, s)["total"]
        gbs = nbytes * steps / t / 1e9
        forms[prec + "_batched"] = {"value": pts * stages * steps / t, "ms_per_step": t * 1000.0 / steps,
                                    "launches_per_step": s.query(binding.Q_NUM_GROUPS),
                                    "tiles": s.query(binding.Q_NUM_TILES),
                                    "algorithmic_bytes_per_step": nbytes, "hbm_gbs": gbs,
                                    "hbm_frac": gbs / HBM_PEAK_GBS}
    line = {"metric": "grid-point RK-stage updates/s", "unit": "grid-point RK-stage updates/s",
            "config": {"workload": desc, "problems": len(base), "total_points": pts, "stages": stages,
                       "form": "at_batch_step, HIP graph of 50 steps"},
            "steps": steps, "warmup": warmup, "data": "synthetic", "forms": forms}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline FP32 batched form (profiler runs)")
    ap.add_argument("--sample", type=int, default=128, help="problems in the oracle sample")
    ap.add_argument("--config", default="c3", choices=["c3"] + sorted(OTHER_CONFIGS),
                    help="c3 (default): the headline line; others: timing of both forms only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the AT batch shards by "
              "problem across GPUs with no communication (one plan and ring per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible: libat has no CPU path", file=sys.stderr)
        sys.exit(1)

    if args.config != "c3":
        run_other(args.config, args.steps, args.warmup)
        return

    base = W.batched_adr_c3()
    S = 4
    total_pts = W.total_points(base)
    K, Wm = args.steps, warmup_steps(args.warmup, args.steps)

    # headline: FP32 compensated, batched + graph
    prs32 = [p.replace(precision="fp32c") for p in base]
    s32, t32, wall32 = time_form(prs32, K, Wm)
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
    s64, t64, _ = time_form(prs64, K, Wm)
    bytes64 = algorithmic_bytes_per_step(prs64, s64)
    # FP32 batched with a 4-byte state (the low part is not kept across steps)
    prsf = [p.replace(precision="fp32") for p in base]
    sf, tf, _ = time_form(prsf, K, Wm)
    bytesf = algorithmic_bytes_per_step(prsf, sf)
    kp = max(2, min(20, K // 50))
    _, tplain, _ = time_form(prs64, kp, 2, method="step", graph_steps=0)

    # accuracy of both forms against the oracle (equal stated error), sampled problems
    idx = list(range(0, len(base), max(1, len(base) // args.sample)))[: args.sample]
    total_steps = K + Wm
    workers = 1
    try:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    except Exception:
        workers = max(1, min(16, os.cpu_count() or 1))
    sample_pts = sum(base[i].n for i in idx)
    if args.no_cpu_baseline:
        err32 = err64 = errf = None
        cpu_rate, owall, ocpu = None, 0.0, 0.0
    else:
        refs, owall, ocpu = oracle_sample(base, idx, total_steps, workers)
        err32 = max(norm_err(s32.state(i), r) for i, r in zip(idx, refs))
        err64 = max(norm_err(s64.state(i), r) for i, r in zip(idx, refs))
        errf = max(norm_err(sf.state(i), r) for i, r in zip(idx, refs))
        cpu_rate = sample_pts * S * total_steps / owall

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
            "form": "at_batch_step, FP32 compensated state, HIP graph of 50 steps",
            "parallelism": "1 GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": bytes32["total"],
            "avg_launch_us": t32 / K * 1e6,
            "launches_per_step": launches,
            "kernel": "at_tile_kernel<Cfg<0, 2, 4, true, 8>, true> (scalar FD, H=2, RK4, FP32C, 8 points/thread, whole-step form)",
        },
        "cpu_baseline": None if cpu_rate is None else {
            "value": cpu_rate,
            "unit": "grid-point RK-stage updates/s",
            "cores": workers,
            "per_core": sample_pts * S * total_steps / ocpu if ocpu > 0 else None,
            "kind": "oracle",
            "sample": f"{len(idx)} of {len(base)} problems (every {len(base) // len(idx)}th, "
                      f"{sample_pts} points), {total_steps} steps, FP64 serial C oracle, "
                      f"{workers} processes, {ocpu:.1f} s CPU; per_core = updates per CPU-second of one process",
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
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
