"""Launch-shape autotuner for the batched form (at_batch_step).

For one workload (a list of problems) it times the batched step under candidate
run options and keeps the fastest.  The options it searches:

- the LDS budget per tile, which sets how many whole PEs a tile packs and how
  many workgroups share a compute unit, for each points-per-thread class of the
  kernels (tile_class 0: the small class, 1: the large one, twice the points per
  thread and per tile);
- the halo staging of the scalar finite-difference kinds: the delayed strips in
  registers, extrapolated once per step by one lane per PE side, or staged in LDS
  by every lane and extrapolated where each stage reads them (halo_lds);
- the launch shape: one workgroup per tile, or a persistent grid of a few
  workgroups per compute unit striding over the tile list;
- the tile order: cost order, or consecutive tiles grouped on one XCD.

The search has three stages: the budgets of both tile classes under the default
launch shape, the halo staging under the best of them (when the workload has a
scalar finite-difference problem), then the launch shapes and orders.  Every
candidate computes the same result bit for bit (the tiles of a step are
independent and every point takes the same arithmetic whatever tile holds it);
only the time differs.  A candidate the planner rejects (a PE that does not fit
the budget) is skipped.  Results can be kept in a JSON cache keyed by a
signature of the workload and the device; ATSolver(..., tuned=CACHE) runs with
the cached choice.

    python -m paper_2204_01133_amd.autotune --workload c3 [--steps 200] [--cache tune.json]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import time
from typing import Callable, Dict, List, Optional, Sequence

# LDS budgets per tile tried in the first stage (0: the planner's default)
BUDGETS_KIB = (0, 20, 22, 24, 26, 28, 32, 40, 64, 96, 128, 160)
# points-per-thread classes tried with every budget
TILE_CLASSES = (0, 1)
# launch shapes and orders tried in the last stage
SHAPES = ({}, {"persistent": 1, "grid_per_cu": 4}, {"persistent": 1, "grid_per_cu": 6},
          {"persistent": 1, "grid_per_cu": 8}, {"xcd_remap": 1})

# problems of the scalar finite-difference kernels (where the halo staging is a choice)
SCALAR_FD_PDES = ("adv_diff", "adr_logistic")

_SIG_FIELDS = ("pde", "scheme", "mode", "rk", "precision", "n", "p", "kmax", "at_levels", "granularity")


def signature(problems: Sequence, device_name: str = "") -> str:
    """Hash of what decides the plan and the kernels of a workload: the problems, the
    device and the library's sources (a cached choice goes stale when the planner or
    the kernels change)."""
    from .build import source_hash
    rows = [[getattr(p, f) for f in _SIG_FIELDS] + [len(getattr(p, "cdf", ()) or ())] for p in problems]
    blob = json.dumps({"device": device_name, "problems": rows, "sources": source_hash()},
                      sort_keys=True).encode()
    return hashlib.sha256(blob).hexdigest()[:24]


def measure(problems: Sequence, opts: Dict, steps: int = 100, graph_steps: int = 50) -> float:
    """Milliseconds per batched step under `opts` (HIP events on a private stream,
    after one graph's worth of untimed steps)."""
    import torch
    from .binding import ATSolver
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = ATSolver(problems, stream=st, graph_steps=graph_steps, **opts)
        s.batch_step(max(graph_steps, 1))
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        s.batch_step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        s.close()
    return ms


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0) if torch.cuda.is_available() else ""
    except Exception:
        return ""


def cached_opts(problems: Sequence, cache: str, device_name: Optional[str] = None) -> Dict:
    """The run options the cache holds for this workload on this device (as autotune
    stored them); raises KeyError when the workload was not tuned (or the library's
    sources changed since)."""
    sig = signature(problems, _device_name() if device_name is None else device_name)
    with open(cache) as fh:
        stored = json.load(fh)
    if sig not in stored:
        raise KeyError(f"no tuned run options for this workload and device in {cache} (signature {sig}); "
                       "run python -m paper_2204_01133_amd.autotune with --cache")
    return dict(stored[sig]["opts"])


def _key(opts: Dict) -> str:
    return json.dumps(opts, sort_keys=True)


def autotune(problems: Sequence, steps: int = 100, graph_steps: int = 50,
             cache: Optional[str] = None, device_name: Optional[str] = None,
             timer: Optional[Callable[[Dict], float]] = None) -> Dict:
    """Fastest run options for `problems`.

    Returns {"opts": best options (ATSolver keyword arguments, graph_steps excluded),
    "ms_per_step": its time, "table": [[options, ms or None], ...], "signature": ...}.
    `timer(opts) -> ms` replaces the GPU measurement (tests); it may raise the
    library's ATError for a candidate the planner rejects."""
    from .binding import ATError
    if device_name is None:
        device_name = _device_name()
    sig = signature(problems, device_name)
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            stored = json.load(fh)
        if sig in stored:
            return stored[sig]
    if timer is None:
        def timer(o):
            return measure(problems, o, steps=steps, graph_steps=graph_steps)

    table: List = []
    seen: Dict[str, Optional[float]] = {}

    def run(o: Dict) -> Optional[float]:
        k = _key(o)
        if k not in seen:
            try:
                seen[k] = float(timer(o))
            except ATError:
                seen[k] = None                     # the planner rejects this candidate
            table.append([o, seen[k]])
        return seen[k]

    def best_of(cands: Sequence[Dict]) -> Dict:
        timed = [(run(o), i, o) for i, o in enumerate(cands)]
        ok = [t for t in timed if t[0] is not None]
        if not ok:
            raise RuntimeError("no candidate run options were accepted for this workload")
        return min(ok, key=lambda t: (t[0], t[1]))[2]

    budgets = [dict({} if kib == 0 else {"lds_budget": kib * 1024}, **({"tile_class": 1} if cls else {}))
               for cls in TILE_CLASSES for kib in BUDGETS_KIB]
    b = best_of(budgets)
    if any(getattr(p, "scheme", "") in ("fd2", "fd4", "fd8") and getattr(p, "pde", "") in SCALAR_FD_PDES
           for p in problems):
        b = best_of([b, dict(b, halo_lds=1)])
    best = best_of([dict(b, **shape) for shape in SHAPES])
    result = {"opts": best, "ms_per_step": seen[_key(best)], "table": table, "signature": sig}
    if cache:
        stored = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                stored = json.load(fh)
        stored[sig] = result
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(stored, fh, indent=1)
        os.replace(tmp, cache)
    return result


def main(argv=None):
    import at_workloads as W
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="c3", choices=["c3", "c4", "c5", "c5batch"])
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32", "fp64"])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args(argv)
    base = {"c3": W.batched_adr_c3, "c4": lambda: [W.euler_sod_c4()], "c5": lambda: [W.detonation_c5()],
            "c5batch": W.detonation_batch_c5}[args.workload]()
    prs = [p.replace(precision=args.precision) for p in base]
    t0 = time.perf_counter()
    res = autotune(prs, steps=args.steps, cache=args.cache)
    for o, ms in res["table"]:
        print(f"{json.dumps(o):60s} {'rejected' if ms is None else f'{ms:.4f} ms/step'}", flush=True)
    print(json.dumps({"workload": args.workload, "precision": args.precision, "best": res["opts"],
                      "ms_per_step": res["ms_per_step"], "tuning_s": time.perf_counter() - t0}))


if __name__ == "__main__":
    main()
