"""Oracle runs of the full-length configurations in worker processes.

The GPU tests submit these at the start of their module, so that the serial oracle
(seconds to a minute per configuration) runs on the host's cores while the GPU
tests before them run.  Workers are spawned (they import the oracle and the
workloads only, never the GPU library)."""
import concurrent.futures as cf
import multiprocessing as mp
import os

import at_workloads as W


def run(args):
    import oracle
    pr, steps = args
    return oracle.run(pr.replace(precision="fp64"), steps)


# configurations at full size and length: name -> (problem, steps)
def full_length_cases():
    import numpy as np
    prs = W.detonation_batch_c5()
    ns = np.array([p.n for p in prs])
    return {
        "c2": (W.reactive_ns_c2(), 2000),
        "c2_chain": (W.reactive_ns_c2().replace(form="chain"), 2000),
        "c4": (W.euler_sod_c4(), 200),
        "c4_interp": (W.euler_sod_c4().replace(scheme="weno5i"), 200),
        # the serial oracle takes seconds per step at 2^20 points
        "c5": (W.detonation_c5(), 20),
        "c5batch_min": (prs[int(ns.argmin())], 200),
        "c5batch_max": (prs[int(ns.argmax())], 200),
        # the acoustic pulse between non-reflecting ends, until it has left the domain
        "acoustic": (W.acoustic_wave(), W.acoustic_wave().steps),
    }


class Refs:
    """Futures of the oracle states of full_length_cases(), by name."""

    def __init__(self, workers=None):
        cases = full_length_cases()
        if workers is None:
            try:
                workers = len(os.sched_getaffinity(0))
            except Exception:
                workers = os.cpu_count() or 1
        workers = max(1, min(len(cases), workers, 16))
        self.ex = cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))
        self.fut = {k: self.ex.submit(run, v) for k, v in cases.items()}

    def get(self, name, timeout=900):
        return self.fut[name].result(timeout=timeout)

    def close(self):
        # runs not needed any more (a selection of the tests, or a failure) are stopped
        for proc in list(getattr(self.ex, "_processes", {}).values()):
            if proc.is_alive():
                proc.terminate()
        self.ex.shutdown(wait=True, cancel_futures=True)
