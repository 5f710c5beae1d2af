"""The headline bench line on the GPU: a short run whose sampled errors against the oracle
stay within each form's stated bound (the timed solvers run untimed warm-up steps beyond
the oracle's step count; the errors come from solvers of the same launch form run for
exactly the oracle's steps)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_line_errors_within_bounds():
    out = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "20", "--warmup", "2",
                          "--sample", "8", "--cpu-steps", "22", "--warmup-s", "0.05"],
                         capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-3000:]
    line = json.loads(out.stdout.strip().splitlines()[-1])
    forms = line["forms"]
    assert forms["fp32c_batched"]["max_norm_err_vs_oracle"] < forms["stated_error_bound"]
    assert forms["fp64_batched"]["max_norm_err_vs_oracle"] < 1e-12
    assert forms["fp32_batched"]["max_norm_err_vs_oracle"] < forms["fp32_batched"]["stated_error_bound"]
    assert line["value"] > 0 and line["roofline"]["frac"] > 0
