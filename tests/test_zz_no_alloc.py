"""The no-allocation binding (at_bind_scratch): the library's own device scratch as
the workspace.  Results equal those of a caller-owned workspace (at_bind) bit for bit,
on two calls in a row (the second with a smaller input, over what the first left in
the scratch); too large a workspace and a displaced context are refused."""
import numpy as np
import pytest

import at_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _states(prs, steps, **kw):
    from paper_2204_01133_amd import ATSolver
    s = ATSolver(prs, log_steps=steps, **kw)
    s.batch_step(steps)
    out = [s.state(b) for b in range(len(prs))]
    logs = [s.delays(b, 0, steps) for b in range(len(prs))]
    s.close()
    return out, logs


def _check(prs, steps):
    ref, ref_logs = _states(prs, steps)
    got, got_logs = _states(prs, steps, scratch=True)
    for b in range(len(prs)):
        assert np.array_equal(got[b], ref[b]), b
        assert np.array_equal(got_logs[b][0], ref_logs[b][0]) and np.array_equal(got_logs[b][1], ref_logs[b][1])


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_scratch_binding_equals_caller_workspace(torch, prec):
    print(f"no-alloc binding {prec}: mixed kinds, then a smaller problem", flush=True)
    # several kernel groups (run one after another on the stream in this binding)
    big = [W.adv_diff_c1(n=1024, p=8, kmax=3), W.euler_sod_c4(n=2048, p=8, kmax=2),
           W.reactive_ns_c2(n=512, p=8), W.adv_diff_c1(n=8192, p=2, kmax=2)]
    big = [p.replace(problem_id=i, precision=prec) for i, p in enumerate(big)]
    _check(big, 15)
    small = [W.adv_diff_c1(n=256, p=4, kmax=2).replace(precision=prec, seed=7)]
    _check(small, 11)


def test_scratch_binding_limits(torch):
    from paper_2204_01133_amd import ATError, ATSolver
    print("no-alloc binding: size limit and displaced context", flush=True)
    with pytest.raises(ATError) as ei:
        ATSolver(W.batched_adr_c3(), scratch=True)      # workspace of ~0.2 GB, above 128 MiB
    assert ei.value.code == -2
    a = ATSolver([W.adv_diff_c1(n=256, p=4)], scratch=True)
    b = ATSolver([W.adv_diff_c1(n=128, p=4)], scratch=True)
    b.batch_step(3)
    with pytest.raises(ATError) as ei:
        a.batch_step(1)                                                 # b holds the scratch now
    assert ei.value.code == -3
    a.close()
    b.batch_step(2)
    b.close()
