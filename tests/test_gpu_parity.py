"""GPU parity of libat (through the C ABI) against the CPU oracle.

Element-by-element comparison on the same seeded inputs: FP64 within 1e-12
norm-wise relative per field, the FP32 forms within their stated bounds, and
delay draws / effective delays bit-exact.  Launch forms (plain per-problem,
batched, persistent, XCD-ordered, HIP-graph replay, per-stage) must agree
bitwise with each other.
"""
import numpy as np
import pytest

import at_workloads as W
import oracle
from cases import batch_case, field_scale, norm_err, single_cases, tol, with_precision

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def solver(prs, **opts):
    from paper_2204_01133_amd import ATSolver
    return ATSolver(prs, **opts)


def _oracle(pr, steps):
    o = oracle.Oracle(pr.replace(precision="fp64"))
    o.step(steps)
    return o


def test_native_library_is_loaded(torch):
    import os
    from paper_2204_01133_amd import binding
    L = binding.load_library()
    for name in binding.EXPORTED:
        assert hasattr(L, name)
    maps = open(f"/proc/{os.getpid()}/maps").read()
    assert "libat.so" in maps


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
@pytest.mark.parametrize("name,pr,steps", single_cases(), ids=[c[0] for c in single_cases()])
def test_gpu_matches_oracle(torch, name, pr, steps, prec):
    print(f"case {name} {prec}", flush=True)
    pr = with_precision(pr, prec)
    s = solver([pr], log_steps=steps + 1)
    s.batch_step(steps)
    o = _oracle(pr, steps)
    err = norm_err(pr, s.state(0), o.state())
    assert err < tol(prec), err
    d1, e1 = s.delays(0, 0, steps)
    d2, e2 = o.delays(0, steps)
    assert np.array_equal(d1, d2) and np.array_equal(e1, e2)


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_gpu_batch_matches_oracle(torch, prec):
    prs, steps = batch_case()
    prs = [with_precision(p, prec) for p in prs]
    s = solver(prs)
    s.batch_step(steps)
    for b, pr in enumerate(prs):
        assert norm_err(pr, s.state(b), _oracle(pr, steps).state()) < tol(prec), b


def _run(prs, steps, method, **opts):
    s = solver(prs, **opts)
    getattr(s, method)(steps)
    return [s.state(b) for b in range(len(prs))]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_launch_forms_agree_bitwise(torch, prec):
    prs, _ = batch_case()
    prs = [with_precision(p, prec) for p in prs]
    steps = 13
    ref = _run(prs, steps, "step")                                     # plain per problem
    variants = [("batch_step", {}), ("batch_step", {"persistent": 1, "grid_per_cu": 1}),
                ("batch_step", {"xcd_remap": 1}), ("batch_step", {"graph_steps": 4}),
                ("batch_step", {"graph_steps": 5, "persistent": 1}), ("batch_step", {"halo_lds": 1}),
                ("batch_step", {"tile_class": 1}), ("step", {"halo_lds": 1, "tile_class": 1}),
                ("batch_step", {"halo_lds": 1, "graph_steps": 4, "persistent": 1})]
    for method, opts in variants:
        got = _run(prs, steps, method, **opts)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (method, opts)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_kernel_groups_run_concurrently(torch, prec):
    """Several kernel groups in one step (four kinds, and a problem whose 4096-point PEs
    need the large-tile class): the groups of a batched step run on concurrent streams,
    launched directly and from graphs, with the results of the plain form (one launch
    per problem, in order) and of the oracle."""
    prs = [W.adv_diff_c1(n=128, p=4, kmax=2), W.euler_sod_c4(n=256, p=4, kmax=2),
           W.reactive_ns_c2(n=256, p=4), W.burgers_sweep(64, p=4, n_ref=64),
           W.adv_diff_c1(n=8192, p=2, kmax=2)]
    prs = [with_precision(p.replace(problem_id=i), prec) for i, p in enumerate(prs)]
    steps = 12
    assert solver(prs).query(2) >= 5           # kernel groups
    ref = _run(prs, steps, "step")
    for opts in ({}, {"graph_steps": 4}, {"graph_steps": 5, "persistent": 1}):
        got = _run(prs, steps, "batch_step", **opts)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), opts
    for b, pr in enumerate(prs):
        assert norm_err(pr, ref[b], _oracle(pr, steps).state()) < tol(prec, pr), b


def test_autotuned_options_agree_bitwise(torch):
    """The autotuner times candidate run options on the GPU; whatever it picks, the
    result equals the default options' bit for bit."""
    from paper_2204_01133_amd.autotune import autotune
    prs, _ = batch_case()
    res = autotune(prs, steps=8, graph_steps=4)
    assert res["ms_per_step"] is not None and res["ms_per_step"] > 0
    assert sum(ms is not None for _, ms in res["table"]) >= 5
    ref = _run(prs, 13, "batch_step")
    got = _run(prs, 13, "batch_step", **res["opts"])
    for a, b in zip(got, ref):
        assert np.array_equal(a, b), res["opts"]


def test_tuned_cache_drives_the_solver(torch, tmp_path):
    """ATSolver(tuned=cache) runs with the options the autotuner stored for the workload
    (explicit options override them), with the default options' result bit for bit."""
    from paper_2204_01133_amd.autotune import autotune
    prs, _ = batch_case()
    cache = str(tmp_path / "tune.json")
    res = autotune(prs, steps=4, graph_steps=2, cache=cache)
    s = solver(prs, tuned=cache)
    assert s.run_opts == res["opts"]
    s.batch_step(13)
    ref = _run(prs, 13, "batch_step")
    for b in range(len(prs)):
        assert np.array_equal(s.state(b), ref[b])
    assert solver(prs, tuned=cache, persistent=0).run_opts["persistent"] == 0


def test_device_state_on_a_side_stream(torch):
    """A solver on a stream that is not the caller's current one, fed and read through
    device tensors (float32 input converted on the current stream, freed right after
    the call; the output consumed on the current stream): the same state as the host
    path, bit for bit."""
    prs, _ = batch_case()
    ref = _run(prs, 9, "batch_step")
    st = torch.cuda.Stream()
    s = solver(prs, stream=st, set_initial=False)
    for b, pr in enumerate(prs):
        q = torch.tensor(pr.q0, dtype=torch.float64, device="cuda")
        s.set_state(b, q)
        del q
        torch.cuda.empty_cache()
    with torch.cuda.stream(st):
        s.batch_step(9)
    got = []
    for b in range(len(prs)):
        t = s.state_device(b)
        got.append((t * 1.0).cpu().numpy())      # consumed on the current stream
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("make", [lambda: W.euler_sod_c4(n=2048, p=8), lambda: W.detonation_c5(n=2048, p=8, precision="fp64")],
                         ids=["sod", "detonation"])
def test_multi_pe_weno_tiles(torch, prec, make):
    """WENO tiles of several PEs (forced by the tile size and budget) equal one PE per
    tile bit for bit, and FP64 stays within 1e-12 of the oracle."""
    pr = with_precision(make(), prec)
    one = solver([pr], lds_budget=20 * 1024)                                  # one PE per tile
    many = solver([pr], tile_points=1024, lds_budget=160 * 1024, tile_class=1)  # four per tile
    assert one.query(1) == pr.p and many.query(1) == pr.p // 4
    one.batch_step(15)
    many.batch_step(15)
    assert np.array_equal(one.state(0), many.state(0))
    if prec == "fp64":
        assert norm_err(pr, many.state(0), _oracle(pr, 15).state()) < 1e-12


def test_graph_replay_on_torch_stream(torch):
    prs, _ = batch_case()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = solver(prs, graph_steps=3, stream=st)
        s.batch_step(10)            # 3 replays + 1 plain step
        s.batch_step(6)             # replays again from the device step counter
        got = [s.state(b) for b in range(len(prs))]
    ref = _run(prs, 16, "step")
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("make", [lambda: W.adv_diff_c1(n=256, p=8, kmax=3),
                                  lambda: W.adv_diff_c1(n=256, p=8, kmax=3, precision="fp32c"),
                                  lambda: W.adv_diff_c1(n=250, p=7, kmax=2, rk="rk2", precision="fp32"),
                                  lambda: W.euler_sod_c4(n=256, p=8),
                                  lambda: W.euler_sod_c4(n=256, p=8, precision="fp32c"),
                                  lambda: W.reactive_ns_c2(n=256, p=4, precision="fp32c")])
def test_per_stage_equals_fused(torch, make):
    pr = make()
    a = solver([pr], stage_api=1)
    b = solver([pr], stage_api=1)
    S = {"fe": 1, "rk2": 2, "ssprk3": 3, "rk4": 4}[pr.rk]
    for _ in range(6):
        a.step(1)
        for s in range(1, S + 1):
            b.rk_stage(s)
    assert np.array_equal(a.state(0), b.state(0))


def test_zero_override_is_bitwise_sync(torch):
    pr = W.euler_sod_c4(n=512, p=8)
    a = solver([pr], override_steps=20)
    a.set_override(0, np.zeros((20, pr.p, 2), np.uint8), 0)
    a.batch_step(20)
    s = solver([pr.replace(mode="sync")])
    s.batch_step(20)
    assert np.array_equal(a.state(0), s.state(0))


def test_sync_independent_of_pe_count(torch):
    ref = None
    for p in (1, 3, 8, 64, 192):
        s = solver([W.adv_diff_c1(n=192, p=p, mode="sync")])
        s.batch_step(25)
        if ref is None:
            ref = s.state(0)
        assert np.array_equal(s.state(0), ref), p


def test_override_schedule_and_stale_rejection(torch):
    from paper_2204_01133_amd import ATError
    pr = W.adv_diff_c1(n=256, p=8, kmax=3)
    sched = np.random.default_rng(3).integers(0, 4, size=(10, 8, 2)).astype(np.uint8)
    s = solver([pr], override_steps=10, log_steps=12)
    s.set_override(0, sched, 2)
    s.batch_step(12)
    o = oracle.Oracle(pr)
    o.set_override(2, sched)
    o.step(12)
    assert norm_err(pr, s.state(0), o.state()) < 1e-12
    d, _ = s.delays(0, 2, 10)
    assert np.array_equal(d, sched)
    with pytest.raises(ATError) as ei:
        s.set_override(0, np.full((2, 8, 2), 4, np.uint8), 20)
    assert ei.value.code == -5


def test_device_state_roundtrip(torch):
    pr = W.euler_sod_c4(n=512, p=8, precision="fp32c")
    s = solver([pr], set_initial=False)
    q = torch.tensor(pr.q0, device="cuda")
    s.set_state(0, q)
    s.batch_step(5)
    dev = s.state_device(0).cpu().numpy()
    assert np.array_equal(dev, s.state(0))


def test_api_errors(torch):
    from paper_2204_01133_amd import ATError
    pr = W.adv_diff_c1(n=64, p=4)
    s = solver([pr])
    with pytest.raises(ATError):
        s.rk_stage(1)                      # stage buffers not reserved
    with pytest.raises(ATError):
        solver([pr.replace(n=10, p=20, q0=np.zeros((1, 10)))])   # P > N
    big = W.adv_diff_c1(n=16384, p=1)
    with pytest.raises(ATError) as ei:
        solver([big])                      # PE larger than a tile
    assert ei.value.code == -2


# --------------------------------------------------------------------------
# full-size configurations, in the launch configuration of the benchmark
# --------------------------------------------------------------------------
def test_full_c1(torch):
    pr = W.adv_diff_c1()
    s = solver([pr], log_steps=pr.steps, graph_steps=50)
    s.batch_step(pr.steps)
    o = _oracle(pr, pr.steps)
    assert norm_err(pr, s.state(0), o.state()) < 1e-12
    assert np.array_equal(s.delays(0, 0, pr.steps)[0], o.delays(0, pr.steps)[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_full_c3_sampled(torch, prec):
    prs = [p.replace(precision=prec) for p in W.batched_adr_c3()]
    steps = prs[0].steps
    s = solver(prs, graph_steps=50, log_steps=4)
    s.batch_step(steps)
    ns = np.array([p.n for p in prs])
    pick = sorted({int(ns.argmin()), int(ns.argmax()), 0, 1, 2047, 4095,
                   int(np.argmax([p.kmax for p in prs])), int(np.argmax([p.p for p in prs]))})
    # the FP32 form rounds its 4-byte state once per step: at most 2^-24 of the scale each
    bound = max(tol(prec), steps * 2.0 ** -24) if prec == "fp32" else tol(prec)
    for b in pick:
        assert norm_err(prs[b], s.state(b), _oracle(prs[b], steps).state()) < bound, b
    # invariants over the whole batch: finite and bounded (logistic keeps u in (0, 1.1))
    for b in range(0, len(prs), 97):
        u = s.state(b)
        assert np.isfinite(u).all() and u.min() > -0.2 and u.max() < 1.3


# the oracle states of the full-length configurations, computed in worker processes on
# the host's cores from the start of this module (see tests/oracle_jobs.py)
@pytest.fixture(scope="module", autouse=True)
def full_refs(request):
    """Started with the module's first test when any full-length test is selected."""
    if not any(it.name.startswith("test_full_") and it.module is request.module
               for it in request.session.items):
        yield None
        return
    import oracle_jobs
    refs = oracle_jobs.Refs()
    yield refs
    refs.close()


def _field_report(name, prec, pr, got, ref):
    errs = np.abs(got - ref).max(axis=1) / field_scale(pr, ref)
    print(f"{name} {prec} N {pr.n}: per-field error " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    return errs


@pytest.mark.parametrize("case", ["c4", "c4_interp"])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_full_c4(torch, full_refs, prec, case):
    """The Euler shock tube at its full size and length (N 65,536, P 256, AT-WENO5 with
    delays up to 4, SSP-RK3, 200 steps) in the launch form of its timing (batched, graphs
    of 50 steps), per field against the oracle; reconstruction and interpolation forms."""
    import oracle_jobs
    pr, steps = oracle_jobs.full_length_cases()[case]
    pr = with_precision(pr, prec)
    s = solver([pr], graph_steps=50)
    s.batch_step(steps)
    errs = _field_report(case, prec, pr, s.state(0), full_refs.get(case))
    assert (errs < tol(prec, pr)).all(), errs


@pytest.mark.parametrize("case", ["c2", "c2_chain"])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_full_c2(torch, full_refs, prec, case):
    """The reactive NS flame at its full size and length (N 8192, P 64, FD8 with the
    3-level halo, delays up to 4, RK4, 2000 steps), graphs of 50 steps, flux and
    chain-rule forms; delay logs of the last 64 steps bit-exact."""
    import oracle_jobs
    pr, steps = oracle_jobs.full_length_cases()[case]
    pr = with_precision(pr, prec)
    s = solver([pr], graph_steps=50, log_steps=64)
    s.batch_step(steps)
    errs = _field_report(case, prec, pr, s.state(0), full_refs.get(case))
    assert (errs < tol(prec, pr)).all(), errs
    # the delays of the last 64 steps against the oracle's generator (one draw per PE and
    # step, both sides); this late every delay is used as drawn
    d, e = s.delays(0, steps - 64, 64)
    want = np.array([[[oracle.draw(pr, n, k, 0)] * 2 for k in range(pr.p)]
                     for n in range(steps - 64, steps)], dtype=np.uint8)
    assert np.array_equal(d, want) and np.array_equal(e, want)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_full_c5_single(torch, full_refs, prec):
    """The 2^20-point detonation (P 4096) in its launch form, as far as the serial oracle
    goes in the time of a test (20 steps)."""
    import oracle_jobs
    pr, steps = oracle_jobs.full_length_cases()["c5"]
    pr = with_precision(pr, prec)
    s = solver([pr], graph_steps=steps)
    s.batch_step(steps)
    errs = _field_report("c5", prec, pr, s.state(0), full_refs.get("c5"))
    assert (errs < tol(prec, pr)).all(), errs


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_full_c5_batch(torch, full_refs, prec):
    """The 256-tube detonation batch (19.2 M points) at its full length (200 steps) in the
    launch configuration of its timing: one launch per step, graphs of 50 steps.  The
    smallest and the largest tube per field against the oracle (the FP32 form within its
    bound for the reacting front); every tube finite with positive density."""
    import oracle_jobs
    cases = oracle_jobs.full_length_cases()
    prs = [p.replace(precision=prec) for p in W.detonation_batch_c5()]
    steps = cases["c5batch_min"][1]
    s = solver(prs, graph_steps=50, log_steps=4)
    s.batch_step(steps)
    for key in ("c5batch_min", "c5batch_max"):
        b = cases[key][0].problem_id
        assert prs[b].n == cases[key][0].n
        errs = _field_report(key, prec, prs[b], s.state(b), full_refs.get(key))
        assert (errs < tol(prec, prs[b])).all(), (key, errs)
    for b in range(0, len(prs), 15):
        u = s.state(b)
        assert np.isfinite(u).all() and u[0].min() > 0.0, b


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_full_acoustic_wave(torch, full_refs, prec):
    """The acoustic pulse between non-reflecting ends (N 512, P 8, FD4 + AT with delays up to
    2, RK4) over its whole run, until it has left through the right end (1743 steps), graphs
    of 50 steps: per field against the oracle, delay logs of the first steps bit-exact."""
    import oracle_jobs
    pr, steps = oracle_jobs.full_length_cases()["acoustic"]
    pr = with_precision(pr, prec)
    s = solver([pr], graph_steps=50, log_steps=steps)
    s.batch_step(steps)
    errs = _field_report("acoustic", prec, pr, s.state(0), full_refs.get("acoustic"))
    assert (errs < tol(prec, pr)).all(), errs
    d, e = s.delays(0, 0, 8)
    want = np.array([[[oracle.draw(pr, n, k, 0)] * 2 for k in range(pr.p)] for n in range(8)], dtype=np.uint8)
    assert np.array_equal(d, want)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_tiles_of_many_pes(torch, prec):
    """Tiles of more PE sides than threads (several sides per thread in the load
    phase): 512 PEs of 4 points packed into 2-3 tiles by an explicit budget."""
    pr = with_precision(W.adv_diff_c1(n=2048, p=512, kmax=2), prec)
    s = solver([pr], lds_budget=160 * 1024, tile_points=2048)
    assert s.query(1) <= 3
    s.batch_step(12)
    assert norm_err(pr, s.state(0), _oracle(pr, 12).state()) < tol(prec)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("levels,scheme", [(4, "fd4"), (5, "fd8")])
def test_more_extrapolation_levels(torch, prec, levels, scheme):
    """J above the default (at_levels): the load phase takes the levels beyond those
    it holds in registers from the ring one at a time."""
    pr = with_precision(W.adv_diff_c1(n=256, p=8, kmax=3, scheme=scheme), prec).replace(at_levels=levels)
    s = solver([pr])
    s.batch_step(12)
    assert norm_err(pr, s.state(0), _oracle(pr, 12).state()) < tol(prec)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("n,p", [(12, 3), (9, 1), (15, 5)])
def test_domains_shorter_than_a_window(torch, prec, n, p):
    """Periodic domains shorter than a boundary window (N < S H): the windows wrap
    round the domain more than once."""
    pr = with_precision(W.adv_diff_c1(n=n, p=p, kmax=2), prec)
    s = solver([pr])
    s.batch_step(10)
    assert norm_err(pr, s.state(0), _oracle(pr, 10).state()) < tol(prec)


# the largest PE each kind takes (a tile of the large points-per-thread class: 256
# threads x 16 points for the scalar FD kind, x 4 for the Euler WENO and reacting NS kinds)
LARGEST_PE = [("adr_fd4", lambda: W.adv_diff_c1(n=8192, p=2, kmax=3), 4096),
              ("sod_weno5", lambda: W.euler_sod_c4(n=2048, p=2), 1024),
              ("flame_fd8", lambda: W.reactive_ns_c2(n=2048, p=2, kmax=2), 1024)]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("name,make,limit", LARGEST_PE, ids=[c[0] for c in LARGEST_PE])
def test_largest_pe_of_each_kind(torch, name, make, limit, prec):
    """A PE at the tile limit runs (against the oracle); one point more is refused."""
    from paper_2204_01133_amd import ATError
    pr = with_precision(make(), prec)
    assert pr.n // pr.p == limit
    s = solver([pr])
    s.batch_step(6)
    assert norm_err(pr, s.state(0), _oracle(pr, 6).state()) < tol(prec, pr)
    over = pr.replace(n=pr.n + 2, q0=np.zeros((pr.q0.shape[0], pr.n + 2)))
    with pytest.raises(ATError) as ei:
        solver([over])
    assert ei.value.code == -2 and "exceeds the tile limit" in str(ei.value)


def test_empty_batch_and_zero_steps(torch):
    """No problems is an argument error; zero steps change nothing."""
    from paper_2204_01133_amd import ATError
    with pytest.raises(ATError) as ei:
        solver([])
    assert ei.value.code == -1
    pr = W.adv_diff_c1(n=256, p=8, kmax=3)
    s = solver([pr])
    s.batch_step(0)
    s.step(0)
    assert s.query(0) == 0 and np.array_equal(s.state(0), np.asarray(pr.q0, dtype=np.float64))


@pytest.mark.parametrize("scheme", ["weno5", "weno5i"])
@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_detonation_front_at_the_chapman_jouguet_speed(torch, prec, scheme):
    """The oracle's Chapman-Jouguet pin run on the GPU: the driver-initiated detonation (AT,
    delays up to 4) runs at the CJ speed within 3 %, its front within a grid point of the
    oracle's at both times."""
    import test_oracle_detonation as D
    pr = with_precision(D._problem(512, "at", 4, scheme=scheme), prec)
    s = solver([pr])
    d = D.front_speed(pr, run=(s.batch_step, lambda: s.state(0)))
    assert abs(d / D.D_CJ - 1.0) < 0.03, (d, D.D_CJ)
    one_cell = 1.0 / (pr.n * 0.03)                 # one grid point over the timed interval
    assert abs(d - D.front_speed(pr.replace(precision="fp64"))) <= 2 * one_cell
