"""The gfx950 kernels' tile code run on the CPU (bounds-checked emulation)
against the oracle, before and beside the GPU runs.

The emulation compiles the kernels' own tile code for the host with every LDS,
register-file and HBM access bounds-checked and LDS / registers poisoned with
NaN, so layout and indexing mistakes fail here without a GPU.  Numerical
parity uses the same cases and tolerances as the GPU tests.
"""
import numpy as np
import pytest

import at_workloads as W
import oracle
from cases import batch_case, norm_err, single_cases, tol, with_precision

at_emu = pytest.importorskip("at_emu")


def _oracle(pr, steps):
    o = oracle.Oracle(pr.replace(precision="fp64"))
    o.step(steps)
    return o


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
@pytest.mark.parametrize("name,pr,steps", single_cases(), ids=[c[0] for c in single_cases()])
def test_emu_matches_oracle(name, pr, steps, prec):
    pr = with_precision(pr, prec)
    e = at_emu.Emu([pr], log_steps=steps + 1)
    e.step(steps)
    o = _oracle(pr, steps)
    assert norm_err(pr, e.state(0), o.state()) < tol(prec)
    d1, e1 = e.delays(0, 0, steps)
    d2, e2 = o.delays(0, steps)
    assert np.array_equal(d1, d2) and np.array_equal(e1, e2)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_emu_batch_matches_oracle(prec):
    prs, steps = batch_case()
    prs = [with_precision(p, prec) for p in prs]
    e = at_emu.Emu(prs)
    e.step(steps)
    for b, pr in enumerate(prs):
        assert norm_err(pr, e.state(b), _oracle(pr, steps).state()) < tol(prec), b


def test_emu_mixed_kinds_one_context():
    prs = [W.adv_diff_c1(n=128, p=4, kmax=2), W.euler_sod_c4(n=256, p=4, kmax=2),
           W.reactive_ns_c2(n=256, p=4), W.burgers_sweep(64, p=4, n_ref=64)]
    prs = [p.replace(problem_id=i) for i, p in enumerate(prs)]
    e = at_emu.Emu(prs)
    assert e.query(2) >= 4   # kernel variants
    e.step(10)
    for b, pr in enumerate(prs):
        assert norm_err(pr, e.state(b), _oracle(pr, 10).state()) < 1e-12, b


@pytest.mark.parametrize("make", [lambda: W.adv_diff_c1(n=256, p=8, kmax=3),
                                  lambda: W.adv_diff_c1(n=256, p=8, kmax=3, precision="fp32c"),
                                  lambda: W.adv_diff_c1(n=250, p=7, kmax=2, rk="rk2", precision="fp32"),
                                  lambda: W.euler_sod_c4(n=256, p=8),
                                  lambda: W.euler_sod_c4(n=256, p=8, precision="fp32c"),
                                  lambda: W.reactive_ns_c2(n=256, p=4),
                                  lambda: W.reactive_ns_c2(n=256, p=4, precision="fp32c")])
def test_emu_per_stage_equals_fused(make):
    pr = make()
    a = at_emu.Emu([pr], stage_api=1)
    b = at_emu.Emu([pr], stage_api=1)
    S = {"fe": 1, "rk2": 2, "ssprk3": 3, "rk4": 4}[pr.rk]
    for _ in range(6):
        a.step(1)
        for s in range(1, S + 1):
            b.rk_stage(s)
    assert np.array_equal(a.state(0), b.state(0))


def test_emu_zero_override_is_bitwise_sync():
    pr = W.euler_sod_c4(n=256, p=8)
    a = at_emu.Emu([pr], override_steps=20)
    a.set_override(0, np.zeros((20, pr.p, 2), np.uint8), 0)
    a.step(20)
    s = at_emu.Emu([pr.replace(mode="sync")])
    s.step(20)
    assert np.array_equal(a.state(0), s.state(0))


def test_emu_sync_independent_of_pe_count():
    ref = None
    for p in (1, 3, 8, 64):
        e = at_emu.Emu([W.adv_diff_c1(n=192, p=p, mode="sync")])
        e.step(25)
        if ref is None:
            ref = e.state(0)
        assert np.array_equal(e.state(0), ref), p


def test_emu_override_stale_rejected():
    pr = W.adv_diff_c1(n=64, p=4, kmax=2)
    e = at_emu.Emu([pr], override_steps=4)
    with pytest.raises(at_emu.EmuError):
        e.set_override(0, np.full((2, 4, 2), 3, np.uint8), 0)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_emu_tiles_of_many_pes(prec):
    """Tiles of more PE sides than threads (several sides per thread in the load
    phase): 512 PEs of 4 points packed into 2-3 tiles by an explicit budget."""
    pr = with_precision(W.adv_diff_c1(n=2048, p=512, kmax=2), prec)
    e = at_emu.Emu([pr], lds_budget=160 * 1024, tile_points=2048)
    assert e.query(1) <= 3
    e.step(12)
    assert norm_err(pr, e.state(0), _oracle(pr, 12).state()) < tol(prec)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("levels,scheme", [(4, "fd4"), (5, "fd8")])
def test_emu_more_extrapolation_levels(prec, levels, scheme):
    """J above the default (at_levels): the load phase takes the levels beyond those
    it holds in registers from the ring one at a time."""
    pr = with_precision(W.adv_diff_c1(n=256, p=8, kmax=3, scheme=scheme), prec).replace(at_levels=levels)
    e = at_emu.Emu([pr])
    e.step(12)
    assert norm_err(pr, e.state(0), _oracle(pr, 12).state()) < tol(prec)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("n,p", [(12, 3), (9, 1), (15, 5)])
def test_emu_domains_shorter_than_a_window(prec, n, p):
    """Periodic domains shorter than a boundary window (N < S H): the windows wrap
    round the domain more than once."""
    pr = with_precision(W.adv_diff_c1(n=n, p=p, kmax=2), prec)
    e = at_emu.Emu([pr])
    e.step(10)
    assert norm_err(pr, e.state(0), _oracle(pr, 10).state()) < tol(prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("make", [lambda: W.euler_sod_c4(n=2048, p=8),
                                  lambda: W.detonation_c5(n=2048, p=8, precision="fp64")])
def test_emu_multi_pe_weno_tiles(prec, make):
    """WENO tiles of several PEs (forced by the tile size and LDS budget) give the result
    of one PE per tile bit for bit, and the oracle's."""
    pr = with_precision(make(), prec)
    one = at_emu.Emu([pr], tile_points=256)
    many = at_emu.Emu([pr], tile_points=1024, lds_budget=160 * 1024)
    assert one.query(1) == pr.p and many.query(1) < pr.p
    one.step(12)
    many.step(12)
    assert np.array_equal(one.state(0), many.state(0))
    assert norm_err(pr, many.state(0), _oracle(pr, 12).state()) < tol(prec, pr)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("opts", [{"halo_lds": 1}, {"tile_class": 1}, {"halo_lds": 1, "tile_class": 1}],
                         ids=["halo_lds", "tile_class", "both"])
def test_emu_run_options_agree_bitwise(prec, opts):
    """The halo staging (LDS or registers) and the tile class change where the work
    runs, not its arithmetic: the states equal the default options' bit for bit, in the
    batched form and in the per-stage form."""
    prs = [with_precision(p, prec) for p in W.batched_adr_c3(n_problems=6, n_min=256, n_max=2048, steps=20)]
    prs.append(with_precision(W.adv_diff_c1(n=250, p=7, kmax=3, scheme="fd8"), prec).replace(problem_id=99))
    steps = 17
    ref = at_emu.Emu(prs)
    got = at_emu.Emu(prs, **opts)
    ref.step(steps)
    got.step(steps)
    for b in range(len(prs)):
        assert np.array_equal(ref.state(b), got.state(b)), b
    pr = with_precision(W.adv_diff_c1(n=256, p=8, kmax=3), prec)
    a = at_emu.Emu([pr], stage_api=1)
    c = at_emu.Emu([pr], stage_api=1, **opts)
    for _ in range(5):
        a.step(1)
        for s in range(1, 5):
            c.rk_stage(s)
    assert np.array_equal(a.state(0), c.state(0))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_largest_scalar_pe_in_emulation(prec):
    """The scalar FD kind's largest PE (4096 points, one large-class tile) under the bounds
    checks of the emulation, against the oracle; 4097 points are refused."""
    pr = W.adv_diff_c1(n=8192, p=2, kmax=3).replace(precision=prec)
    e = at_emu.Emu([pr])
    assert e.query(1) == 2
    e.step(3)
    o = oracle.Oracle(pr.replace(precision="fp64"))
    o.step(3)
    assert norm_err(pr, e.state(0), o.state()) < tol(prec)
    with pytest.raises(at_emu.EmuError, match="exceeds the tile limit 4096"):
        at_emu.Emu([pr.replace(n=8194, q0=np.zeros((1, 8194)))])
