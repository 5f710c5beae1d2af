"""Pins of the oracle's delay stream (Sec. 2.1: random delay per PE boundary;
Sec. 5 and Table dels: delay probabilities).

The generator is the SplitMix64 finaliser of Steele, Lea & Flood (2014) used
as a counter-based hash.  Its published reference sequence pins the mixing
function; frequencies are pinned by chi-square against the requested p_k.
"""
import numpy as np
import pytest
from scipy import stats

import at_workloads as W
import oracle

GOLDEN = 0x9E3779B97F4A7C15


def test_splitmix64_reference_sequence():
    # SplitMix64 seeded with 1234567: the generator's first five outputs are
    # mix64(seed + k * golden gamma), k = 1..5 (published reference values).
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    got = [oracle.mix64(1234567 + k * GOLDEN) for k in range(1, 6)]
    assert got == ref


def _delay_run(kmax, cdf, gran="per_pe_side", steps=12, n=1 << 15):
    # one-point PEs, synchronous numerics (cheap), delays logged for every PE side
    pr = W.Problem(pde="adv_diff", scheme="fd2", n=n, p=n, dt=1e-3, q0=np.zeros((1, n)),
                   mode="sync", rk="fe", kmax=kmax, cdf=cdf, granularity=gran, c=1.0, seed=7)
    o = oracle.Oracle(pr)
    o.step(steps)
    d, e = o.delays(0, steps)
    return d, e


@pytest.mark.parametrize("kmax", [1, 3, 4])
def test_uniform_delay_frequencies(kmax):
    d, _ = _delay_run(kmax, ())
    counts = np.bincount(d.ravel(), minlength=kmax + 1)
    assert counts.size == kmax + 1
    exp = np.full(kmax + 1, d.size / (kmax + 1))
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, kmax) > 1e-3, (counts, chi2)


@pytest.mark.parametrize("name", ["set1", "set2", "set3", "half", "third"])
def test_table_delay_frequencies(name):
    probs = np.array(W.DELAY_SETS[name])
    kmax = len(probs) - 1
    d, _ = _delay_run(kmax, W.delay_cdf(probs))
    counts = np.bincount(d.ravel(), minlength=kmax + 1)
    exp = probs * d.size
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, kmax) > 1e-3, (counts, exp)


def test_set4_is_synchronous():
    d, _ = _delay_run(2, W.delay_cdf(W.DELAY_SETS["set4"]), steps=3, n=4096)
    assert (d == 0).all()


def test_granularity_semantics():
    d, _ = _delay_run(4, (), gran="per_pe", steps=3, n=256)
    assert (d[:, :, 0] == d[:, :, 1]).all()
    d, _ = _delay_run(4, (), gran="per_boundary", steps=3, n=256)
    # the right boundary of PE p is the left boundary of PE p+1 (periodic)
    assert (d[:, :, 1] == np.roll(d[:, :, 0], -1, axis=1)).all()
    d, _ = _delay_run(4, (), gran="per_pe_side", steps=3, n=4096)
    assert (d[:, :, 0] != d[:, :, 1]).mean() > 0.7


def test_effective_delay_clamp_at_start():
    # AT with J levels cannot reach before level 0: k_eff = max(0, min(k, n - J + 1))
    n = 64
    pr = W.adv_diff_c1(n=n, p=16, kmax=4, steps=8)
    o = oracle.Oracle(pr)
    o.step(8)
    d, e = o.delays(0, 8)
    J = 3
    for step in range(8):
        want = np.clip(np.minimum(d[step].astype(int), step - J + 1), 0, None)
        assert (e[step] == want).all()
    pa = pr.replace(mode="as")
    o = oracle.Oracle(pa)
    o.step(8)
    d, e = o.delays(0, 8)
    for step in range(8):
        assert (e[step] == np.minimum(d[step], step)).all()


def test_draws_depend_on_every_counter_field():
    pr = W.adv_diff_c1(n=64, p=8, kmax=15)
    base = [oracle.draw(pr, 5, 3, 0) for _ in range(2)]
    assert base[0] == base[1]
    others = {
        "step": [oracle.draw(pr, s, 3, 0) for s in range(40)],
        "pe": [oracle.draw(pr, 5, p, 0) for p in range(40)],
        "seed": [oracle.draw(pr.replace(seed=s), 5, 3, 0) for s in range(40)],
        "problem": [oracle.draw(pr.replace(problem_id=b), 5, 3, 0) for b in range(40)],
    }
    for k, v in others.items():
        assert len(set(v)) > 8, k
