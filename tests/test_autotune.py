"""The autotuner's search and cache (host logic, with a stand-in timer)."""
import json

import pytest

import at_workloads as W
from paper_2204_01133_amd import ATError
from paper_2204_01133_amd.autotune import BUDGETS_KIB, SHAPES, TILE_CLASSES, autotune, cached_opts, signature


def _fake_timer(calls):
    def timer(opts):
        calls.append(dict(opts))
        b = opts.get("lds_budget", 26 * 1024)
        if b < 21 * 1024:
            raise ATError(-2, "a PE does not fit the budget")
        ms = 0.1 + abs(b - 28 * 1024) / 1e6                   # best budget: 28 KiB
        ms += 0.002 * opts.get("tile_class", 0)               # the large class is slower
        ms -= 0.0005 * opts.get("halo_lds", 0)                # LDS staging is faster
        if opts.get("persistent"):
            ms -= 0.001 * opts["grid_per_cu"] if opts["grid_per_cu"] <= 6 else -0.01
        return ms
    return timer


def test_two_stage_search_picks_the_fastest_and_skips_rejected():
    prs = W.batched_adr_c3(n_problems=16)
    calls = []
    res = autotune(prs, device_name="test", timer=_fake_timer(calls))
    assert res["opts"] == {"lds_budget": 28 * 1024, "halo_lds": 1, "persistent": 1, "grid_per_cu": 6}
    # every budget of both tile classes, the halo staging (scalar FD workload), then every
    # shape under the best, each timed once
    assert len(calls) == len(BUDGETS_KIB) * len(TILE_CLASSES) + 1 + len(SHAPES) - 1
    rejected = [o for o, ms in res["table"] if ms is None]
    assert rejected == [{"lds_budget": 20 * 1024}, {"lds_budget": 20 * 1024, "tile_class": 1}]
    assert res["ms_per_step"] == min(ms for _, ms in res["table"] if ms is not None)


def test_halo_staging_only_for_scalar_fd_workloads():
    calls = []
    prs = [W.euler_sod_c4(n=512, p=8)]
    autotune(prs, device_name="test", timer=_fake_timer(calls))
    assert not any("halo_lds" in c for c in calls)
    assert len(calls) == len(BUDGETS_KIB) * len(TILE_CLASSES) + len(SHAPES) - 1


def test_cached_opts_lookup(tmp_path):
    prs = W.batched_adr_c3(n_problems=16)
    cache = str(tmp_path / "tune.json")
    res = autotune(prs, device_name="test", cache=cache, timer=_fake_timer([]))
    assert cached_opts(prs, cache, device_name="test") == res["opts"]
    with pytest.raises(KeyError):
        cached_opts(prs, cache, device_name="another device")
    with pytest.raises(KeyError):
        cached_opts(prs[:8], cache, device_name="test")


def test_cache_roundtrip_and_signature(tmp_path):
    prs = [p.replace(precision="fp32c") for p in W.batched_adr_c3(n_problems=16)]
    cache = str(tmp_path / "tune.json")
    calls = []
    first = autotune(prs, device_name="test", cache=cache, timer=_fake_timer(calls))
    n = len(calls)
    again = autotune(prs, device_name="test", cache=cache, timer=_fake_timer(calls))
    assert len(calls) == n and again == json.loads(json.dumps(first))
    # another precision or device is another workload
    other = [p.replace(precision="fp64") for p in prs]
    assert signature(other, "test") != signature(prs, "test")
    assert signature(prs, "other") != signature(prs, "test")
