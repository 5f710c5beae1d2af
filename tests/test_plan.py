"""The planner's tiling rules (host code, run through the CPU build of the library).

- Tiles hold whole PEs.  A workload too small to fill the GPU is spread to about
  two tiles per compute unit, as far as its PEs allow (one PE per tile at most).
- The default LDS per tile is 26 KiB for the FP32 scalar finite-difference kernels
  of halo width up to 2 (6 workgroups per CU) and 40 KiB otherwise (4 per CU); an
  explicit budget is respected; no launch exceeds the 160 KiB of a CU.
"""
import pytest

import at_workloads as W

at_emu = pytest.importorskip("at_emu")

Q_TILES, Q_GROUPS, Q_POINTS, Q_LDS = 1, 2, 3, 6


def _plan(prs, **opts):
    return at_emu.Emu(prs, **opts)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_small_workloads_one_pe_per_tile(prec):
    for pr in (W.adv_diff_c1(), W.reactive_ns_c2()):
        e = _plan([pr.replace(precision=prec)])
        assert e.query(Q_TILES) == pr.p, (pr.pde, e.query(Q_TILES))


def test_large_batch_packs_several_pes_per_tile():
    prs = W.batched_adr_c3(n_problems=512)
    e = _plan([p.replace(precision="fp32c") for p in prs])
    assert e.query(Q_POINTS) == W.total_points(prs)
    # about two tiles per CU would be 512; the LDS budget, not the spread, sets the size
    assert e.query(Q_TILES) < sum(p.p for p in prs)


@pytest.mark.parametrize("prec,budget", [("fp32c", 26 * 1024), ("fp64", 40 * 1024)])
def test_default_lds_budget(prec, budget):
    prs = W.batched_adr_c3(n_problems=512)
    e = _plan([p.replace(precision=prec) for p in prs])
    assert e.query(Q_LDS) <= budget
    assert e.query(Q_LDS) > budget // 2          # tiles are packed up to it


def test_explicit_lds_budget_respected():
    # PEs are packed up to the budget; a tile of one PE may exceed it
    prs = [p.replace(precision="fp32c") for p in W.batched_adr_c3(n_problems=512)]
    small = _plan(prs, lds_budget=16 * 1024)
    large = _plan(prs, lds_budget=40 * 1024)
    assert small.query(Q_TILES) > large.query(Q_TILES)
    assert small.query(Q_LDS) <= large.query(Q_LDS) <= 40 * 1024


def test_explicit_tile_points_respected():
    pr = W.adv_diff_c1(n=4096, p=64).replace(precision="fp32c")
    e = _plan([pr], tile_points=256)
    assert e.query(Q_TILES) == 4096 // 256


Q_STATE, Q_STRIP, Q_PES = 4, 7, 8


@pytest.mark.parametrize("prec", ["fp32c", "fp32", "fp64"])
@pytest.mark.parametrize("make,S,H,F", [(lambda: W.batched_adr_c3(n_problems=64), 4, 2, 1),
                                        (lambda: [W.reactive_ns_c2()], 4, 4, 4),
                                        (lambda: [W.euler_sod_c4(n=4096, p=16)], 3, 3, 3)])
def test_algorithmic_bytes_follow_the_layout(prec, make, S, H, F):
    """The byte counts behind the roofline figures.  The state is read and written once
    per point and field: 8 B for FP64 and for FP32 hi + lo, 4 B for FP32.  Every PE
    side writes one ring record of the stage values at its H halo points: 8*S*H*F bytes
    in FP64, 4*(S+1)*H*F in the FP32 forms (the low parts of stage 1 ride along)."""
    prs = [p.replace(precision=prec) for p in make()]
    e = _plan(prs)
    s_state = {"fp64": 8, "fp32c": 8, "fp32": 4}[prec]
    rec = 8 * S * H * F if prec == "fp64" else 4 * (S + 1) * H * F
    npts = sum(p.n for p in prs)
    npes = sum(p.p for p in prs)
    assert e.query(Q_PES) == npes
    assert e.query(Q_STATE) == 2 * F * npts * s_state
    assert e.query(Q_STRIP) == 2 * npes * rec


@pytest.mark.parametrize("prec,pes_per_tile", [("fp32c", 2), ("fp32", 2), ("fp64", 1)])
def test_weno_default_budget_packs_two_pes_in_fp32(prec, pes_per_tile):
    """The FP32 Euler WENO kernels default to 64 KiB per tile: a tile packs two of the
    detonation's 256-point PEs (their registers admit only 2-3 waves per SIMD, so the
    larger tile costs no occupancy); the FP64 form keeps one PE per tile (one PE already
    exceeds its 40 KiB default, which a single-PE tile may)."""
    pr = W.detonation_c5().replace(precision=prec)
    e = _plan([pr])
    assert e.query(Q_TILES) == pr.p // pes_per_tile
    assert e.query(Q_LDS) <= (64 if prec != "fp64" else 160) * 1024


def test_uncompiled_combination_rejected():
    """A pde / scheme combination that validates but has no compiled kernel (the reactive
    Navier-Stokes kernels exist for the 4th- and 8th-order stencils only) is refused with
    a clear message instead of a plan built from unset sizes."""
    pr = W.reactive_ns_c2(n=512, p=8).replace(scheme="fd2")
    with pytest.raises(at_emu.EmuError) as ei:
        _plan([pr])
    assert "-2" in str(ei.value) and "no compiled kernel" in str(ei.value)


def test_non_periodic_ends_rules():
    """Non-periodic ends run on the reactive NS kind only, and need the first and last PE
    to hold max(4, S*H) points (so that no boundary window reaches an end)."""
    ok = W.acoustic_wave(n=256, p=8)
    _plan([ok])
    with pytest.raises(at_emu.EmuError) as ei:
        _plan([ok.replace(n=64, p=16, q0=ok.q0[:, :64])])          # 4-point PEs, S*H = 8
    assert "-2" in str(ei.value)
    sod = W.euler_sod_c4(n=256, p=4).replace(bc="nscbc")
    with pytest.raises(at_emu.EmuError):
        _plan([sod])
