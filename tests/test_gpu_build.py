"""GPU deep-buffer build against the FP64 reference: bit-exact (integer selection, exact float32
offsets, round-to-nearest-even binary16)."""
import numpy as np
import pytest

import afr_scenes as S
import oracle as O
from helpers import assert_buffers_equal, gpu_build, oracle_build_cached, workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,precision", [("c1", "fp32"), ("c1", "fp16"), ("c2", "fp32"),
                                            ("c0", "fp32"), ("c3", "fp16"), ("c4", "fp32")])
def test_build_matches_reference(name, precision):
    """Every chunk size the launch picks is covered: 6 samples per thread for the small workloads,
    8 for c4 (2.1M samples), 10 for c3 (4.9M) on a 256-CU device."""
    wl = workload(name)
    print(f"build parity {name} {precision} {wl.width}x{wl.height} K={wl.k} n={len(wl.stream)}",
          flush=True)
    gbuf, gd = gpu_build(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref)
    obuf, od = oracle_build_cached(name, precision, wl.k)
    assert gd == od
    assert_buffers_equal(gbuf, obuf)


@pytest.mark.parametrize("k", [1, 3, 17, 40, 100])
def test_build_depths_and_ties(k):
    """Depths on every selection path (register lists up to 64, scan selection above), a stream with
    many equal times (ties broken by stream index) and unstratified occupancy up to ~60 per pixel."""
    rng = np.random.default_rng(100 + k)
    w, h, n = 37, 23, 37 * 23 * 30
    x = (rng.random(n) ** 2 * w).astype(np.float32)  # skewed: dense columns on the left
    y = (rng.random(n) * h).astype(np.float32)
    t = rng.choice(np.arange(0, 50, 0.5, dtype=np.float32), n)
    c = rng.random((3, n)).astype(np.float32)
    s = S.Stream(x, y, t, c[0], c[1], c[2])
    print(f"build depth K={k} n={n}", flush=True)
    for precision in ("fp32", "fp16"):
        gbuf, gd = gpu_build(s, w, h, k, precision, 40.0)
        obuf, od = O.build_buffer(s, w, h, k, precision, 40.0)
        assert gd == od
        assert_buffers_equal(gbuf, obuf)


def test_build_drops_invalid_samples_and_handles_empty_streams():
    w, h = 9, 5
    x = np.array([0.0, 8.9999, 9.0, -1e-3, 4.5, np.nan, 4.5, 4.5, 2.5, 1.0, 3.0], np.float32)
    y = np.array([0.0, 4.9999, 1.0, 1.00, 5.0, 1.0, 1.5, 1.5, 0.5, np.inf, 2.0], np.float32)
    t = np.array([1.0, 2.0, 1.0, 1.0, 1.0, 1.0, 5.0, 1.0, 1.0, 1.0, -7e4], np.float32)
    r = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, np.inf, 0.9, 1.0, 0.5], np.float32)
    g = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 7e4, 1.0, 0.5], np.float32)
    s = S.Stream(x, y, t, r, g, r.copy())
    for precision, expect_dropped in (("fp32", 7), ("fp16", 9)):
        # fp16 additionally drops the colour 7e4 and the age 4 - (-7e4) > 65504
        gbuf, gd = gpu_build(s, w, h, 2, precision, 4.0)
        obuf, od = O.build_buffer(s, w, h, 2, precision, 4.0)
        assert gd == od == expect_dropped
        assert_buffers_equal(gbuf, obuf)
    empty = S.Stream(*(np.zeros(0, np.float32) for _ in range(6)))
    gbuf, gd = gpu_build(empty, w, h, 3, "fp32", 4.0)
    assert gd == 0 and int(gbuf.count.sum().item()) == 0
    assert bool((gbuf.src == -1).all().item()) and bool((gbuf.planes == 0).all().item())


def _dense_stream(rng, w, h, per_px):
    """Stratified positions with per-pixel multiplicity ``per_px`` (an [h, w] int array), distinct
    times drawn from a coarse grid (ties) and uniform colours."""
    ys, xs = np.nonzero(per_px >= 0)
    reps = per_px[ys, xs]
    px = np.repeat(xs, reps).astype(np.float64)
    py = np.repeat(ys, reps).astype(np.float64)
    n = px.size
    x = (px + rng.random(n)).astype(np.float32)
    y = (py + rng.random(n)).astype(np.float32)
    t = rng.choice(np.arange(0, 500, 0.25, dtype=np.float32), n)
    c = rng.random((3, n)).astype(np.float32)
    perm = rng.permutation(n)
    return S.Stream(x[perm], y[perm], t[perm], c[0][perm], c[1][perm], c[2][perm])


@pytest.mark.parametrize("case", ["row_passes", "dense_row_scan", "huge_bin_scan"])
def test_build_select_paths_for_large_bins(case):
    """Bins beyond the register sweep: passes over row groups, a single row beyond the LDS list
    (direct scan of that row) and a bin beyond 16-bit record positions (direct scan of the bin)."""
    rng = np.random.default_rng({"row_passes": 1, "dense_row_scan": 2, "huge_bin_scan": 3}[case])
    if case == "row_passes":
        w, h, k = 64, 8, 16
        per = np.full((h, w), 50)
    elif case == "dense_row_scan":
        w, h, k = 64, 4, 8
        per = np.full((h, w), 6)
        per[1] = 120
    else:
        w, h, k = 16, 4, 3
        per = np.full((h, w), 1100)
    s = _dense_stream(rng, w, h, per)
    print(f"build select path {case}: {w}x{h} K={k} n={len(s)}", flush=True)
    for precision in ("fp32", "fp16"):
        gbuf, gd = gpu_build(s, w, h, k, precision, 500.0)
        obuf, od = O.build_buffer(s, w, h, k, precision, 500.0)
        assert gd == od == 0
        assert_buffers_equal(gbuf, obuf)


def test_staged_build_equals_build_and_times_every_stage():
    import torch
    import paper_2510_15876_amd as afr
    wl = workload("c2")
    dev = torch.device("cuda:0")
    arrs = [torch.from_numpy(a).to(dev) for a in wl.stream.arrays()]
    a, da = afr.build_deep_buffer(*arrs, wl.width, wl.height, wl.k, "fp16", wl.t_ref)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(afr.build_stage_count() + 1)]
    evs[0].record()
    b, db = afr.build_deep_buffer(*arrs, wl.width, wl.height, wl.k, "fp16", wl.t_ref,
                                  stage_events=evs[1:])
    torch.cuda.synchronize()
    assert torch.equal(a.planes, b.planes) and torch.equal(a.count, b.count)
    assert torch.equal(a.src, b.src) and int(da.item()) == int(db.item())
    times = [evs[i].elapsed_time(evs[i + 1]) for i in range(len(evs) - 1)]
    assert all(t >= 0.0 for t in times) and sum(times) > 0.0


@pytest.mark.parametrize("name,precision", [("c1", "fp32"), ("c3", "fp16"), ("c4", "fp32")])
def test_reprojected_build_matches_reference(name, precision):
    """Samples advanced by their surface velocity to the reference time before binning: the same
    bit-exact selection as the plain build, on the moving-disc workloads."""
    wl = workload(name)
    print(f"reprojected build {name} {precision} n={len(wl.stream)}", flush=True)
    gbuf, gd = gpu_build(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref, reproject=True)
    obuf, od = O.build_buffer(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref,
                              reproject=True)
    assert gd == od
    assert_buffers_equal(gbuf, obuf)
    # the moving discs do move samples to other pixels
    plain, _ = oracle_build_cached(name, precision, wl.k)
    assert not np.array_equal(plain.src, obuf.src)


def test_reprojection_drops_samples_moved_out_and_non_finite_motion():
    """Fast random velocities push many samples across bins and out of the image; non-finite
    velocities, and an infinite velocity at age 0, drop the sample; t > t_ref stays dropped."""
    rng = np.random.default_rng(77)
    w, h, n, t_ref = 150, 70, 150 * 70 * 6, 30.0
    x = (rng.random(n) * w).astype(np.float32)
    y = (rng.random(n) * h).astype(np.float32)
    t = rng.choice(np.arange(0, 32, 0.125, dtype=np.float32), n)   # some later than t_ref
    t[:50] = np.float32(t_ref)                                      # age 0
    vx = (rng.standard_normal(n) * 2.0).astype(np.float32)
    vy = (rng.standard_normal(n) * 0.5).astype(np.float32)
    vx[:20] = np.inf
    vx[50:60] = np.nan
    vy[60:70] = -np.inf
    c = rng.random((3, n)).astype(np.float32)
    s = S.Stream(x, y, t, c[0], c[1], c[2], vx, vy)
    print(f"reprojection drops n={n}", flush=True)
    for precision in ("fp32", "fp16"):
        for k in (3, 9):
            gbuf, gd = gpu_build(s, w, h, k, precision, t_ref, reproject=True)
            obuf, od = O.build_buffer(s, w, h, k, precision, t_ref, reproject=True)
            assert gd == od > n // 4
            assert_buffers_equal(gbuf, obuf)
