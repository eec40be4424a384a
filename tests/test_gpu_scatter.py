"""GPU scatter form and adaptive splat size (Sec. 5.2, 6.2) against the FP64 reference.

Footprints, coverage counts, mean splat sizes and the size rule are integer or exactly rounded
binary32 decisions on both sides: compared bit for bit. Colours are sums of float32 terms (one
partial per source pixel, added in binary64 in a fixed order per output pixel): max |C - C_ref| <=
1e-5 on [0, 1] colours, as for the gather, and two runs give the same bits.
"""
import numpy as np
import pytest

import oracle as O
from helpers import (DEV, afr_mod, gpu_build, oracle_build_cached, params, stats_f32_as_f64,
                     stats_to_gpu, torch_mod, workload)

pytestmark = pytest.mark.gpu


def _sizes(rng, h, w):
    """Per-pixel splat edges on the 1/256 px grid, from a fraction of a pixel to 9 px."""
    v = rng.choice(np.array([0.75, 1.0, 2.5, 3.0, 5.0, 5.5, 9.0], np.float32), (h, w))
    v[rng.random((h, w)) < 0.1] = 20.0   # above max_size below: capped
    return v.astype(np.float32)


def _run(gbuf, obuf, st, gp, op, size, max_size):
    torch = torch_mod()
    afr = afr_mod()
    gsize = torch.from_numpy(size).to(DEV)
    rgb, aux, cov = afr.reconstruct_scatter(gbuf, stats_to_gpu(st), gp, gsize, max_size)
    orgb, oaux, (on, osz) = O.scatter(obuf, stats_f32_as_f64(st), op, size, max_size)
    cov = cov.cpu().numpy()
    np.testing.assert_array_equal(cov[0], on)
    np.testing.assert_array_equal(cov[1], osz)
    err = float(np.abs(rgb.cpu().numpy() - orgb).max())
    assert err <= 1e-5, err
    a = aux.cpu().numpy()
    hit = on > 0
    np.testing.assert_allclose(a[0][hit], oaux[0][hit], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(a[1][hit], oaux[1][hit], rtol=1e-5)
    assert np.all(a[:, ~hit] == 0.0)
    return rgb, cov


@pytest.mark.parametrize("name,precision,sizes", [
    ("c1", "fp32", "block"), ("c1", "fp32", "mixed"), ("c1", "fp16", "large"),
    ("c2", "fp32", "block"), ("c2", "fp32", "mixed"), ("c3", "fp16", "block")])
def test_scatter_matches_reference(name, precision, sizes):
    wl = workload(name)
    print(f"scatter parity {name} {precision} {sizes}", flush=True)
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref)
    obuf, _ = oracle_build_cached(name, precision, wl.k)
    gp, op = params(wl.t_now)
    st = O.estimate(obuf, op)
    if sizes == "block":
        size = np.full((wl.height, wl.width), 5.0, np.float32)
        max_size = 16.0
    elif sizes == "mixed":
        size = _sizes(np.random.default_rng(3), wl.height, wl.width)
        max_size = 12.0
    else:  # splats above 16 px: the walk reads sizes and counts from global memory
        size = _sizes(np.random.default_rng(4), wl.height, wl.width)
        max_size = 40.0
    _run(gbuf, obuf, st, gp, op, size, max_size)


def test_block_sized_scatter_equals_gather():
    """Splat edge 2R + 1 with offsets strictly inside (0, 1): the scatter covers exactly the
    gather's blocks, so the two forms give the same image (to float32 summation order)."""
    afr = afr_mod()
    torch = torch_mod()
    wl = workload("c2")
    s = wl.stream
    keep = (s.x != np.floor(s.x)) & (s.y != np.floor(s.y))
    gbuf, _ = gpu_build(s.select(keep), wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    gp, _ = params(wl.t_now)
    st = afr.estimate_gradients(gbuf, gp)
    size = torch.full((wl.height, wl.width), 5.0, device=DEV)
    rgb, aux, cov = afr.reconstruct_scatter(gbuf, st, gp, size, 5.0)
    grgb, gaux = afr.reconstruct(gbuf, st, gp)
    assert float((rgb - grgb).abs().max().item()) <= 1e-5
    hit = cov[0] > 0
    assert bool(((gaux[1] > 0) == hit).all().item())


def test_splat_size_rule_matches_reference():
    torch = torch_mod()
    afr = afr_mod()
    rng = np.random.default_rng(12)
    h, w = 37, 53
    n = rng.choice(np.array([0, 1, 3, 4, 5, 17, 32, 33, 40, 200], np.float32), (h, w))
    m = (np.rint(rng.uniform(0.5, 20.0, (h, w)) * 256) / 256).astype(np.float32)
    m[n == 0] = 0.0
    m[0, :5] = np.float32(3.3)   # not on the 1/256 grid
    for sp in (O.SplatParams(), O.SplatParams(size_default=3.0, size_min=0.5, size_max=24.0,
                                              grow=2.0, shrink=0.9, n_low=2, n_high=8)):
        gsp = afr.SplatParams(**sp.__dict__)
        cov = torch.from_numpy(np.stack([n, m])).to(DEV)
        g = afr.splat_sizes(w, h, cov, gsp).cpu().numpy()
        np.testing.assert_array_equal(g, O.splat_sizes(w, h, (n, m), sp))
        g0 = afr.splat_sizes(w, h, None, gsp, device=DEV).cpu().numpy()
        np.testing.assert_array_equal(g0, O.splat_sizes(w, h, None, sp))


def test_adaptive_splat_loop_matches_reference():
    """Three images of the splat-size feedback loop on the same buffer: every image's coverage map
    and the sizes derived from it agree bit for bit, and the colours to 1e-5."""
    torch = torch_mod()
    afr = afr_mod()
    wl = workload("c2")
    print("adaptive splat loop c2", flush=True)
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    obuf, _ = oracle_build_cached("c2", "fp32", wl.k)
    gp, op = params(wl.t_now)
    st = O.estimate(obuf, op)
    sp = O.SplatParams()
    gsp = afr.SplatParams(**sp.__dict__)
    ocov = None
    gcov = None
    for it in range(3):
        osize = O.splat_sizes(wl.width, wl.height, ocov, sp)
        gsize = afr.splat_sizes(wl.width, wl.height, gcov, gsp, device=DEV)
        np.testing.assert_array_equal(gsize.cpu().numpy(), osize)
        _, cov = _run(gbuf, obuf, st, gp, op, osize, sp.size_max)
        gcov = torch.from_numpy(cov).to(DEV)
        _, _, ocov = O.scatter(obuf, stats_f32_as_f64(st), op, osize, sp.size_max)


@pytest.mark.parametrize("max_size", [16.0, 40.0])
def test_scatter_is_deterministic(max_size):
    """Every output pixel adds its splats in a fixed order: two runs (and a run on another stream)
    give identical images, aux and coverage, for LDS-staged (<= 16 px) and global-memory walks."""
    torch = torch_mod()
    afr = afr_mod()
    wl = workload("c2")
    print(f"scatter determinism max_size={max_size}", flush=True)
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, "fp16", wl.t_ref)
    gp, _ = params(wl.t_now)
    st = afr.estimate_gradients(gbuf, gp)
    size = torch.from_numpy(_sizes(np.random.default_rng(9), wl.height, wl.width)).to(DEV)
    a = afr.reconstruct_scatter(gbuf, st, gp, size, max_size)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b = afr.reconstruct_scatter(gbuf, st, gp, size, max_size)
    torch.cuda.current_stream().wait_stream(side)
    c = afr.reconstruct_scatter(gbuf, st, gp, size, max_size)
    torch.cuda.synchronize()
    for x, y, z in zip(a, b, c):
        assert torch.equal(x, y) and torch.equal(x, z)
