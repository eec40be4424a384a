"""GPU sampler feedback statistics and tile selection (Sec. 4, 4.1, 6.1) against the FP64 reference.

Tile selection is exact integer arithmetic on the same float32 errors, and the spots are binary32
expressions of the same random bits: compared bit for bit. The statistics are FP64 sums in another
order: tile errors within 1e-6 relative, undersampling within 1e-7, the global figures within 1e-9.
"""
import numpy as np
import pytest

import oracle as O
from helpers import (DEV, afr_mod, gpu_build, params, stats_f32_as_f64, stats_to_gpu, torch_mod,
                     workload)

pytestmark = pytest.mark.gpu


def _sparse(name, frac, seed):
    wl = workload(name)
    keep = np.random.default_rng(seed).random(len(wl.stream)) < frac
    return wl, wl.stream.select(keep)


@pytest.mark.parametrize("name,precision,frac,tile", [("c2", "fp32", 0.15, 8), ("c3", "fp16", 0.2, 8),
                                                      ("c1", "fp32", 0.5, 4)])
def test_sampler_stats_match_reference(name, precision, frac, tile):
    afr = afr_mod()
    wl, s = _sparse(name, frac, 5)
    print(f"sampler stats {name} {precision} frac={frac}", flush=True)
    b = 4  # the sampler's queue depth (Sec. 4)
    gbuf, _ = gpu_build(s, wl.width, wl.height, b, precision, wl.t_ref)
    obuf, _ = O.build_buffer(s, wl.width, wl.height, b, precision, wl.t_ref)
    gp, op = params(wl.t_now, tile=tile)
    ost = O.estimate(obuf, op)
    seen_u = 0.0
    for sp in (O.SamplerParams(), O.SamplerParams(kappa=0.2, lam=0.8, m=0.5, gain=3.0)):
        gsp = afr.SamplerParams(sp.kappa, sp.lam, sp.m, sp.gain)
        E, u, g = afr.sampler_stats(gbuf, stats_to_gpu(ost), gp, gsp)
        oE, ou, og = O.sampler_stats(obuf, stats_f32_as_f64(ost), op, sp)
        np.testing.assert_allclose(u.cpu().numpy(), ou, rtol=0, atol=1e-7)
        np.testing.assert_allclose(E.cpu().numpy(), oE, rtol=1e-6, atol=1e-12)
        g = g.cpu().numpy()
        for i, key in enumerate(O.SAMPLER_GLOBALS):
            np.testing.assert_allclose(g[i], og[key], rtol=1e-9, err_msg=key)
        assert og["sum_v"] > 0
        seen_u += og["sum_u"]
    assert seen_u > 0   # the undersampling share is exercised (m = 0.5 marks sparse tiles)


def _rnd(rng, n):
    return rng.integers(0, 2 ** 32, 3 * n, dtype=np.uint64).astype(np.uint32)


@pytest.mark.parametrize("w,h,tile", [(256, 256, 8), (250, 131, 8), (637, 9, 16), (40, 30, 1)])
def test_sampler_select_matches_reference(w, h, tile):
    torch = torch_mod()
    afr = afr_mod()
    rng = np.random.default_rng(w + h + tile)
    ty, tx = O.tiles_shape(w, h, tile)
    n = 200_000
    cases = {"random": (rng.random((ty, tx)) ** 3).astype(np.float32),
             "zero": np.zeros((ty, tx), np.float32)}
    odd = cases["random"].copy()
    odd.reshape(-1)[::7] = 0.0
    odd.reshape(-1)[1::11] = -1.0
    odd.reshape(-1)[2::13] = np.nan
    odd.reshape(-1)[3::17] = np.inf
    cases["odd"] = odd
    for label, E in cases.items():
        print(f"sampler select {w}x{h} tile={tile} {label}", flush=True)
        r = _rnd(rng, n)
        x, y, t = afr.sampler_select(w, h, tile, torch.from_numpy(E).to(DEV),
                                     torch.from_numpy(r.view(np.int32)).to(DEV))
        ox, oy, ot = O.sampler_select(w, h, tile, E, r)
        np.testing.assert_array_equal(t.cpu().numpy(), ot)
        np.testing.assert_array_equal(x.cpu().numpy(), ox)
        np.testing.assert_array_equal(y.cpu().numpy(), oy)
        assert np.all((ox >= 0) & (ox < w) & (oy >= 0) & (oy < h))


def test_sampler_select_edge_cases():
    torch = torch_mod()
    afr = afr_mod()
    E = torch.ones((2, 3), device=DEV)
    x, y, t = afr.sampler_select(20, 10, 8, E, torch.zeros(0, dtype=torch.int32, device=DEV))
    assert x.numel() == 0 and t.numel() == 0
    # the far-edge rounding case: clipped tile at x0 = 632 of width 3
    E = np.zeros((1, 80), np.float32)
    E[0, 79] = 1.0
    r = np.array([0, (2 ** 24 - 1) << 8, 0], np.uint64).astype(np.uint32)
    x, y, t = afr.sampler_select(635, 8, 8, torch.from_numpy(E).to(DEV),
                                 torch.from_numpy(r.view(np.int32)).to(DEV))
    ox, oy, ot = O.sampler_select(635, 8, 8, E, r)
    assert x.item() == ox[0] == np.nextafter(np.float32(635), np.float32(0)) and t.item() == 79


@pytest.mark.parametrize("w,h,tile", [(256, 256, 8), (250, 131, 8), (637, 9, 16), (40, 30, 1),
                                      (2048, 8, 1)])
def test_sampler_tile_weights_match_reference(w, h, tile):
    torch = torch_mod()
    afr = afr_mod()
    rng = np.random.default_rng(7 * w + h)
    ty, tx = O.tiles_shape(w, h, tile)
    nt = ty * tx
    E = (rng.random((ty, tx)) ** 4).astype(np.float32)
    E.reshape(-1)[::5] = 0.0
    E.reshape(-1)[1::9] = np.nan
    E.reshape(-1)[2::11] = -2.0
    gE = torch.from_numpy(E).to(DEV)
    print(f"tile weights {w}x{h} tile={tile} ({nt} tiles)", flush=True)
    for n_parts in (1, 7, max(1, nt // 3), nt):
        P = afr.sampler_tile_weights(w, h, tile, gE, n_parts=n_parts).cpu().numpy()
        np.testing.assert_array_equal(P, O.sampler_tile_weights(w, h, tile, E, n_parts=n_parts))
    for target in (37.4, 0.3, 1e30, np.inf, np.nan):
        g = torch.zeros(8, dtype=torch.float64, device=DEV)
        g[7] = float(target)
        P = afr.sampler_tile_weights(w, h, tile, gE, globals_=g).cpu().numpy()
        np.testing.assert_array_equal(P, O.sampler_tile_weights(w, h, tile, E, target=target))
    Z = torch.zeros((ty, tx), device=DEV)
    np.testing.assert_array_equal(afr.sampler_tile_weights(w, h, tile, Z, n_parts=5).cpu().numpy(),
                                  O.sampler_tile_weights(w, h, tile, np.zeros((ty, tx), np.float32),
                                                         n_parts=5))
