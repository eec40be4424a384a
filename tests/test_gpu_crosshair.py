"""GPU crosshair gradient estimator (Sec. 4.1) against the FP64 reference.

The crosshair queues are compared bit for bit: every record value is an FP64 expression of stored
float32 inputs evaluated with the same operations in the same order (no contraction) and rounded
once to float32, and the queue selection is the deep-buffer build's. Tile statistics get the
estimator's tolerance (rtol 2e-6, absolute floor 1e-7), the gather on them 1e-5 on [0, 1] colours.
"""
import functools

import numpy as np
import pytest

import afr_scenes as S
import oracle as O
from helpers import (DEV, afr_mod, assert_buffers_equal, dev_stream, gpu_build, params, torch_mod)

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _workload():
    return S.make_crosshair_workload()


def _dev_xh(xh):
    torch = torch_mod()
    return [torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(DEV) for a in xh.arrays()]


def _gpu_xbuf(stream, xh, w, h, k, t_ref, dt_floor=1e-3):
    afr = afr_mod()
    p = afr.Params(t_now=float(t_ref), dt_floor=dt_floor)
    buf, dropped = afr.build_crosshair_buffer(dev_stream(stream), _dev_xh(xh), w, h, k, p, t_ref)
    return buf, int(dropped.item())


def _stat_tol(name):
    return {"vol": (2e-6, 0.0), "var": (2e-6, 1e-9), "lmean": (2e-6, 1e-7)}.get(name, (2e-6, 1e-7))


@pytest.mark.parametrize("k_xh", [1, 4, 7])
def test_crosshair_queues_match_reference(k_xh):
    cw = _workload()
    wl, xh = cw.workload, cw.crosshairs
    print(f"crosshair queues K={k_xh} n={len(xh)}", flush=True)
    gx, gd = _gpu_xbuf(wl.stream, xh, wl.width, wl.height, k_xh, wl.t_ref)
    ox, od = O.crosshair_buffer(wl.stream, xh, wl.width, wl.height, k_xh, wl.t_ref)
    assert gd == od == 0
    assert_buffers_equal(gx, ox)


def test_crosshair_records_edge_cases():
    """Absent and out-of-range indices, non-finite colours, an old sample later than the centre,
    centres outside the image or later than t_ref, and the empty crosshair list."""
    rng = np.random.default_rng(41)
    w, h, n = 40, 24, 3000
    x = (rng.random(n) * (w + 4) - 2).astype(np.float32)        # some outside the image
    y = (rng.random(n) * (h + 4) - 2).astype(np.float32)
    t = rng.choice(np.arange(0, 34, 0.25, dtype=np.float32), n)  # some later than t_ref = 32
    c = rng.random((3, n)).astype(np.float32)
    c[0, :40] = np.nan
    c[1, 40:60] = np.inf
    s = S.Stream(x, y, t, c[0], c[1], c[2])
    m = 2500
    pick = lambda: rng.integers(-200, n + 200, m).astype(np.int32)  # absent or past the end too
    xh = S.Crosshairs(pick(), pick(), pick(), pick(), pick(), pick())
    xh.centre[:5] = np.int32(2 ** 31 - 1)
    xh.old[5:10] = np.int32(-2 ** 31)
    for k in (2, 5):
        gx, gd = _gpu_xbuf(s, xh, w, h, k, 32.0)
        ox, od = O.crosshair_buffer(s, xh, w, h, k, 32.0)
        assert gd == od > 0
        assert_buffers_equal(gx, ox)
    empty = S.Crosshairs(*(np.zeros(0, np.int32) for _ in range(6)))
    gx, gd = _gpu_xbuf(s, empty, w, h, 3, 32.0)
    assert gd == 0 and int(gx.count.sum().item()) == 0


def _gpu_and_ref_stats(k_xh=4, **kw):
    afr = afr_mod()
    cw = _workload()
    wl, xh = cw.workload, cw.crosshairs
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    obuf, _ = O.build_buffer(wl.stream, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    gx, _ = _gpu_xbuf(wl.stream, xh, wl.width, wl.height, k_xh, wl.t_ref)
    ox, _ = O.crosshair_buffer(wl.stream, xh, wl.width, wl.height, k_xh, wl.t_ref)
    gp, op = params(wl.t_now, **kw)
    gst = afr.estimate_gradients_crosshair(gbuf, gx, gp)
    ost = O.estimate_crosshair(obuf, ox, op)
    return gbuf, obuf, gst, ost, gp, op


@pytest.mark.parametrize("kw", [{}, {"tau": 2.0, "sigma": 0.7}, {"tile": 4}, {"tile": 16}])
def test_crosshair_statistics_match_reference(kw):
    print(f"crosshair statistics {kw}", flush=True)
    _, _, gst, ost, _, _ = _gpu_and_ref_stats(**kw)
    g = gst.cpu().numpy().astype(np.float64)
    for i, n in enumerate(O.STAT_NAMES):
        rtol, atol = _stat_tol(n)
        np.testing.assert_allclose(g[i], ost[i], rtol=rtol, atol=atol, err_msg=f"stat {n}")


def test_forward_with_crosshair_statistics_matches_reference():
    afr = afr_mod()
    print("crosshair forward", flush=True)
    gbuf, obuf, gst, ost, gp, op = _gpu_and_ref_stats()
    rgb, _ = afr.reconstruct(gbuf, gst, gp)
    orgb, _ = O.reconstruct(obuf, ost, op)
    err = float(np.abs(rgb.cpu().numpy() - orgb).max())
    assert err <= 1e-5, err


def test_static_scene_has_zero_temporal_gradient_on_gpu():
    """A static scene: every collocated pair has equal colour, so the crosshair G_t is exactly 0
    in every tile while the scattered estimator's is not (its new/old halves sit at different
    sub-pixel spots)."""
    afr = afr_mod()
    rng = np.random.default_rng(9)
    scene = S.DiscScene(96, 64, rng, 6, 0.0, speed=0.0, checker=8.0)
    s, xh = S.crosshair_stream(scene, 96, 64, 4, 64.0, 64.0, rng)
    gbuf, _ = gpu_build(s, 96, 64, 16, "fp32", 64.0)
    gx, gd = _gpu_xbuf(s, xh, 96, 64, 4, 64.0)
    assert gd == 0
    gp, _ = params(64.0)
    st = afr.estimate_gradients_crosshair(gbuf, gx, gp).cpu().numpy()
    st0 = afr.estimate_gradients(gbuf, gp).cpu().numpy()
    assert np.all(st[O.STAT["gt"]] == 0.0) and np.all(st[O.STAT["kt2"]] == 0.0)
    assert st0[O.STAT["gt"]].max() > 1e-4


@pytest.mark.parametrize("radius", [2, 4])
def test_tiles_without_buffered_samples_take_the_large_volume_limit(radius):
    """Tiles that hold crosshair records but no buffered samples (V = +inf, G_t > 0): widths at the
    clamp's ceiling e_min^2 + e_max^2, kt2 = 0, no NaN anywhere; statistics, forward and adjoint
    against the reference."""
    torch = torch_mod()
    afr = afr_mod()
    cw = _workload()
    wl, xh = cw.workload, cw.crosshairs
    print(f"crosshair empty tiles radius={radius}", flush=True)
    x, y = wl.stream.x, wl.stream.y
    # tiles (1, 26) and (2, 12) of 8 px: moving content, so their crosshair G_t is > 0
    empty = (((x >= 208) & (x < 216) & (y >= 8) & (y < 16))
             | ((x >= 96) & (x < 104) & (y >= 16) & (y < 24)))
    s = wl.stream.select(~empty)
    gbuf, _ = gpu_build(s, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    obuf, _ = O.build_buffer(s, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    gx, _ = _gpu_xbuf(wl.stream, xh, wl.width, wl.height, 4, wl.t_ref)
    ox, _ = O.crosshair_buffer(wl.stream, xh, wl.width, wl.height, 4, wl.t_ref)
    gp, op = params(wl.t_now, radius=radius, e_min=0.5, e_max=2.0)
    gst = afr.estimate_gradients_crosshair(gbuf, gx, gp)
    ost = O.estimate_crosshair(obuf, ox, op)
    g = gst.cpu().numpy().astype(np.float64)
    assert not np.isnan(g).any() and not np.isnan(ost).any()
    st = O.STAT
    for ty, tx in ((1, 26), (2, 12)):
        assert np.isinf(ost[st["vol"]][ty, tx]) and ost[st["gt"]][ty, tx] > 0
        assert g[st["sx2"]][ty, tx] == np.float32(4.25) and g[st["kt2"]][ty, tx] == 0.0
    for i, n in enumerate(O.STAT_NAMES):
        rtol, atol = _stat_tol(n)
        np.testing.assert_allclose(g[i], ost[i], rtol=rtol, atol=atol, err_msg=f"stat {n}")
    rgb, aux = afr.reconstruct(gbuf, gst, gp)
    orgb, _ = O.reconstruct(obuf, ost, op)
    r = rgb.cpu().numpy()
    assert np.array_equal(np.isnan(r), np.isnan(orgb))
    assert float(np.nanmax(np.abs(r - orgb))) <= 1e-5
    # the adjoint on the same float32 statistics
    ost32 = np.ascontiguousarray(g)
    og = np.random.default_rng(radius).standard_normal(orgb.shape) * 1e-3
    og[np.isnan(orgb)] = 0.0
    _, gpar = afr.reconstruct_backward(gbuf, gst, gp, rgb, aux, torch.from_numpy(og).float().to(DEV))
    _, opar = O.backward(obuf, ost32, op, og)
    assert np.all(np.isfinite(gpar.cpu().numpy()))
    np.testing.assert_allclose(gpar.cpu().numpy(), opar, rtol=1e-4)
