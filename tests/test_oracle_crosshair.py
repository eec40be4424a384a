"""Pins of the FP64 reference's crosshair gradient estimator (Sec. 4.1).

Expected values come from closed forms of constructed streams (static ramps, colour linear in time,
hand-computed crosshairs), not from the reference's own formulas.
"""
import numpy as np
import pytest

import afr_scenes as S


def _stream(rows):
    """rows: (x, y, t, grey) per sample; grey colours make the luminance equal to the grey level."""
    a = np.array(rows, np.float64)
    f = lambda v: v.astype(np.float32)
    return S.Stream(f(a[:, 0]), f(a[:, 1]), f(a[:, 2]), f(a[:, 3]), f(a[:, 3]), f(a[:, 3]))


def _xh(*cols):
    return S.Crosshairs(*(np.array(c, np.int32) for c in cols))


def test_hand_computed_crosshairs(oracle):
    #        x     y     t     grey
    s = _stream([(5.5, 5.5, 10.0, 0.5),    # 0 centre
                 (4.5, 5.5, 10.0, 0.25),   # 1 x - 1
                 (6.5, 5.5, 10.0, 1.0),    # 2 x + 1
                 (5.5, 6.5, 10.0, 0.5),    # 3 y + 1
                 (5.5, 5.5, 2.0, 0.75),    # 4 old, 8 ms earlier
                 (5.5, 5.5, 12.0, 0.75),   # 5 "old" that is later than the centre
                 (5.5, 5.5, 10.0, np.nan)])  # 6 non-finite colour
    xh = _xh([0, 0, 0, -1, 6, 0],          # centre
             [1, -1, 6, 1, 1, 7],          # xm (7 is outside the stream: absent)
             [2, -1, -1, 2, 2, -1],        # xp
             [-1, -1, -1, -1, -1, -1],     # ym
             [3, 3, -1, 3, 3, -1],         # yp
             [4, 5, -1, 4, 4, 4])          # old
    (cx, cy, ct), (gx, gy, gt) = oracle.crosshair_records(s, xh, dt_floor=1e-3)
    tol = dict(rtol=0, atol=1e-15)
    # crosshair 0: both horizontal neighbours, one vertical, a proper old sample
    np.testing.assert_allclose([gx[0], gy[0], gt[0]], [0.375, 0.0, 0.25 / 8.0], **tol)
    assert (cx[0], cy[0], ct[0]) == (np.float32(5.5), np.float32(5.5), np.float32(10.0))
    # crosshair 1: no horizontal neighbour, old sample later than the centre
    np.testing.assert_allclose([gx[1], gy[1], gt[1]], [-1.0, 0.0, -1.0], **tol)
    # crosshair 2: the only horizontal neighbour has a NaN colour, no vertical one, no old sample
    assert (gx[2], gy[2], gt[2]) == (-1.0, -1.0, -1.0)
    # crosshairs 3, 4: absent centre, non-finite centre colour -> dropped (NaN position)
    for i in (3, 4):
        assert np.isnan(cx[i]) and np.isnan(cy[i]) and np.isnan(ct[i])
    # crosshair 5: index past the end of the stream counts as absent
    np.testing.assert_allclose([gx[5], gy[5], gt[5]], [-1.0, -1.0, 0.25 / 8.0], **tol)


def _ramp_scene(a, b, c=0.0, base=0.3):
    class Ramp:
        def shade(self, x, y, t):
            v = base + a * x + b * y + c * t
            z = np.zeros_like(v)
            return v, v, v, z, z

        def color(self, x, y, t):
            return self.shade(x, y, t)[:3]
    return Ramp()


@pytest.mark.parametrize("a,b", [(0.01, 0.02), (-0.015, 0.005)])
def test_static_ramp_gives_slopes_and_no_temporal_gradient(oracle, a, b):
    """Crosshair neighbours sit exactly one pixel away, so a static luminance ramp gives its slopes
    (up to the float32 rounding of the stored colours), and the collocated earlier sample of a
    static scene has the same colour: G_t is exactly 0. The scattered-sample estimator, whose
    new/old halves sit at different sub-pixel spots, reports a temporal gradient on the same stream
    (the static-edge bias the crosshair removes)."""
    w = h = 24
    rng = np.random.default_rng(5)
    s, xh = S.crosshair_stream(_ramp_scene(a, b), w, h, 4, 64.0, 64.0, rng)
    (cx, cy, ct), (gx, gy, gt) = oracle.crosshair_records(s, xh)
    full = (xh.xm >= 0) & (xh.xp >= 0)
    np.testing.assert_allclose(gx[full], abs(a), rtol=0, atol=2e-7)
    full = (xh.ym >= 0) & (xh.yp >= 0)
    np.testing.assert_allclose(gy[full], abs(b), rtol=0, atol=2e-7)
    assert np.all(gt == 0.0)
    p = oracle.Params(t_now=64.0, tile=8)
    buf, _ = oracle.build_buffer(s, w, h, 16, "fp32", 64.0)
    xbuf, dropped = oracle.crosshair_buffer(s, xh, w, h, 4, 64.0)
    assert dropped == 0
    st = oracle.estimate_crosshair(buf, xbuf, p)
    st_scattered = oracle.estimate(buf, p)
    gi, ti = oracle.STAT["gx"], oracle.STAT["gt"]
    np.testing.assert_allclose(st[gi], abs(a), rtol=0, atol=2e-7)
    assert np.all(st[ti] == 0.0)
    assert np.all(st_scattered[ti] > 1e-5)
    # the planes that do not depend on gradients come from the sample buffer unchanged
    for name in ("vol", "var", "lmean"):
        np.testing.assert_array_equal(st[oracle.STAT[name]], st_scattered[oracle.STAT[name]])
    # G_t = 0: the temporal limit (every age weighs the same) and the narrowest spatial filter
    assert np.all(st[oracle.STAT["kt2"]] == 0.0)


@pytest.mark.parametrize("c", [0.004, -0.0025])
def test_colour_linear_in_time_gives_its_rate(oracle, c):
    """Spatially uniform colour L = base + c t: zero spatial gradients and G_t = |c| (up to the
    float32 rounding of the stored colours and times) for every crosshair and tile."""
    w = h = 16
    rng = np.random.default_rng(6)
    s, xh = S.crosshair_stream(_ramp_scene(0.0, 0.0, c, base=0.5), w, h, 4, 64.0, 64.0, rng)
    (cx, cy, ct), (gx, gy, gt) = oracle.crosshair_records(s, xh)
    assert np.all(gt >= 0)
    # colours are exact functions of the float32 times, rounded once to float32 (half an ulp,
    # < 3e-8 at these levels), so |L_c - L_old| is |c| dt to within 6e-8
    dt = s.t[xh.centre].astype(np.float64) - s.t[xh.old].astype(np.float64)
    assert np.all(np.abs(gt - abs(c)) <= 6e-8 / dt + 1e-12)
    assert np.all(gx[gx >= 0] == 0.0) and np.all(gy[gy >= 0] == 0.0)
    p = oracle.Params(t_now=64.0, tile=8)
    buf, _ = oracle.build_buffer(s, w, h, 16, "fp32", 64.0)
    xbuf, _ = oracle.crosshair_buffer(s, xh, w, h, 4, 64.0)
    st = oracle.estimate_crosshair(buf, xbuf, p)
    np.testing.assert_allclose(st[oracle.STAT["gt"]], abs(c), rtol=0, atol=6e-8 / dt.min())


def _xbuf(oracle, w, h, k):
    return oracle.Buffer.empty(w, h, k, fp16=False, t_ref=100.0)


def _put(xb, j, i, k, t, g3):
    xb.ta[j, i, k] = t
    xb.r[j, i, k], xb.g[j, i, k], xb.b[j, i, k] = g3
    xb.count[j, i] = max(xb.count[j, i], k + 1)
    xb.src[j, i, k] = 0


def test_tile_average_weights_and_undefined_records(oracle):
    """Equal gradients average to themselves for any ages; two records at ages 0 and ln(2)/alpha
    (weights 1 and 1/2) give (2 g1 + g2) / 3; records marked undefined (-1) are skipped, and a tile
    with none defined gets 0."""
    w, h, k = 16, 8, 3
    alpha = 3.47e-3
    t_now = 100.0
    xb = _xbuf(oracle, w, h, k)
    # tile 0: gx = 0.3 everywhere at scattered ages; gy two records with weights 1 and 1/2
    for j in range(8):
        for i in range(8):
            _put(xb, j, i, 0, t_now - 3.0 * (i + j), (0.3, -1.0, -1.0))
    _put(xb, 2, 3, 1, t_now, (0.3, 0.6, -1.0))
    _put(xb, 5, 6, 1, t_now - np.log(2.0) / alpha, (0.3, 0.9, 0.05))
    # tile 1: every record undefined
    for j in range(8):
        _put(xb, j, 8 + j, 0, t_now - 1.0, (-1.0, -1.0, -1.0))
    buf = oracle.Buffer.empty(w, h, 2, fp16=False, t_ref=t_now)
    for j in range(h):
        for i in range(w):
            buf.ta[j, i, 0] = t_now - 10.0
            buf.count[j, i] = 1
    p = oracle.Params(t_now=t_now, tile=8, alpha=alpha)
    st = oracle.estimate_crosshair(buf, xb, p)
    np.testing.assert_allclose(st[oracle.STAT["gx"]][0, 0], 0.3, rtol=1e-14)
    np.testing.assert_allclose(st[oracle.STAT["gy"]][0, 0], (2 * 0.6 + 0.9) / 3.0, rtol=1e-14)
    np.testing.assert_allclose(st[oracle.STAT["gt"]][0, 0], 0.05, rtol=1e-14)
    for name in ("gx", "gy", "gt"):
        assert st[oracle.STAT[name]][0, 1] == 0.0


def test_crosshair_queue_keeps_the_newest_per_pixel(oracle):
    """The sampler's queue of depth k holds each pixel's k newest crosshairs (by centre time),
    newest first."""
    rng = np.random.default_rng(8)
    w = h = 12
    scene = _ramp_scene(0.01, 0.0)
    s, xh = S.crosshair_stream(scene, w, h, 6, 64.0, 64.0, rng)
    xbuf, dropped = oracle.crosshair_buffer(s, xh, w, h, 3, 64.0)
    assert dropped == 0
    px = np.floor(s.x[xh.centre]).astype(int) + w * np.floor(s.y[xh.centre]).astype(int)
    tc = s.t[xh.centre]
    for p in range(w * h):
        mine = np.nonzero(px == p)[0]
        newest = mine[np.lexsort((mine, tc[mine]))][::-1][:3]
        j, i = divmod(p, w)
        assert xbuf.count[j, i] == min(3, mine.size)
        np.testing.assert_array_equal(xbuf.src[j, i, :xbuf.count[j, i]], newest)


def test_empty_tile_with_crosshair_gradients_takes_the_large_volume_limit(oracle):
    """A 4 px tile whose pixels hold crosshair records but no buffered samples has V = +inf. With a
    temporal gradient its spatial widths sit at the clamp's ceiling e_min^2 + e_max^2 and kt2 = 0;
    the gather at radius 4 reaches the neighbouring tiles' slots from every pixel of it, and the
    gather and its adjoint stay finite."""
    w, h, t_now = 12, 8, 100.0
    rng = np.random.default_rng(12)
    xb = _xbuf(oracle, w, h, 2)
    for j in range(h):
        for i in range(w):
            _put(xb, j, i, 0, t_now - 1.0, (0.2, 0.1, 0.05))
    buf = oracle.Buffer.empty(w, h, 2, fp16=False, t_ref=t_now)
    for j in range(h):
        for i in range(w):
            if i < 4 and j < 4:
                continue  # tile (0, 0) stays empty
            buf.ta[j, i, 0] = t_now - rng.random() * 20.0
            buf.ox[j, i, 0], buf.oy[j, i, 0] = rng.random(2)
            buf.r[j, i, 0], buf.g[j, i, 0], buf.b[j, i, 0] = rng.random(3)
            buf.count[j, i] = 1
    p = oracle.Params(t_now=t_now, tile=4, e_min=0.5, e_max=2.0, radius=4)
    st = oracle.estimate_crosshair(buf, xb, p)
    S_ = oracle.STAT
    assert np.isinf(st[S_["vol"]][0, 0]) and st[S_["gt"]][0, 0] == pytest.approx(0.05, rel=1e-14)
    assert st[S_["sx2"]][0, 0] == 4.25 and st[S_["sy2"]][0, 0] == 4.25 and st[S_["kt2"]][0, 0] == 0.0
    for n in ("sx2", "sy2", "kt2"):
        assert np.all(np.isfinite(st[S_[n]]))
    rgb, aux = oracle.reconstruct(buf, st, p)
    assert np.all(np.isfinite(rgb)) and np.all(aux[1] > 0)
    gs, gp = oracle.backward(buf, st, p, rng.standard_normal(rgb.shape))
    assert np.all(np.isfinite(gs)) and np.all(np.isfinite(gp))
