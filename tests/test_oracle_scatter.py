"""Pins of the FP64 reference's scatter form and adaptive splat size (Sec. 5.2, Sec. 6.2)."""
import numpy as np
import pytest

import afr_scenes as S


def _single(oracle, w, h, x, y, t, rgb, t_now=10.0, k=2):
    buf = oracle.Buffer.empty(w, h, k, fp16=False, t_ref=t_now)
    i, j = int(np.floor(x)), int(np.floor(y))
    buf.ox[j, i, 0], buf.oy[j, i, 0], buf.ta[j, i, 0] = x - i, y - j, t
    buf.r[j, i, 0], buf.g[j, i, 0], buf.b[j, i, 0] = rgb
    buf.count[j, i] = 1
    buf.src[j, i, 0] = 0
    return buf


def _flat_stats(oracle, w, h, p, sx2=0.8, sy2=1.1, kt2=1e-4):
    ty, tx = oracle.tiles_shape(w, h, p.tile)
    st = np.zeros((oracle.NSTAT, ty, tx))
    st[oracle.STAT["sx2"]], st[oracle.STAT["sy2"]], st[oracle.STAT["kt2"]] = sx2, sy2, kt2
    return st


@pytest.mark.parametrize("radius", [1, 2, 3])
def test_scatter_with_block_sized_splats_is_the_gather(oracle, radius):
    """Splats of edge 2R + 1 around samples whose offsets lie strictly inside (0, 1) cover exactly
    the pixels whose gather block holds the sample, so the scatter image is the gather image."""
    wl = S.make_workload("c1")
    s = wl.stream
    keep = (s.x != np.floor(s.x)) & (s.y != np.floor(s.y))
    buf, _ = oracle.build_buffer(s.select(keep), wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    p = oracle.Params(t_now=wl.t_now, radius=radius)
    st = oracle.estimate(buf, p)
    size = np.full((wl.height, wl.width), 2 * radius + 1, np.float32)
    rgb, aux, (n, ms) = oracle.scatter(buf, st, p, size, 16.0)
    grgb, gaux = oracle.reconstruct(buf, st, p)
    np.testing.assert_allclose(rgb, grgb, rtol=0, atol=1e-12)
    np.testing.assert_allclose(aux[0], gaux[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(aux[1], gaux[1], rtol=1e-12)
    # every covering splat is a slot of the block: n is the block's slot count
    c = buf.count.astype(np.int64)
    pad = np.pad(c, radius)
    block = sum(pad[radius + dy:radius + dy + wl.height, radius + dx:radius + dx + wl.width]
                for dy in range(-radius, radius + 1) for dx in range(-radius, radius + 1))
    np.testing.assert_array_equal(n, block)
    assert np.all(ms[n > 0] == 2 * radius + 1)


def test_lone_sample_paints_its_footprint(oracle):
    """Sample at (5.3, 7.8), splat edge 3 (half-width 1.5): covers the pixels whose centres lie
    within 1.5 px in x and y, i.e. columns 4..6 and rows 6..8, with its own colour; the rest of the
    image is a hole (0, coverage 0)."""
    w, h = 12, 12
    buf = _single(oracle, w, h, 5.3, 7.8, 6.0, (0.25, 0.5, 0.75))
    p = oracle.Params(t_now=10.0)
    st = _flat_stats(oracle, w, h, p)
    size = np.full((h, w), 3.0, np.float32)
    rgb, aux, (n, ms) = oracle.scatter(buf, st, p, size, 16.0)
    cov = np.zeros((h, w), bool)
    cov[6:9, 4:7] = True
    np.testing.assert_array_equal(n, cov.astype(np.float32))
    np.testing.assert_array_equal(ms, np.where(cov, 3.0, 0.0))
    for c, v in enumerate((0.25, 0.5, 0.75)):
        np.testing.assert_allclose(rgb[c][cov], v, rtol=1e-15)
        assert np.all(rgb[c][~cov] == 0.0)
    assert np.all(aux[1][cov] == 1.0) and np.all(aux[:, ~cov] == 0.0)
    # the splat size of the sample's own pixel decides, and max_size caps it
    size2 = size.copy()
    size2[7, 5] = 9.0
    _, _, (n2, _) = oracle.scatter(buf, st, p, size2, 5.0)
    assert n2.sum() == 25 and n2[5:10, 3:8].sum() == 25


@pytest.mark.parametrize("size,expect_n", [(1.0, 1), (2.5, 9), (5.0, 25), (7.0, 49)])
def test_coverage_of_a_regular_grid(oracle, size, expect_n):
    """One sample at every pixel centre: d = q - p exactly, so a splat of edge s covers the
    (2 floor(s/2) + 1)^2 nearest pixel centres; the interior coverage count is that number and the
    mean size is s."""
    w, h = 20, 16
    buf = oracle.Buffer.empty(w, h, 1, fp16=False, t_ref=10.0)
    buf.ox[:], buf.oy[:], buf.ta[:] = 0.5, 0.5, 9.0
    buf.r[:] = buf.g[:] = buf.b[:] = 0.5
    buf.count[:] = 1
    buf.src[:] = 0
    p = oracle.Params(t_now=10.0)
    st = _flat_stats(oracle, w, h, p)
    _, _, (n, ms) = oracle.scatter(buf, st, p, np.full((h, w), size, np.float32), 16.0)
    r = int(np.floor(size / 2))
    assert np.all(n[r:h - r, r:w - r] == expect_n)
    assert n[0, 0] == (r + 1) ** 2
    assert np.all(ms == np.float32(size))


def test_splat_size_rule(oracle):
    """Sec. 6.2: the previous mean size, x4 where fewer than 4 splats arrived, x0.7 where more than
    32 did; the default where none arrived or there is no previous image; clamped; multiples of
    1/256 px."""
    sp = oracle.SplatParams(size_default=5.0, size_min=1.0, size_max=16.0)
    n = np.array([[0, 2, 4, 20, 32, 33, 100, 3, 50]], np.float32)
    m = np.array([[0, 1.5, 3.0, 6.0, 2.0, 5.0, 1.25, 6.0, 1.0]], np.float32)
    out = oracle.splat_sizes(9, 1, (n, m), sp)
    expect = [16.0,          # nothing arrived: default 5 x 4 = 20, clamped to 16
              6.0,           # 1.5 x 4
              3.0, 6.0, 2.0,  # within [4, 32]: unchanged
              3.5,           # 5 x 0.7 = 3.4999998 in binary32, rounded to 1/256 px
              1.0,           # 1.25 x 0.7 = 0.875, clamped to the minimum
              16.0,          # 6 x 4 = 24, clamped to the maximum
              1.0]           # 1.0 x 0.7 = 0.7, clamped to the minimum
    np.testing.assert_array_equal(out[0], np.array(expect, np.float32))
    assert np.all(oracle.splat_sizes(4, 3, None, sp) == 5.0)
    q = oracle.splat_sizes(1, 1, (np.array([[40.0]], np.float32), np.array([[3.3]], np.float32)),
                           oracle.SplatParams(size_min=0.1))
    assert q[0, 0] == np.float32(np.rint(np.float32(3.3) * np.float32(0.7) * 256) / 256)
