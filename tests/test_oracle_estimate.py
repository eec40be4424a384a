"""Pins of the FP64 reference's gradient, density and extent estimates (Sec. 4, 4.1, 5.1).

Each test builds a deep buffer by hand so that the expected statistic has a closed form that does
not go through the reference's own formulas.
"""
import numpy as np
import pytest


def _buffer(oracle, w, h, k, t_now=100.0):
    return oracle.Buffer.empty(w, h, k, fp16=False, t_ref=t_now)


def _fill(buf, j, i, k, *, ox=0.5, oy=0.5, t=0.0, rgb=(0.0, 0.0, 0.0)):
    buf.ox[j, i, k], buf.oy[j, i, k], buf.ta[j, i, k] = ox, oy, t
    buf.r[j, i, k], buf.g[j, i, k], buf.b[j, i, k] = rgb
    buf.count[j, i] = max(buf.count[j, i], k + 1)
    buf.src[j, i, k] = 0


def _grey(v):
    # equal channels: the luminance weights sum to one, so L equals the grey level
    return (v, v, v)


@pytest.mark.parametrize("a,b", [(0.01, 0.02), (-0.013, 0.004), (0.0, -0.02)])
def test_linear_ramp_gives_its_slopes(oracle, a, b):
    w = h = 16
    buf = _buffer(oracle, w, h, 2)
    for j in range(h):
        for i in range(w):
            L = 0.4 + a * (i + 0.5) + b * (j + 0.5)
            for k, t in enumerate((90.0, 80.0)):  # same colour at two times: static
                _fill(buf, j, i, k, t=t, rgb=_grey(L))
    p = oracle.Params(t_now=100.0, tile=8)
    ps = oracle.pixel_stats(buf, p)
    np.testing.assert_allclose(ps["gx"], abs(a), rtol=0, atol=1e-13)
    np.testing.assert_allclose(ps["gy"], abs(b), rtol=0, atol=1e-13)
    np.testing.assert_allclose(ps["gt"], 0.0, atol=1e-13)
    st = oracle.estimate(buf, p)
    np.testing.assert_allclose(st[oracle.STAT["gx"]], abs(a), atol=1e-13)
    np.testing.assert_allclose(st[oracle.STAT["gy"]], abs(b), atol=1e-13)
    assert np.all(st[oracle.STAT["gt"]] == 0.0)


@pytest.mark.parametrize("c", [0.004, -0.0025])
def test_luminance_linear_in_time_gives_its_rate(oracle, c):
    """Fixed positions, L = L0 + c t: the new-half/old-half difference quotient is exactly |c|."""
    w, h, k = 8, 8, 5
    buf = _buffer(oracle, w, h, k)
    rng = np.random.default_rng(3)
    for j in range(h):
        for i in range(w):
            ts = np.sort(rng.uniform(20.0, 99.0, k))[::-1]  # newest first
            for s, t in enumerate(ts):
                _fill(buf, j, i, s, ox=0.3, oy=0.7, t=t, rgb=_grey(0.5 + c * (t - 60.0)))
    p = oracle.Params(t_now=100.0)
    ps = oracle.pixel_stats(buf, p)
    np.testing.assert_allclose(ps["gt"], abs(c), rtol=1e-12)
    st = oracle.estimate(buf, p)
    np.testing.assert_allclose(st[oracle.STAT["gt"]], abs(c), rtol=1e-12)


def test_rank_split_uses_ceil_half(oracle):
    """n = 3: the new half holds ranks {0, 1}, the old half rank {2}."""
    buf = _buffer(oracle, 1, 1, 3)
    for s, (t, L) in enumerate(((99.0, 0.9), (97.0, 0.7), (90.0, 0.2))):
        _fill(buf, 0, 0, s, t=t, rgb=_grey(L))
    ps = oracle.pixel_stats(buf, oracle.Params(t_now=100.0))
    new_l, old_l = (0.9 + 0.7) / 2, 0.2
    new_a, old_a = (1.0 + 3.0) / 2, 10.0
    assert ps["gt"][0, 0] == pytest.approx(abs(new_l - old_l) / (old_a - new_a), rel=1e-14)


def test_constant_colour_has_no_gradient_and_no_variance(oracle):
    w, h, k = 12, 10, 4
    buf = _buffer(oracle, w, h, k)
    rng = np.random.default_rng(5)
    for j in range(h):
        for i in range(w):
            for s in range(rng.integers(1, k + 1)):
                _fill(buf, j, i, s, ox=rng.random(), oy=rng.random(), t=rng.uniform(0, 99),
                      rgb=(0.25, 0.5, 0.75))
    st = oracle.estimate(buf, oracle.Params(t_now=100.0, tile=4))
    L = 0.2126 * 0.25 + 0.7152 * 0.5 + 0.0722 * 0.75
    for name in ("gx", "gy", "gt", "var"):
        np.testing.assert_allclose(st[oracle.STAT[name]], 0.0, atol=1e-15)
    np.testing.assert_allclose(st[oracle.STAT["lmean"]], L, rtol=1e-14)
    # no temporal change: the temporal filter is flat and the spatial std sits at e_min
    np.testing.assert_array_equal(st[oracle.STAT["kt2"]], 0.0)
    np.testing.assert_allclose(st[oracle.STAT["sx2"]], 0.25, rtol=0, atol=0)


def test_sample_volume_from_an_age_grid(oracle):
    """Every pixel holds samples of ages {1, 3, 5, 7} ms: mean age 4, span 8 ms, 4 samples per
    px over 8 ms gives R_l = 0.5 per px ms and V = 2 px ms per sample (Sec. 5.1)."""
    w = h = 8
    buf = _buffer(oracle, w, h, 4)
    for j in range(h):
        for i in range(w):
            for s, age in enumerate((1.0, 3.0, 5.0, 7.0)):
                _fill(buf, j, i, s, t=100.0 - age, rgb=_grey(0.5))
    st = oracle.estimate(buf, oracle.Params(t_now=100.0))
    assert st[oracle.STAT["vol"]][0, 0] == pytest.approx(2.0, rel=1e-14)
    # half the pixels with only the two newest samples: 3 samples/px on average, mean age 10/3 ...
    buf2 = _buffer(oracle, w, h, 4)
    for j in range(h):
        for i in range(w):
            ages = (1.0, 3.0, 5.0, 7.0) if (i + j) % 2 == 0 else (1.0, 3.0)
            for s, age in enumerate(ages):
                _fill(buf2, j, i, s, t=100.0 - age, rgb=_grey(0.5))
    st2 = oracle.estimate(buf2, oracle.Params(t_now=100.0))
    n_t, area = 32 * 4 + 32 * 2, 64
    abar = (32 * 16.0 + 32 * 4.0) / n_t
    assert st2[oracle.STAT["vol"]][0, 0] == pytest.approx(area * 2 * abar / n_t, rel=1e-14)


def test_variance_of_two_valued_luminance(oracle):
    """Equal ages make the age weights equal, so v_T is the variance of a two-point
    distribution: p (1 - p) (L1 - L2)^2 (Sec. 4 tile variation)."""
    w = h = 8
    buf = _buffer(oracle, w, h, 2)
    n1 = 0
    for j in range(h):
        for i in range(w):
            for s in range(2):
                hi = (i * 2 + s + j) % 5 == 0
                n1 += hi
                _fill(buf, j, i, s, t=50.0, rgb=_grey(0.9 if hi else 0.3))
    st = oracle.estimate(buf, oracle.Params(t_now=100.0))
    p1 = n1 / 128
    assert st[oracle.STAT["var"]][0, 0] == pytest.approx(p1 * (1 - p1) * 0.6 ** 2, rel=1e-12)
    assert st[oracle.STAT["lmean"]][0, 0] == pytest.approx(p1 * 0.9 + (1 - p1) * 0.3, rel=1e-13)


def test_tile_gradient_is_age_weighted(oracle):
    """Two 1-px-wide columns with different temporal rates and different ages: the tile average
    weighs each pixel by the summed e^{-3.47 a} of its samples, a in seconds (Sec. 4.1)."""
    buf = _buffer(oracle, 2, 1, 2)
    ages = {0: (2.0, 40.0), 1: (300.0, 500.0)}     # ms
    rates = {0: 0.001, 1: 0.003}
    for i in (0, 1):
        for s, a in enumerate(ages[i]):
            _fill(buf, 0, i, s, t=1000.0 - a, rgb=_grey(0.5 - rates[i] * a))
    p = oracle.Params(t_now=1000.0, tile=8)
    w = [sum(np.exp(-3.47 * a / 1000.0) for a in ages[i]) for i in (0, 1)]
    expect = (w[0] * rates[0] + w[1] * rates[1]) / (w[0] + w[1])
    st = oracle.estimate(buf, p)
    assert st[oracle.STAT["gt"]][0, 0] == pytest.approx(expect, rel=1e-12)


def test_missing_neighbours_are_skipped(oracle):
    """A pixel with an empty left neighbour uses only its right difference; an isolated pixel has
    no spatial gradient and does not enter the tile average."""
    buf = _buffer(oracle, 4, 1, 1)
    _fill(buf, 0, 0, 0, t=90, rgb=_grey(0.1))       # isolated (pixel 1 empty)
    _fill(buf, 0, 2, 0, t=90, rgb=_grey(0.2))
    _fill(buf, 0, 3, 0, t=90, rgb=_grey(0.5))
    ps = oracle.pixel_stats(buf, oracle.Params(t_now=100.0))
    assert np.isnan(ps["gx"][0, 0]) and np.isnan(ps["gx"][0, 1])
    assert ps["gx"][0, 2] == pytest.approx(0.3) and ps["gx"][0, 3] == pytest.approx(0.3)
    st = oracle.estimate(buf, oracle.Params(t_now=100.0))
    assert st[oracle.STAT["gx"]][0, 0] == pytest.approx(0.3, rel=1e-14)
    assert st[oracle.STAT["gt"]][0, 0] == 0.0  # one sample per pixel: no temporal estimate


def test_empty_tile(oracle):
    buf = _buffer(oracle, 16, 8, 2)
    for j in range(8):
        for i in range(8):
            _fill(buf, j, i, 0, t=90, rgb=_grey(0.5))
    st = oracle.estimate(buf, oracle.Params(t_now=100.0))
    assert np.isinf(st[oracle.STAT["vol"]][0, 1])
    assert st[oracle.STAT["sx2"]][0, 1] == 0.25 and st[oracle.STAT["kt2"]][0, 1] == 0.0


@pytest.mark.parametrize("g", [(0.1, 0.2, 0.01, 4.0), (0.7, 0.05, 0.3, 0.5), (1e-3, 2.0, 5.0, 37.0)])
def test_extents_satisfy_the_paper_constraints(oracle, g):
    """Test mode (no floors, no clamp, sigma = tau = 1): e_x G_x = e_y G_y = e_t G_t and
    e_x e_y e_t = V with e_t = 1 / k_t (Sec. 5.1)."""
    gx, gy, gt, vol = g
    p = oracle.Params(g_floor=0.0, e_min=0.0, e_max=np.inf, sigma=1.0, tau=1.0)
    e = oracle.extents(gx, gy, gt, vol, p)
    ex, ey, et = np.sqrt(e["ex2"]), np.sqrt(e["ey2"]), 1.0 / np.sqrt(e["kt2"])
    assert ex * ey * et == pytest.approx(vol, rel=1e-13)
    assert ex * gx == pytest.approx(ey * gy, rel=1e-13)
    assert ex * gx == pytest.approx(et * gt, rel=1e-13)
    assert e["sx2"] == pytest.approx(e["ex2"], rel=1e-15)


def test_extents_are_unit_covariant(oracle):
    """Measuring time in seconds instead of ms scales G_t by 1000 and V by 1/1000: spatial extents
    are unchanged and the temporal rate scales by 1000."""
    p = oracle.Params()
    a = oracle.extents(0.05, 0.2, 0.01, 4.0, p)
    b = oracle.extents(0.05, 0.2, 0.01 * 1000.0, 4.0 / 1000.0, p)
    for n in ("ex2", "ey2", "sx2", "sy2"):
        assert a[n] == pytest.approx(b[n], rel=1e-13)
    assert b["kt2"] == pytest.approx(a["kt2"] * 1e6, rel=1e-13)


def test_extents_clamp_limits(oracle):
    p = oracle.Params(e_min=0.5, e_max=1.0)
    lo = oracle.extents(0.3, 0.3, 0.0, 4.0, p)   # static: floor width, flat in time
    assert lo["sx2"] == 0.25 and lo["kt2"] == 0.0 and lo["ex2"] == 0.0
    hi = oracle.extents(1e-3, 1e-3, 10.0, 400.0, p.with_(sigma=1e4))
    assert 0.25 < hi["sx2"] < 1.25 and hi["sx2"] == pytest.approx(1.25, rel=1e-6)
    big_gt = oracle.extents(0.1, 0.1, 1.0, 4.0, p)
    small_gt = oracle.extents(0.1, 0.1, 0.001, 4.0, p)
    # a larger temporal gradient gives a shorter temporal filter and a wider spatial one (Sec. 5.1)
    assert big_gt["kt2"] > small_gt["kt2"] and big_gt["sx2"] > small_gt["sx2"]


def test_extents_large_volume_limit(oracle):
    """V = +inf with a temporal gradient (crosshair gradients over a tile with no buffered samples)
    gives the limit of the extents as V grows (Sec. 5.1): ex2, ey2 -> inf, the clamped width at its
    ceiling e_min^2 + e_max^2, kt2 -> 0; with no clamp the width is infinite."""
    p = oracle.Params(e_min=0.5, e_max=2.0)
    lim = oracle.extents(0.1, 0.3, 0.2, np.inf, p)
    assert lim["ex2"] == np.inf and lim["ey2"] == np.inf and lim["kt2"] == 0.0
    assert lim["sx2"] == 4.25 and lim["sy2"] == 4.25
    prev_kt2 = np.inf
    for v in (1e6, 1e12, 1e24):
        e = oracle.extents(0.1, 0.3, 0.2, v, p)
        z = p.sigma ** 2 * e["ex2"]
        # 4.25 - sx2 = e_max^4 / (e_max^2 + z) < 16 / z, up to rounding of the sum
        assert 0.0 <= lim["sx2"] - e["sx2"] <= 16.0 / z + 1e-15
        assert 0.0 < e["kt2"] < prev_kt2
        prev_kt2 = e["kt2"]
    assert oracle.extents(0.1, 0.3, 0.2, np.inf, p.with_(e_max=np.inf))["sx2"] == np.inf


@pytest.mark.parametrize("g_floor", [0.0, -1e-3])
def test_estimate_requires_a_positive_gradient_floor(oracle, g_floor):
    """With no floor a spatially flat tile that changes in time divides by a zero gradient."""
    buf = oracle.Buffer.empty(16, 8, 2, fp16=False, t_ref=10.0)
    with pytest.raises(ValueError):
        oracle.estimate(buf, oracle.Params(t_now=10.0, g_floor=g_floor))
