"""Pins of the FP64 reference's deep-buffer build (Sec. 4 per-pixel queues; Sec. 5.2 stream).

The reference replays queue insertion; these tests check it against a sort-and-take-top-K brute
force, counting invariants, and NumPy's binary16 conversion.
"""
import numpy as np
import pytest

import afr_scenes as S


def _stream(rng, n, w, h, t_levels=None, t_max=10.0):
    x = (rng.random(n) * w).astype(np.float32)
    y = (rng.random(n) * h).astype(np.float32)
    if t_levels is not None:  # few distinct times: many ties on t
        t = rng.choice(np.asarray(t_levels, np.float32), n)
    else:
        t = (rng.random(n) * t_max).astype(np.float32)
    c = rng.random((3, n)).astype(np.float32)
    return S.Stream(x, y, t, c[0], c[1], c[2])


def _brute_force(stream, w, h, k, t_ref):
    """Per pixel: sort valid samples by (t, index) descending, keep the first k."""
    x, y, t = stream.x, stream.y, stream.t
    per = {}
    dropped = 0
    for i in range(len(stream)):
        f = [stream.x[i], stream.y[i], stream.t[i], stream.r[i], stream.g[i], stream.b[i]]
        if not all(np.isfinite(f)) or not (0 <= x[i] < w and 0 <= y[i] < h) or t[i] > t_ref:
            dropped += 1
            continue
        per.setdefault((int(np.floor(y[i])), int(np.floor(x[i]))), []).append((float(t[i]), i))
    src = np.full((h, w, k), -1, np.int64)
    count = np.zeros((h, w), np.int64)
    for (j, i), lst in per.items():
        lst.sort(reverse=True)
        top = [idx for _, idx in lst[:k]]
        count[j, i] = len(top)
        src[j, i, :len(top)] = top
    return src, count, dropped, per


@pytest.mark.parametrize("seed,k,levels", [(0, 3, None), (1, 2, [1.0, 2.0, 3.0]), (2, 4, [5.0]),
                                           (3, 1, None), (4, 7, [0.5, 0.25])])
def test_build_matches_sorted_top_k(oracle, seed, k, levels):
    rng = np.random.default_rng(seed)
    w, h = 5, 4
    s = _stream(rng, 300, w, h, levels)
    t_ref = float(np.float32(8.0))
    buf, dropped = oracle.build_buffer(s, w, h, k, "fp32", t_ref)
    src, count, d_ref, _ = _brute_force(s, w, h, k, t_ref)
    assert dropped == d_ref
    np.testing.assert_array_equal(buf.count, count)
    np.testing.assert_array_equal(buf.src, src)
    sel = src >= 0
    idx = src[sel]
    np.testing.assert_array_equal(buf.ox[sel], s.x[idx].astype(np.float64) - np.floor(s.x[idx]))
    np.testing.assert_array_equal(buf.oy[sel], s.y[idx].astype(np.float64) - np.floor(s.y[idx]))
    np.testing.assert_array_equal(buf.ta[sel], s.t[idx])
    np.testing.assert_array_equal(buf.r[sel], s.r[idx])
    np.testing.assert_array_equal(buf.b[sel], s.b[idx])
    # empty slots are zero
    assert np.all(buf.r[~sel] == 0) and np.all(buf.ta[~sel] == 0)


def test_build_is_independent_of_stream_order(oracle):
    rng = np.random.default_rng(7)
    s = _stream(rng, 500, 6, 6, None, t_max=4.0)  # distinct times: the key order is the time order
    a, _ = oracle.build_buffer(s, 6, 6, 3, "fp32", 4.0)
    perm = rng.permutation(len(s))
    s2 = s.select(perm)
    b, _ = oracle.build_buffer(s2, 6, 6, 3, "fp32", 4.0)
    np.testing.assert_array_equal(a.count, b.count)
    # stream indices differ after the permutation; map back and compare
    np.testing.assert_array_equal(np.where(b.src >= 0, perm[np.maximum(b.src, 0)], -1), a.src)
    np.testing.assert_array_equal(a.r, b.r)


def test_invalid_samples_are_dropped(oracle):
    w, h = 4, 3
    x = np.array([0.0, 3.999, 4.0, -0.001, 1.5, np.nan, 1.5, 1.5, 2.5, 1.0], np.float32)
    y = np.array([0.0, 2.999, 1.0, 1.00, 3.0, 1.0, 1.5, 1.5, 0.5, np.inf], np.float32)
    t = np.array([1.0, 2.0, 1.0, 1.0, 1.0, 1.0, 5.0, 1.0, 1.0, 1.0], np.float32)
    r = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, np.inf, 0.9, 1.0], np.float32)
    s = S.Stream(x, y, t, r, r.copy(), r.copy())
    buf, dropped = oracle.build_buffer(s, w, h, 2, "fp32", 4.0)
    # kept: 0 (edge 0,0), 1 (3.999, 2.999), 8; dropped: x=W, x<0, y=H, NaN, t>t_ref, inf colour, inf y
    assert dropped == 7
    assert buf.count.sum() == 3
    assert buf.src[0, 0, 0] == 0 and buf.src[2, 3, 0] == 1 and buf.src[0, 2, 0] == 8


def test_count_is_min_of_k_and_arrivals_and_deep_k_keeps_everything(oracle):
    wl = S.make_workload("c0")  # unstratified: occupancy varies, some pixels empty
    s = wl.stream.select(slice(0, 60000))
    occ = np.zeros((wl.height, wl.width), np.int64)
    np.add.at(occ, (np.floor(s.y).astype(int), np.floor(s.x).astype(int)), 1)
    k = 3
    buf, dropped = oracle.build_buffer(s, wl.width, wl.height, k, "fp32", wl.t_ref)
    assert dropped == 0
    np.testing.assert_array_equal(buf.count, np.minimum(occ, k))
    # A depth at least the largest occupancy never evicts: the buffer holds the whole stream, which
    # is the reconstructor's global newest-N queue of Sec. 5.2.
    kd = int(occ.max())
    full, _ = oracle.build_buffer(s, wl.width, wl.height, kd, "fp32", wl.t_ref)
    np.testing.assert_array_equal(full.count, occ)
    kept = np.sort(full.src[full.src >= 0])
    np.testing.assert_array_equal(kept, np.arange(len(s)))
    # slots are newest first in every pixel
    filled = np.arange(kd)[None, None, :] < full.count[:, :, None]
    t = np.where(filled, full.ta, -np.inf)
    assert np.all(np.diff(t, axis=2)[filled[:, :, 1:]] <= 0)


def test_f16_round_matches_numpy_binary16(oracle):
    rng = np.random.default_rng(11)
    mags = np.concatenate([
        rng.random(3000),                              # [0, 1)
        10.0 ** rng.uniform(-9, 5, 3000),              # across binades incl. binary16 subnormals
        np.array([65504, 65519.99, 65520, 65536, 1e9, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26,
                  2.0 ** -14, 2.0 ** -14 - 2.0 ** -25, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11]),
    ])
    v32 = (mags * rng.choice([-1, 1], mags.size)).astype(np.float32)
    ours = oracle.f16_round(v32.astype(np.float64))
    ref = v32.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(ours, ref)


def test_fp16_build_stores_binary16_of_the_fp32_values(oracle):
    wl = S.make_workload("c1")
    buf32, _ = oracle.build_buffer(wl.stream, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    buf16, _ = oracle.build_buffer(wl.stream, wl.width, wl.height, wl.k, "fp16", wl.t_ref)
    np.testing.assert_array_equal(buf32.src, buf16.src)
    sel = buf32.src >= 0
    h = lambda a: a.astype(np.float32).astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(buf16.ox[sel], h(buf32.ox[sel]))
    np.testing.assert_array_equal(buf16.r[sel], h(buf32.r[sel]))
    age32 = (np.float32(wl.t_ref) - buf32.ta[sel].astype(np.float32)).astype(np.float32)
    np.testing.assert_array_equal(buf16.ta[sel], h(age32))


def _with_velocity(s, vx, vy):
    return S.Stream(*s.arrays(), np.asarray(vx, np.float32), np.asarray(vy, np.float32))


def test_reprojection_with_zero_velocity_is_the_plain_build(oracle):
    rng = np.random.default_rng(31)
    s = _stream(rng, 3000, 19, 13)
    z = np.zeros(len(s), np.float32)
    for precision in ("fp32", "fp16"):
        a, da = oracle.build_buffer(s, 19, 13, 5, precision, 10.0)
        b, db = oracle.build_buffer(_with_velocity(s, z, z), 19, 13, 5, precision, 10.0,
                                    reproject=True)
        assert da == db
        for f in ("ox", "oy", "ta", "r", "g", "b", "count", "src"):
            np.testing.assert_array_equal(getattr(a, f), getattr(b, f), err_msg=f)


def test_reprojection_moves_samples_by_whole_pixels(oracle):
    """Velocities that displace every sample by an exact whole number of pixels by t_ref (binary32
    arithmetic is exact here: dyadic velocities and ages) land each sample on the shifted pixel with
    the same sub-pixel offset; samples moved outside the image are dropped."""
    w, h, t_ref = 16, 8, 32.0
    x = np.array([0.25, 3.5, 15.75, 7.125], np.float32)
    y = np.array([0.5, 2.25, 7.5, 4.0], np.float32)
    t = np.array([24.0, 28.0, 30.0, 16.0], np.float32)          # ages 8, 4, 2, 16 ms
    vx = np.array([0.25, -0.5, 0.5, 0.0], np.float32)          # +2, -2, +1 (out), 0 px
    vy = np.array([0.125, 0.25, 0.0, -0.1875], np.float32)     # +1, +1, 0, -3 px
    c = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    s = S.Stream(x, y, t, c, c, c, vx, vy)
    buf, dropped = oracle.build_buffer(s, w, h, 2, "fp32", t_ref, reproject=True)
    assert dropped == 1                                          # 15.75 + 1 >= 16
    expect = {(1, 2): 0, (3, 1): 1, (1, 7): 3}                   # (y, x) of the new home pixel
    assert int(buf.count.sum()) == 3
    for (py, px), i in expect.items():
        assert buf.count[py, px] == 1
        assert buf.src[py, px, 0] == i
        assert buf.ox[py, px, 0] == x[i] - np.floor(x[i])
        assert buf.oy[py, px, 0] == y[i] - np.floor(y[i])


def test_reprojection_matches_binary32_advection_brute_force(oracle):
    """Random velocities: the reprojected build equals the plain build of a stream whose positions
    were advanced in binary32 (subtract, multiply, add, each rounded) outside the reference."""
    rng = np.random.default_rng(32)
    w, h, t_ref = 23, 17, 40.0
    s = _stream(rng, 4000, w, h, t_max=t_ref)
    vx = (rng.standard_normal(len(s)) * 0.2).astype(np.float32)
    vy = (rng.standard_normal(len(s)) * 0.2).astype(np.float32)
    d = (np.float32(t_ref) - s.t).astype(np.float32)
    xa = (s.x + (vx * d).astype(np.float32)).astype(np.float32)
    ya = (s.y + (vy * d).astype(np.float32)).astype(np.float32)
    moved = S.Stream(xa, ya, s.t, s.r, s.g, s.b)
    for precision in ("fp32", "fp16"):
        a, da = oracle.build_buffer(_with_velocity(s, vx, vy), w, h, 6, precision, t_ref,
                                    reproject=True)
        b, db = oracle.build_buffer(moved, w, h, 6, precision, t_ref)
        assert da == db > 0
        for f in ("ox", "oy", "ta", "r", "g", "b", "count", "src"):
            np.testing.assert_array_equal(getattr(a, f), getattr(b, f), err_msg=f)
