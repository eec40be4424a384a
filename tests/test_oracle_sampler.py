"""Pins of the FP64 reference's sampler feedback statistics and tile selection (Sec. 4, 4.1, 6.1)."""
import numpy as np
import pytest

import afr_scenes as S


def _buffer(oracle, w, h, k, counts, ages, t_now=100.0):
    buf = oracle.Buffer.empty(w, h, k, fp16=False, t_ref=t_now)
    for j in range(h):
        for i in range(w):
            n = counts[j][i]
            buf.count[j, i] = n
            for s in range(n):
                buf.ta[j, i, s] = t_now - ages[s % len(ages)]
                buf.src[j, i, s] = 0
    return buf


def _stats(oracle, w, h, tile, **planes):
    ty, tx = oracle.tiles_shape(w, h, tile)
    st = np.zeros((oracle.NSTAT, ty, tx))
    for name, v in planes.items():
        st[oracle.STAT[name]] = v
    return st


@pytest.mark.parametrize("m,u1", [(1.0, 0.5), (2.0, 0.0), (0.5, 0.75)])
def test_two_tile_undersampling_and_error(oracle, m, u1):
    """Two one-pixel tiles, depth 4: one full, one holding a single sample. 8 slots, 5 samples: 1.5
    empty per tile on average; the full tile has u = 0, the other u = 1 - min(1, 1.5 m / 3). With
    v = (0.2, 0.05): E_0 = 0.8 kappa, E_1 = 0.2 kappa + lambda (its u is all of sum u when > 0)."""
    buf = _buffer(oracle, 2, 1, 4, [[4, 1]], [5.0])
    st = _stats(oracle, 2, 1, 1, var=np.array([[0.2, 0.05]]))
    p = oracle.Params(t_now=100.0, tile=1)
    sp = oracle.SamplerParams(kappa=0.7, lam=0.3, m=m)
    E, u, g = oracle.sampler_stats(buf, st, p, sp)
    np.testing.assert_allclose(u[0], [0.0, u1], rtol=0, atol=1e-15)
    assert g["mean_empty"] == 1.5
    np.testing.assert_allclose(g["sum_v"], 0.25, rtol=1e-15)
    e1 = 0.2 * 0.7 + (0.3 if u1 > 0 else 0.0)
    np.testing.assert_allclose(E[0], [0.8 * 0.7, e1], rtol=1e-14)


def test_error_shares_sum_to_the_weights(oracle):
    """On any buffer with some variation and some undersampling, sum over tiles of E_T / s_T is
    kappa + lambda (each share is normalised by its sum over tiles); clipped border tiles count
    their own size."""
    wl = S.make_workload("c1")
    rng = np.random.default_rng(4)
    keep = rng.random(len(wl.stream)) < 0.3   # a sparse sampler buffer: undersampled tiles
    buf, _ = oracle.build_buffer(wl.stream.select(keep), 60, 44, 4, "fp32", wl.t_ref)
    p = oracle.Params(t_now=wl.t_now, tile=8)
    st = oracle.estimate(buf, p)
    sp = oracle.SamplerParams(kappa=0.6, lam=0.25, m=1.0)
    E, u, g = oracle.sampler_stats(buf, st, p, sp)
    assert g["sum_v"] > 0 and g["sum_u"] > 0
    ty, tx = E.shape
    sizes = np.outer([8] * (ty - 1) + [44 - 8 * (ty - 1)], [8] * (tx - 1) + [60 - 8 * (tx - 1)])
    np.testing.assert_allclose((E / sizes).sum(), 0.85, rtol=1e-13)
    assert np.all((u >= 0) & (u <= 1))


def test_gain_control(oracle):
    """Gradients (G_x, G_y, G_t) = (0.02, 0.04, 0.001) everywhere and sample ages 10 and 30 ms: dC/ds
    = 0.03, dC/dt = 0.001, T = 20 ms, S = i dC/dt T / dC/ds = 2i/3 and the target tile count is
    w h / S^2; static content (G_t = 0) asks for the finest tiling (S = 0, unbounded tile count)."""
    w, h = 16, 8
    buf = _buffer(oracle, w, h, 4, [[2] * w for _ in range(h)], [10.0, 30.0])
    p = oracle.Params(t_now=100.0, tile=8)
    for gain in (1.0, 3.0):
        st = _stats(oracle, w, h, 8, gx=0.02, gy=0.04, gt=0.001)
        _, _, g = oracle.sampler_stats(buf, st, p, oracle.SamplerParams(gain=gain))
        np.testing.assert_allclose([g["dcds"], g["dcdt"], g["mean_age"]], [0.03, 0.001, 20.0],
                                   rtol=1e-14)
        np.testing.assert_allclose(g["S"], 2.0 * gain / 3.0, rtol=1e-13)
        np.testing.assert_allclose(g["target_tiles"], w * h / (2.0 * gain / 3.0) ** 2, rtol=1e-13)
    st = _stats(oracle, w, h, 8, gx=0.02, gy=0.04, gt=0.0)
    _, _, g = oracle.sampler_stats(buf, st, p, oracle.SamplerParams())
    assert g["S"] == 0.0 and np.isinf(g["target_tiles"])


def _rnd(rng, n):
    return rng.integers(0, 2 ** 32, 3 * n, dtype=np.uint64).astype(np.uint32)


def test_selection_by_hand(oracle):
    """Tiles 0 and 1 (8 x 8 each) with E = (1, 3): q = (floor(2^24 / 3), 2^24) = (5592405, 16777216).
    The first tile takes the draws with (r Q) >> 24 < 5592405, r = rnd >> 8."""
    E = np.array([[1.0, 3.0]], np.float32)
    Q = 5592405 + 16777216
    r_edge = -(-5592405 * 2 ** 24 // Q)          # smallest r whose target reaches tile 1
    rs = np.array([0, r_edge - 1, r_edge, 2 ** 24 - 1], np.uint64)
    rnd = np.concatenate([rs << 8, np.zeros(4, np.uint64), (np.full(4, 2 ** 24 - 1, np.uint64)) << 8])
    x, y, t = oracle.sampler_select(16, 8, 8, E, rnd.astype(np.uint32))
    np.testing.assert_array_equal(t, [0, 0, 1, 1])
    np.testing.assert_array_equal(x, np.float32([0, 0, 8, 8]))
    # u2 = 1 - 2^-24: y = 8 (1 - 2^-24) rounds to the float just below 8 (exact scaling by 8)
    assert np.all(y == np.float32(8 * (1 - 2.0 ** -24)))


def test_selection_frequencies_and_spots(oracle):
    """Tile frequencies follow E (within 5 sigma over 400K draws), spots fall inside their (clipped)
    tiles, and uniform E (all zero) gives every tile the same weight."""
    rng = np.random.default_rng(17)
    w, h, B = 21, 10, 8                       # tiles 3 x 2, the last column and row clipped
    E = np.array([[1.0, 2.0, 0.0], [3.0, 4.0, 5.0]], np.float32)
    n = 400_000
    x, y, t = oracle.sampler_select(w, h, B, E, _rnd(rng, n))
    p = E.reshape(-1) / E.sum()
    f = np.bincount(t, minlength=6) / n
    assert np.all(np.abs(f - p) <= 5 * np.sqrt(p * (1 - p) / n) + 1e-7)
    tx, ty = t % 3, t // 3
    assert np.all((x >= tx * B) & (x < np.minimum((tx + 1) * B, w)))
    assert np.all((y >= ty * B) & (y < np.minimum((ty + 1) * B, h)))
    # spots are uniform inside the tile: mean offset half the clipped width
    last = t == 5
    np.testing.assert_allclose((x[last] - 16).mean(), 2.5, atol=0.02)
    _, _, t0 = oracle.sampler_select(w, h, B, np.zeros((2, 3), np.float32), _rnd(rng, 60_000))
    f0 = np.bincount(t0, minlength=6) / 60_000
    assert np.all(np.abs(f0 - 1 / 6) < 0.01)


def test_spot_never_reaches_the_far_edge(oracle):
    """A tile at x0 = 632 of clipped width 3 with u1 = 1 - 2^-24: 632 + 3 u1 rounds to 635 in
    binary32, so the spot is moved to the float below 635 (still inside the image)."""
    w, h, B = 635, 8, 8
    E = np.zeros((1, 80), np.float32)
    E[0, 79] = 1.0
    rnd = np.array([0, (2 ** 24 - 1) << 8, 0], np.uint64).astype(np.uint32)
    x, y, t = oracle.sampler_select(w, h, B, E, rnd)
    assert t[0] == 79 and x[0] == np.nextafter(np.float32(635), np.float32(0)) and y[0] == 0


def test_equal_error_tiles_one_part_is_uniform_by_area(oracle):
    rng = np.random.default_rng(21)
    w, h, B = 37, 29, 8
    E = rng.random(oracle.tiles_shape(w, h, B)).astype(np.float32)
    P = oracle.sampler_tile_weights(w, h, B, E, n_parts=1)
    ty, tx = E.shape
    area = np.outer([8] * (ty - 1) + [h - 8 * (ty - 1)], [8] * (tx - 1) + [w - 8 * (tx - 1)])
    np.testing.assert_allclose(P, area / (w * h), rtol=1e-7)
    # no error anywhere: uniform by area whatever the part count
    P0 = oracle.sampler_tile_weights(w, h, B, np.zeros_like(E), n_parts=7)
    np.testing.assert_array_equal(P0, area.astype(np.float32))


def test_equal_error_tiles_follow_the_z_curve(oracle):
    """4 x 4 tiles, error 1 on the top-left 2 x 2 quadrant (the first four tiles on the Z-curve),
    four parts: the first three quadrant tiles are parts of their own (weight 1), the fourth shares
    the last part with the 12 error-free tiles (weight 1/13 each). A row-major order would give the
    tile below the top-left corner 1/3 instead."""
    E = np.zeros((4, 4), np.float32)
    E[:2, :2] = 1.0
    P = oracle.sampler_tile_weights(32, 32, 8, E, n_parts=4)
    assert P[0, 0] == 1.0 and P[0, 1] == 1.0 and P[1, 0] == 1.0
    rest = np.ones((4, 4), bool)
    rest[0, 0] = rest[0, 1] = rest[1, 0] = False
    np.testing.assert_allclose(P[rest], 1.0 / 13.0, rtol=1e-7)
    np.testing.assert_allclose(P.sum(), 4.0, rtol=1e-6)


def test_equal_error_tiles_equal_errors_and_a_dominant_tile(oracle):
    """Equal errors with as many parts as tiles: one part per tile, weight 1 each. All error in one
    tile (in the middle of the curve): that tile takes N - 2 whole parts plus its share of the
    first run; the error-free tiles before and after it share the first and the last part. The
    weights always sum to N, and the gain target rounds and clamps into [1, tiles]."""
    E = np.ones((6, 8), np.float32)
    np.testing.assert_array_equal(oracle.sampler_tile_weights(64, 48, 8, E, n_parts=48), 1.0)
    E = np.zeros((6, 8), np.float32)
    # tile (x 2, y 3): Z-code spread(2) | spread(3) << 1 = 4 | 10 = 14, and the 14 smaller codes
    # all lie in the top-left 4 x 4 block of the grid: curve position 14 of 48
    E[3, 2] = 5.0
    N = 10
    P = oracle.sampler_tile_weights(64, 48, 8, E, n_parts=N)
    assert P[3, 2] == np.float32(1.0 / 15.0 + (N - 2))
    np.testing.assert_allclose(P.sum(), N, rtol=1e-6)
    np.testing.assert_allclose(P[0, 0], 1.0 / 15.0, rtol=1e-7)   # in the first run (14 + 1 tiles)
    np.testing.assert_allclose(P[5, 7], 1.0 / 33.0, rtol=1e-7)   # in the last run (33 tiles)
    rng = np.random.default_rng(2)
    E = (rng.random((6, 8)) ** 4).astype(np.float32)
    for target, n in ((0.2, 1), (7.4, 7), (7.6, 8), (1e9, 48), (np.inf, 48), (np.nan, 1)):
        P = oracle.sampler_tile_weights(64, 48, 8, E, target=target)
        np.testing.assert_allclose(P.sum(), n, rtol=1e-6)
