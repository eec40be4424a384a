"""Pins of the FP64 reference's gather reconstruction (Sec. 5.1 Gaussian filter, Sec. 5.2 normalised
weighted average, Sec. 5 traditional frameless display) and of its adjoint.

Pins: hand-derived values, invariants (constant colour, convexity, linearity, mirror and shift
covariance), special cases that reduce to a simpler definition computed independently here (a
spatial Gaussian kernel average built on scipy's normal pdf; the newest sample at each pixel), and,
for the adjoint, FP64 central finite differences and the identity <J v, u> = <v, J^T u>.
"""
import json
import os

import numpy as np
import pytest
from scipy import stats as sps

import afr_scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_buffer(oracle, w, h, k, seed, t_now=100.0, fill=1.0, empty_frac=0.0):
    rng = np.random.default_rng(seed)
    buf = oracle.Buffer.empty(w, h, k, fp16=False, t_ref=t_now)
    for j in range(h):
        for i in range(w):
            if rng.random() < empty_frac:
                continue
            n = int(rng.integers(1, k + 1)) if fill < 1.0 else k
            ts = np.sort(rng.uniform(t_now - 60.0, t_now, n))[::-1]
            for s in range(n):
                buf.ox[j, i, s], buf.oy[j, i, s] = rng.random(), rng.random()
                buf.ta[j, i, s] = ts[s]
                buf.r[j, i, s], buf.g[j, i, s], buf.b[j, i, s] = rng.random(3)
                buf.src[j, i, s] = 0
            buf.count[j, i] = n
    return buf


def _random_stats(oracle, w, h, tile, seed):
    rng = np.random.default_rng(seed)
    ty, tx = oracle.tiles_shape(w, h, tile)
    st = np.zeros((oracle.NSTAT, ty, tx))
    st[oracle.STAT["sx2"]] = rng.uniform(0.25, 1.25, (ty, tx))
    st[oracle.STAT["sy2"]] = rng.uniform(0.25, 1.25, (ty, tx))
    st[oracle.STAT["kt2"]] = rng.uniform(0.0, 0.01, (ty, tx))
    st[oracle.STAT["ex2"]] = rng.uniform(0.0, 1.0, (ty, tx))
    st[oracle.STAT["ey2"]] = rng.uniform(0.0, 1.0, (ty, tx))
    return st


def test_golden_two_slot_row(oracle):
    g = json.load(open(os.path.join(GOLDEN, "two_slot_row.json")))
    buf = oracle.Buffer.empty(g["width"], g["height"], g["k"], t_ref=g["t_now"])
    for s in g["slots"]:
        i, j = s["pixel"]
        buf.ox[j, i, 0], buf.oy[j, i, 0], buf.ta[j, i, 0] = s["ox"], s["oy"], s["t"]
        buf.r[j, i, 0], buf.g[j, i, 0], buf.b[j, i, 0] = s["rgb"]
        buf.count[j, i] = 1
    st = np.zeros((oracle.NSTAT, 1, 1))
    st[oracle.STAT["sx2"]], st[oracle.STAT["sy2"]], st[oracle.STAT["kt2"]] = g["sx2"], g["sy2"], g["kt2"]
    p = oracle.Params(t_now=g["t_now"], radius=g["radius"], tile=g["tile"])
    rgb, aux = oracle.reconstruct(buf, st, p)
    np.testing.assert_allclose(rgb, np.array(g["expect_rgb"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(aux[0], np.array(g["expect_emax"]), atol=0)
    np.testing.assert_allclose(aux[1], np.array(g["expect_wsum"]), rtol=1e-15)


def test_constant_colour_is_reproduced(oracle):
    buf = _random_buffer(oracle, 13, 11, 3, 1, fill=0.5)
    buf = buf.with_colours(np.broadcast_to(np.array([0.3, 0.6, 0.9])[:, None, None, None],
                                           (3, 11, 13, 3)))
    st = _random_stats(oracle, 13, 11, 4, 2)
    rgb, aux = oracle.reconstruct(buf, st, oracle.Params(t_now=100.0, tile=4))
    for c, v in enumerate((0.3, 0.6, 0.9)):
        np.testing.assert_allclose(rgb[c], v, rtol=1e-14)
    assert np.all(aux[1] >= 1.0)  # the shifted weights include exp(0) = 1


def test_output_is_a_convex_combination_and_linear_in_colours(oracle):
    w, h, k = 10, 9, 3
    buf = _random_buffer(oracle, w, h, k, 3, fill=0.5)
    st = _random_stats(oracle, w, h, 4, 4)
    p = oracle.Params(t_now=100.0, tile=4, radius=2)
    rgb, _ = oracle.reconstruct(buf, st, p)
    for j in range(h):
        for i in range(w):
            blk = (slice(max(0, j - 2), j + 3), slice(max(0, i - 2), i + 3))
            m = np.arange(k)[None, None, :] < buf.count[blk][:, :, None]
            vals = buf.r[blk][m]
            assert vals.min() - 1e-15 <= rgb[0, j, i] <= vals.max() + 1e-15
    rng = np.random.default_rng(9)
    c1, c2 = rng.random((3, h, w, k)), rng.random((3, h, w, k))
    a, b = 0.7, -1.9
    r1, _ = oracle.reconstruct(buf.with_colours(c1), st, p)
    r2, _ = oracle.reconstruct(buf.with_colours(c2), st, p)
    r12, _ = oracle.reconstruct(buf.with_colours(a * c1 + b * c2), st, p)
    np.testing.assert_allclose(r12, a * r1 + b * r2, atol=1e-13)


def _spatial_gaussian_gather(buf, radius, std):
    """Independent definition for the static case: Gaussian kernel average with a fixed isotropic
    std over the samples whose home pixel lies in the (2R+1)^2 block, built on scipy's pdf."""
    h, w, k = buf.height, buf.width, buf.k
    jj, ii, kk = np.meshgrid(np.arange(h), np.arange(w), np.arange(k), indexing="ij")
    filled = kk < buf.count[:, :, None]
    X = (ii + buf.ox)[filled]
    Y = (jj + buf.oy)[filled]
    HI, HJ = ii[filled], jj[filled]
    cols = np.stack([buf.r[filled], buf.g[filled], buf.b[filled]])
    out = np.zeros((3, h, w))
    for j in range(h):
        for i in range(w):
            m = (np.abs(HI - i) <= radius) & (np.abs(HJ - j) <= radius)
            wts = sps.norm.pdf(X[m], loc=i + 0.5, scale=std) * sps.norm.pdf(Y[m], loc=j + 0.5, scale=std)
            out[:, j, i] = (cols[:, m] * wts).sum(axis=1) / wts.sum()
    return out


def test_static_limit_is_a_spatial_gaussian_gather(oracle):
    """tau = 0 removes the temporal term and pins the spatial std at e_min (Sec. 5.1: static content
    lets old samples count fully)."""
    wl = S.make_workload("c1")
    sub = wl.stream.select((wl.stream.x < 24) & (wl.stream.y < 20))
    buf, _ = oracle.build_buffer(sub, 24, 20, 4, "fp32", wl.t_ref)
    p = oracle.Params(t_now=wl.t_now, tau=0.0, e_min=0.6)
    rgb, _, st = oracle.forward(buf, p)
    assert np.all(st[oracle.STAT["kt2"]] == 0) and np.all(st[oracle.STAT["sx2"]] == 0.36)
    np.testing.assert_allclose(rgb, _spatial_gaussian_gather(buf, 2, 0.6), rtol=0, atol=1e-13)


def test_collocated_static_samples_give_zero_temporal_gradient(oracle):
    """The paper's temporal gradient compares samples at one sub-pixel spot (Sec. 4.1). When each
    pixel re-samples the same spot of a static scene, G_t is exactly 0 and the result equals the
    spatial-only gather."""
    rng = np.random.default_rng(21)
    w, h, k = 16, 16, 4
    scene = S.CheckerDiscScene(cell=3.0, speed=0.0, radius=5.0, x0=8.0, y0=8.0)
    buf = oracle.Buffer.empty(w, h, k, t_ref=100.0)
    for j in range(h):
        for i in range(w):
            ox, oy = rng.random(), rng.random()
            r, g, b = scene.color(np.array([i + ox]), np.array([j + oy]), np.array([0.0]))
            for s, t in enumerate(np.sort(rng.uniform(0, 100, k))[::-1]):
                buf.ox[j, i, s], buf.oy[j, i, s], buf.ta[j, i, s] = ox, oy, t
                buf.r[j, i, s], buf.g[j, i, s], buf.b[j, i, s] = r[0], g[0], b[0]
            buf.count[j, i] = k
    p = oracle.Params(t_now=100.0)
    rgb, _, st = oracle.forward(buf, p)
    assert np.all(st[oracle.STAT["gt"]] == 0.0)
    np.testing.assert_allclose(rgb, _spatial_gaussian_gather(buf, 2, 0.5), atol=1e-13)


def test_single_sample_blocks_return_that_sample(oracle):
    buf = _random_buffer(oracle, 6, 5, 1, 31)
    st = _random_stats(oracle, 6, 5, 8, 32)
    rgb, aux = oracle.reconstruct(buf, st, oracle.Params(t_now=100.0, radius=0))
    np.testing.assert_array_equal(rgb, buf.colours()[..., 0])
    np.testing.assert_array_equal(aux[1], 1.0)
    # a sparse image where every (2R+1)^2 block holds at most one slot
    sp = oracle.Buffer.empty(9, 9, 2, t_ref=100.0)
    for (j, i) in ((0, 0), (0, 6), (6, 3)):
        sp.ox[j, i, 0], sp.oy[j, i, 0], sp.ta[j, i, 0] = 0.2, 0.9, 50.0
        sp.r[j, i, 0], sp.g[j, i, 0], sp.b[j, i, 0] = 0.1 * (i + 1), 0.2, 0.05 * (j + 1)
        sp.count[j, i] = 1
    rgb, aux = oracle.reconstruct(sp, _random_stats(oracle, 9, 9, 8, 33), oracle.Params(t_now=100.0, radius=2))
    assert rgb[0, 1, 1] == sp.r[0, 0, 0] and rgb[2, 5, 4] == sp.b[6, 3, 0]
    # pixels whose block holds nothing are black with zero coverage
    assert rgb[0, 3, 3] == 0 and aux[1, 3, 3] == 0


def test_sharp_temporal_filter_gives_traditional_frameless(oracle):
    """With R = 0 and a very narrow temporal filter, each pixel shows its newest sample: the
    traditional frameless display of Sec. 5."""
    buf = _random_buffer(oracle, 7, 6, 4, 41, fill=0.5)
    st = _random_stats(oracle, 7, 6, 8, 42)
    st[oracle.STAT["kt2"]] = 1e4
    rgb, _ = oracle.reconstruct(buf, st, oracle.Params(t_now=100.0, radius=0))
    np.testing.assert_allclose(rgb, buf.colours()[..., 0], rtol=0, atol=1e-300)


def test_mirror_and_shift_covariance(oracle):
    w, h, k, tile = 16, 8, 3, 4
    buf = _random_buffer(oracle, w, h, k, 51, fill=0.5)
    st = _random_stats(oracle, w, h, tile, 52)
    p = oracle.Params(t_now=100.0, tile=tile)
    rgb, _ = oracle.reconstruct(buf, st, p)
    # mirror in x: pixel i -> W-1-i, offset ox -> 1 - ox, tiles mirrored
    m = oracle.Buffer(w, h, k, False, buf.t_ref, (1.0 - buf.ox)[:, ::-1].copy(), buf.oy[:, ::-1].copy(),
                      buf.ta[:, ::-1].copy(), buf.r[:, ::-1].copy(), buf.g[:, ::-1].copy(),
                      buf.b[:, ::-1].copy(), buf.count[:, ::-1].copy(), buf.src[:, ::-1].copy())
    rgb_m, _ = oracle.reconstruct(m, st[:, :, ::-1].copy(), p)
    np.testing.assert_allclose(rgb_m[:, :, ::-1], rgb, atol=1e-13)
    # shift by one tile in x (away from the border, with the same content)
    pad = lambda a, v: np.concatenate([np.full((h, tile) + a.shape[2:], v, a.dtype), a], axis=1)
    sh = oracle.Buffer(w + tile, h, k, False, buf.t_ref, pad(buf.ox, 0.0), pad(buf.oy, 0.0),
                       pad(buf.ta, 0.0), pad(buf.r, 0.0), pad(buf.g, 0.0), pad(buf.b, 0.0),
                       pad(buf.count, 0), pad(buf.src, -1))
    st_sh = np.concatenate([np.broadcast_to(st[:, :, :1], st[:, :, :1].shape), st], axis=2)
    rgb_s, _ = oracle.reconstruct(sh, st_sh, p)
    np.testing.assert_allclose(rgb_s[:, :, tile + 2:], rgb[:, :, 2:], atol=1e-13)


# ------------------------------------------------------------------------------------------------
# adjoint
# ------------------------------------------------------------------------------------------------

def _small_workload(oracle):
    wl = S.make_workload("c1")
    sub = wl.stream.select((wl.stream.x < 40) & (wl.stream.y < 32) & (wl.stream.x >= 8))
    sub.x = (sub.x - 8).astype(np.float32)
    buf, _ = oracle.build_buffer(sub, 32, 32, 4, "fp32", wl.t_ref)
    target = S.ground_truth(wl.scene, 40, 32, wl.t_now, 4)[:, :, 8:]
    return buf, target, wl.t_now


def test_param_gradients_match_central_differences(oracle):
    buf, target, t_now = _small_workload(oracle)
    p0 = oracle.Params(t_now=t_now, sigma=1.3, tau=0.8)
    h = 1e-3

    def loss(p):
        rgb, _, _ = oracle.forward(buf, p)
        return oracle.rms(rgb, target)

    rgb, aux, st = oracle.forward(buf, p0)
    _, gpar = oracle.backward(buf, st, p0, oracle.rms_grad(rgb, target))
    fd_s = (loss(p0.with_(sigma=p0.sigma + h)) - loss(p0.with_(sigma=p0.sigma - h))) / (2 * h)
    fd_t = (loss(p0.with_(tau=p0.tau + h)) - loss(p0.with_(tau=p0.tau - h))) / (2 * h)
    assert abs(gpar[0]) > 1e-6 and abs(gpar[1]) > 1e-6
    assert gpar[0] == pytest.approx(fd_s, rel=1e-4)
    assert gpar[1] == pytest.approx(fd_t, rel=1e-4)


def test_colour_gradients_match_central_differences(oracle):
    buf, target, t_now = _small_workload(oracle)
    p = oracle.Params(t_now=t_now)
    rgb, _, st = oracle.forward(buf, p)
    gslot, _ = oracle.backward(buf, st, p, oracle.rms_grad(rgb, target))
    rng = np.random.default_rng(61)
    filled = np.argwhere(np.arange(buf.k)[None, None, :] < buf.count[:, :, None])
    h = 1e-3
    for (j, i, s) in filled[rng.choice(len(filled), 12, replace=False)]:
        ch = int(rng.integers(0, 3))
        vals = []
        for sgn in (1, -1):
            cols = buf.colours().copy()
            cols[ch, j, i, s] += sgn * h
            r2, _ = oracle.reconstruct(buf.with_colours(cols), st, p)  # statistics held fixed
            vals.append(oracle.rms(r2, target))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert gslot[ch, j, i, s] == pytest.approx(fd, rel=1e-4, abs=1e-4 * np.abs(gslot).max() * 1e-3)


def test_adjoint_identity_and_partition_of_unity(oracle):
    w, h, k = 12, 10, 3
    buf = _random_buffer(oracle, w, h, k, 71, fill=0.5, empty_frac=0.1)
    st = _random_stats(oracle, w, h, 4, 72)
    p = oracle.Params(t_now=100.0, tile=4, tau=0.7)
    rng = np.random.default_rng(73)
    v = rng.standard_normal((3, h, w, k))
    u = rng.standard_normal((3, h, w))
    jv, aux = oracle.reconstruct(buf.with_colours(v), st, p)
    jtu, _ = oracle.backward(buf, st, p, u)
    filled = np.arange(k)[None, None, :] < buf.count[:, :, None]
    lhs = float((jv * u).sum())
    rhs = float((v * jtu * filled[None]).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)
    assert np.all(jtu[:, ~filled] == 0)
    covered = aux[1] > 0
    np.testing.assert_allclose(jtu.sum(axis=(1, 2, 3)), (u * covered).sum(axis=(1, 2)), rtol=1e-12)
