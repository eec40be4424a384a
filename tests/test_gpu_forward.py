"""GPU estimate and gather against the FP64 reference.

Tolerances:
  * gather, float32 arithmetic, same stored buffer and statistics: max |C - C_ref| <= 1e-5 on [0,1]
    colours (the target for plain FP32 output); the same bound holds end to end, statistics
    included, and for the FP16-storage buffer against the reference on the same FP16 buffer;
  * FP16 storage against the reference on the FP32 buffer: <= 2e-3 (storage quantisation);
  * tile statistics: the estimator accumulates in FP64; an age weight is 2^-n (exact) times a
    float32 power of two of the fractional part (<= 2 ulp, 2.4e-7 relative), and the statistics
    are stored as float32, so gradients and means get rtol 2e-6 with an absolute floor of
    1e-7 / px (luminance in [0, 1]).
"""
import numpy as np
import pytest

import afr_scenes as S
import oracle as O
from helpers import (DEV, afr_mod, gpu_build, log_weight_sum, oracle_build_cached, params,
                     reconstruct, stats_f32_as_f64, stats_to_gpu, torch_mod, workload)

pytestmark = pytest.mark.gpu

FORMS = ["plain", "tiled"]
CASES = [("c1", "fp32"), ("c2", "fp32"), ("c0", "fp32"), ("c3", "fp16")]


def _stat_tol(name):
    return {"vol": (2e-6, 0.0), "var": (2e-6, 1e-9), "lmean": (2e-6, 1e-7)}.get(name, (2e-6, 1e-7))


@pytest.mark.parametrize("name,precision", CASES + [("c3", "fp32")])
def test_estimate_matches_reference(name, precision):
    afr = afr_mod()
    wl = workload(name)
    print(f"estimate parity {name} {precision}", flush=True)
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref)
    obuf, _ = oracle_build_cached(name, precision, wl.k)
    gp, op = params(wl.t_now)
    gst = afr.estimate_gradients(gbuf, gp).cpu().numpy().astype(np.float64)
    ost = O.estimate(obuf, op)
    for i, n in enumerate(O.STAT_NAMES):
        rtol, atol = _stat_tol(n)
        np.testing.assert_allclose(gst[i], ost[i], rtol=rtol, atol=atol, err_msg=f"stat {n}")


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name,precision", CASES)
def test_gather_matches_reference_on_reference_statistics(form, name, precision):
    wl = workload(name)
    print(f"gather parity {form} {name} {precision}", flush=True)
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref)
    obuf, _ = oracle_build_cached(name, precision, wl.k)
    gp, op = params(wl.t_now)
    ost = O.estimate(obuf, op)
    rgb, aux = reconstruct(form, gbuf, stats_to_gpu(ost), gp)
    orgb, oaux = O.reconstruct(obuf, stats_f32_as_f64(ost), op)
    err = np.abs(rgb.cpu().numpy() - orgb).max()
    print(f"  max |C - C_ref| = {err:.3g}", flush=True)
    assert err <= 1e-5
    ga = aux.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(log_weight_sum(ga), log_weight_sum(oaux), rtol=0, atol=2e-5)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name,precision", CASES)
def test_end_to_end_matches_reference(form, name, precision):
    afr = afr_mod()
    wl = workload(name)
    print(f"end-to-end parity {form} {name} {precision}", flush=True)
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref)
    obuf, _ = oracle_build_cached(name, precision, wl.k)
    gp, op = params(wl.t_now)
    rgb, _ = reconstruct(form, gbuf, afr.estimate_gradients(gbuf, gp), gp)
    orgb, _, _ = O.forward(obuf, op)
    err = np.abs(rgb.cpu().numpy() - orgb).max()
    print(f"  max |C - C_ref| = {err:.3g}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("form", FORMS)
def test_fp16_storage_error_against_fp32_reference(form):
    """The FP16-storage path against the FP64 reference run on the FP32 buffer: the storage
    quantisation bound."""
    afr = afr_mod()
    wl = workload("c3")
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, "fp16", wl.t_ref)
    obuf, _ = oracle_build_cached("c3", "fp32", wl.k)
    gp, op = params(wl.t_now)
    rgb, _ = reconstruct(form, gbuf, afr.estimate_gradients(gbuf, gp), gp)
    orgb, _, _ = O.forward(obuf, op)
    d = np.abs(rgb.cpu().numpy() - orgb)
    print(f"fp16 storage {form}: max {d.max():.3g} p99 {np.quantile(d, 0.99):.3g} mean {d.mean():.3g}",
          flush=True)
    assert d.max() <= 2e-3


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("w,h,k,radius,tile", [(37, 23, 3, 2, 8), (1, 1, 2, 2, 8), (13, 5, 1, 0, 8),
                                               (29, 31, 4, 4, 5), (40, 17, 5, 1, 16),
                                               (19, 11, 2, 3, 1), (64, 8, 6, 2, 8)])
def test_edge_geometries(form, w, h, k, radius, tile):
    """Ragged image edges, a 1x1 image, R from 0 to 4, tiles from 1 to 16, holes (empty pixels)."""
    afr = afr_mod()
    rng = np.random.default_rng(w * 1000 + h * 10 + k)
    n = max(1, int(w * h * k * 0.8))
    scene = S.DiscScene(w, h, rng, 6, 50.0, speed=0.3, radius=(2.0, 6.0))
    s = S.uniform_stream(scene, w, h, n, 50.0, 50.0, rng)
    print(f"edge geometry {form} {w}x{h} K={k} R={radius} B={tile}", flush=True)
    for precision in ("fp32", "fp16"):
        gbuf, _ = gpu_build(s, w, h, k, precision, 50.0)
        obuf, _ = O.build_buffer(s, w, h, k, precision, 50.0)
        gp, op = params(53.0, radius=radius, tile=tile)
        rgb, aux = reconstruct(form, gbuf, afr.estimate_gradients(gbuf, gp), gp)
        orgb, oaux, _ = O.forward(obuf, op)
        assert np.abs(rgb.cpu().numpy() - orgb).max() <= 1e-5
        ga = aux.cpu().numpy()
        assert np.array_equal(ga[1] > 0, oaux[1] > 0)  # coverage agrees exactly


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_old_samples(precision):
    """Samples up to 80 s old (stored ages up to 60 s, 20 s from the stream's reference time to the
    reconstruction time): e^{-alpha a} drops below the float32 range past about 30 s, so the age
    weights must be evaluated over the FP64 range for the statistics to match the reference."""
    afr = afr_mod()
    w, h, k = 40, 24, 6
    rng = np.random.default_rng(80)
    scene = S.DiscScene(w, h, rng, 6, 60000.0, speed=1e-4, radius=(3.0, 8.0))
    s = S.uniform_stream(scene, w, h, w * h * 5, 60000.0, 60000.0, rng)
    print(f"old samples {precision}", flush=True)
    gbuf, _ = gpu_build(s, w, h, k, precision, 60000.0)
    obuf, _ = O.build_buffer(s, w, h, k, precision, 60000.0)
    gp, op = params(80000.0)
    gst = afr.estimate_gradients(gbuf, gp)
    ost = O.estimate(obuf, op)
    g64 = gst.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(g64))
    for i, n in enumerate(O.STAT_NAMES):
        rtol, atol = _stat_tol(n)
        np.testing.assert_allclose(g64[i], ost[i], rtol=rtol, atol=atol, err_msg=f"stat {n}")
    for form in FORMS:
        rgb, _ = reconstruct(form, gbuf, gst, gp)
        orgb, _, _ = O.forward(obuf, op)
        assert np.abs(rgb.cpu().numpy() - orgb).max() <= 1e-5


@pytest.mark.parametrize("w,h,radius", [(37, 23, 2), (72, 40, 2), (45, 17, 1), (24, 9, 0), (33, 30, 3)])
def test_launch_shapes_give_identical_output(w, h, radius):
    """One, two or four tiles per wave sum the same terms in the same order: colours and aux agree
    bit for bit, including tile columns that do not fill a group."""
    torch = torch_mod()
    afr = afr_mod()
    rng = np.random.default_rng(w * 7 + h)
    scene = S.DiscScene(w, h, rng, 5, 40.0, speed=0.2, radius=(2.0, 7.0))
    s = S.uniform_stream(scene, w, h, w * h * 6, 40.0, 40.0, rng)
    print(f"launch shapes {w}x{h} R={radius}", flush=True)
    for precision in ("fp32", "fp16"):
        gbuf, _ = gpu_build(s, w, h, 8, precision, 40.0)
        gp, op = params(41.0, radius=radius)
        st = afr.estimate_gradients(gbuf, gp)
        outs = [afr.reconstruct_launch(gbuf, st, gp, tpw) for tpw in (1, 2, 4)]
        for rgb, aux in outs[1:]:
            assert torch.equal(rgb, outs[0][0]) and torch.equal(aux, outs[0][1])
        fst, frgb, faux = afr.forward(gbuf, gp)  # the fused launch, the library's shape
        assert torch.equal(fst, st) and torch.equal(frgb, outs[0][0]) and torch.equal(faux, outs[0][1])
        obuf, _ = O.build_buffer(s, w, h, 8, precision, 40.0)
        orgb, _, _ = O.forward(obuf, op)
        assert np.abs(outs[0][0].cpu().numpy() - orgb).max() <= 1e-5


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_launch_shapes_identical_with_mixed_widths(precision):
    """Tiles side by side on both sides of the width bound below which the separable factors are
    evaluated one exponential each (every other tile column 0.1 px wide in x, every fourth tile
    column narrow in y): a wave that holds tiles of both kinds evaluates each tile as a wave of its
    own would, so one, two and four tiles per wave give the same bits, and the output matches the
    reference on the same statistics."""
    torch = torch_mod()
    afr = afr_mod()
    w, h, k = 72, 40, 6
    rng = np.random.default_rng(5150)
    scene = S.DiscScene(w, h, rng, 6, 40.0, speed=0.2, radius=(2.0, 7.0))
    s = S.uniform_stream(scene, w, h, w * h * 5, 40.0, 40.0, rng)
    print(f"launch shapes, mixed widths {precision}", flush=True)
    gbuf, _ = gpu_build(s, w, h, k, precision, 40.0)
    obuf, _ = O.build_buffer(s, w, h, k, precision, 40.0)
    gp, op = params(41.0)
    ost = O.estimate(obuf, op)
    ost[O.STAT["sx2"]][:, 0::2] = 0.01
    ost[O.STAT["sy2"]][:, 1::4] = 0.015
    st = stats_to_gpu(ost)
    outs = [afr.reconstruct_launch(gbuf, st, gp, tpw) for tpw in (1, 2, 4)]
    for rgb, aux in outs[1:]:
        assert torch.equal(rgb, outs[0][0]) and torch.equal(aux, outs[0][1])
    orgb, _ = O.reconstruct(obuf, stats_f32_as_f64(ost), op)
    err = np.abs(outs[0][0].cpu().numpy() - orgb).max()
    print(f"  max |C - C_ref| = {err:.3g}", flush=True)
    assert err <= 1e-5


def test_reference_statistics_round_trip_and_constants():
    """A constant-colour buffer reproduces the constant through the GPU gather (a normalised
    average of equal colours is that colour), and the tiled and plain forms agree to float32
    rounding.

    Bound: the tiled form sums each slot plane's <= (2R+1)^2 terms in float32 and adds the plane
    partials with compensation, so numerator and denominator each carry <= ((2R+1)^2 + 4) u relative
    error (u = 2^-24), plus the division and the colour product: ((2R+1)^2 + 8) u |c|. The direct
    form sums all <= K (2R+1)^2 terms in one float32 running sum; its bound is K (2R+1)^2 u |c|,
    and 1e-5 (the output tolerance) applies."""
    torch = torch_mod()
    afr = afr_mod()
    wl = workload("c2")
    gbuf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    gp, _ = params(wl.t_now)
    filled = (torch.arange(wl.k, device=DEV)[:, None, None] < gbuf.count[None, :, :].long())
    const = torch.tensor([0.25, 0.5, 0.75], device=DEV)[:, None, None, None] * filled
    stats = afr.estimate_gradients(gbuf, gp)
    u = 2.0 ** -24
    for fn, tol in ((afr.reconstruct, lambda v: (25 + 8) * u * v),
                    (afr.reconstruct_plain, lambda v: 1e-5)):
        rgb, _ = fn(gbuf, stats, gp, colours=const.float().contiguous())
        for c, v in enumerate((0.25, 0.5, 0.75)):
            err = float((rgb[c] - v).abs().max())
            print(f"  constant {v}: max error {err:.3g} (bound {tol(v):.3g})", flush=True)
            assert err <= tol(v)
    a, _ = afr.reconstruct(gbuf, stats, gp)
    b, _ = afr.reconstruct_plain(gbuf, stats, gp)
    assert float((a - b).abs().max()) <= 2e-6


@pytest.mark.parametrize("w,h,radius,precision", [(37, 23, 2, "fp16"), (72, 40, 1, "fp32"),
                                                  (24, 9, 0, "fp16"), (33, 30, 3, "fp32"),
                                                  (41, 19, 4, "fp16"), (640, 480, 2, "fp16")])
def test_fused_forward_equals_estimate_then_gather(w, h, radius, precision):
    """afr_forward (statistics and gather of each tile group in one launch) gives the statistics of
    afr_estimate_gradients and the image and aux of afr_reconstruct bit for bit, for every launch
    shape, including groups past the last tile column."""
    torch = torch_mod()
    afr = afr_mod()
    if (w, h) == (640, 480):
        wl = workload("c3")
        s, k, t_ref, t_now = wl.stream, wl.k, wl.t_ref, wl.t_now
    else:
        rng = np.random.default_rng(w * 31 + h)
        scene = S.DiscScene(w, h, rng, 5, 40.0, speed=0.2, radius=(2.0, 7.0))
        s, k, t_ref, t_now = S.uniform_stream(scene, w, h, w * h * 6, 40.0, 40.0, rng), 8, 40.0, 41.0
    print(f"fused forward {w}x{h} R={radius} {precision}", flush=True)
    gbuf, _ = gpu_build(s, w, h, k, precision, t_ref)
    gp, _ = params(t_now, radius=radius)
    st = afr.estimate_gradients(gbuf, gp)
    rgb, aux = afr.reconstruct(gbuf, st, gp)
    fst, frgb, faux = afr.forward(gbuf, gp)
    assert torch.equal(fst, st) and torch.equal(frgb, rgb) and torch.equal(faux, aux)
