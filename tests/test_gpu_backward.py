"""GPU adjoint against the FP64 reference adjoint and FP64 central finite differences (h = 1e-3).

Slot-colour gradients are sums over up to (2R+1)^2 pixels of g(p) pi_s(p) with mixed signs, so the
float32 result carries an absolute error proportional to the sum of the absolute terms,
A_s = sum_p |g(p)| pi_s(p) (computed by the reference adjoint on |g|), not to |g_ref|. The tiled
adjoint evaluates weights relative to the tile's age reference (the forward's shift); a pixel the
forward keeps on that path has a weight sum of at least 1e-30 of the reference, and its terms below
float32's normal range (2^-126 of the reference) are zero, so slots whose gradient is more than ~1e-8
below the largest can lose those contributions. Tolerance per component:
|g - g_ref| <= 1e-4 |g_ref| + 1e-5 A_s + 1e-7 max|g_ref| + FLT_MIN.
d(sigma) and d(tau): 1e-4 relative.
"""
import numpy as np
import pytest

import afr_scenes as S
import oracle as O
from helpers import (DEV, afr_mod, gpu_build, params, slots_to_reference_layout, stats_f32_as_f64,
                     stats_to_gpu, torch_mod)

pytestmark = pytest.mark.gpu


def _frame(seq, f, k):
    wl = seq.frame_workload(f)
    return wl


def _loss_grad_gpu(rgb, gt):
    torch = torch_mod()
    d = rgb.double() - gt
    e = torch.sqrt((d * d).mean())
    return (d / (d.numel() * e)).float()


def _check_slots(g, g_ref, a_ref):
    # below FLT_MIN both sides are float32 subnormal noise
    tol = (1e-4 * np.abs(g_ref) + 1e-5 * a_ref + 1e-7 * np.abs(g_ref).max()
           + np.finfo(np.float32).tiny)
    bad = np.abs(g - g_ref) > tol
    rel = np.abs(g - g_ref).max() / max(np.abs(g_ref).max(), 1e-300)
    print(f"  slot grads: max |diff| / max |g_ref| = {rel:.3g}", flush=True)
    assert not bad.any(), f"{bad.sum()} slot gradients off; worst {np.abs(g - g_ref)[bad].max():.3g}"


@pytest.mark.parametrize("form", ["plain", "tiled"])
@pytest.mark.parametrize("size,k,precision", [(96, 4, "fp32"), (128, 8, "fp16"), (512, 8, "fp32")])
def test_backward_matches_reference_adjoint(form, size, k, precision):
    torch = torch_mod()
    afr = afr_mod()
    seq = S.make_c4_sequence(n_frames=2, width=size, height=size, k=k)
    wl = seq.frame_workload(1)
    print(f"backward parity {form} {size}x{size} K={k} {precision}", flush=True)
    gt = S.ground_truth(seq.scene, size, size, wl.t_now, 4)
    gbuf, _ = gpu_build(wl.stream, size, size, k, precision, wl.t_ref)
    obuf, _ = O.build_buffer(wl.stream, size, size, k, precision, wl.t_ref)
    gp, op = params(wl.t_now, sigma=1.0, tau=0.5)
    stats = afr.estimate_gradients(gbuf, gp)
    fn = afr.reconstruct if form == "tiled" else afr.reconstruct_plain
    rgb, aux = fn(gbuf, stats, gp)
    ost = O.estimate(obuf, op)
    orgb, _ = O.reconstruct(obuf, ost, op)
    # one upstream gradient, computed by the reference, drives both adjoints
    og = O.rms_grad(orgb, gt)
    g = torch.from_numpy(og).float().to(DEV)
    gslot, gpar = afr.reconstruct_backward(gbuf, stats, gp, rgb, aux, g)
    oslot, opar = O.backward(obuf, ost, op, og)
    aslot, _ = O.backward(obuf, ost, op, np.abs(og))
    print(f"  d(sigma, tau) gpu {gpar.cpu().numpy()} ref {opar}", flush=True)
    np.testing.assert_allclose(gpar.cpu().numpy(), opar, rtol=1e-4)
    _check_slots(slots_to_reference_layout(gslot.cpu().numpy()).astype(np.float64), oslot, aslot)


@pytest.mark.timeout(600)
def test_c4_gradients_match_finite_differences():
    """The 32-frame 512x512 K=8 FP32 sequence (60 Hz frames) as configured; loss = mean over frames
    of the RMS error against the analytic ground truth (Sec. 7). Gradients through the autograd
    Function (tile statistics estimated from the buffer's stored samples, held constant) against
    FP64 central differences (h = 1e-3) of the reference forward: sigma and tau over all frames, and
    four seeded slot colours in each of the first and last frames.

    sigma and tau at 1e-4 relative. A colour entry's gradient sums the upstream RMS gradient over the
    pixels the slot reaches; the GPU's upstream gradient comes from its own image, which differs from
    the reference's by dC <= 1e-5, i.e. by up to dC / (N RMS) per pixel. So the colour bound is
    1e-4 |fd| + 2 (dC / (N RMS F)) sum_p pi_s(p), the last sum being the reference adjoint of a
    ones image. Entries are drawn (seeded) from the filled slots whose reference gradient is in the
    top tenth by magnitude, where that term is small against the gradient."""
    torch = torch_mod()
    afr = afr_mod()
    F, W, H, K = 32, 512, 512, 8
    seq = S.make_c4_sequence(n_frames=F, width=W, height=H, k=K)
    sig0, tau0, h = 1.0, 0.5, 1e-3
    pick = np.random.default_rng(404)
    g_gpu = np.zeros(2)
    fd = np.zeros(2)
    worst = 0.0
    for f in range(F):
        wl = seq.frame_workload(f)
        print(f"c4 frame {f}", flush=True)
        gt = S.ground_truth(seq.scene, W, H, wl.t_now, 4)
        gbuf, _ = gpu_build(wl.stream, W, H, K, "fp32", wl.t_ref)
        gp, op = params(wl.t_now, sigma=sig0, tau=tau0)
        sig = torch.tensor(sig0, device=DEV, requires_grad=True)
        tau = torch.tensor(tau0, device=DEV, requires_grad=True)
        col = gbuf.colours().clone().requires_grad_(True)
        rgb = afr.reconstruct_differentiable(gbuf, gp, sig, tau, colours=col)
        d = rgb.double() - torch.from_numpy(gt).to(DEV)
        (torch.sqrt((d * d).mean()) / F).backward()
        g_gpu += (sig.grad.item(), tau.grad.item())
        obuf, _ = O.build_buffer(wl.stream, W, H, K, "fp32", wl.t_ref)
        for i, name in enumerate(("sigma", "tau")):
            lp = O.rms(O.forward(obuf, op.with_(**{name: getattr(op, name) + h}))[0], gt)
            lm = O.rms(O.forward(obuf, op.with_(**{name: getattr(op, name) - h}))[0], gt)
            fd[i] += (lp - lm) / (2 * h) / F
        if f not in (0, F - 1):
            continue
        ost = O.estimate(obuf, op)
        orgb, _ = O.reconstruct(obuf, ost, op)
        oslot, _ = O.backward(obuf, ost, op, O.rms_grad(orgb, gt) / F)
        pi_sum, _ = O.backward(obuf, ost, op, np.ones_like(orgb))
        dC = float(np.abs(rgb.detach().cpu().numpy() - orgb).max())
        assert dC <= 1e-5
        dg = dC / (orgb.size * O.rms(orgb, gt) * F)
        filled = np.arange(K)[None, None, :] < obuf.count[:, :, None]   # [H, W, K]
        mag = np.abs(oslot) * filled[None]
        top = np.argwhere(mag >= np.quantile(mag[:, filled], 0.9))
        gcol = col.grad.cpu().numpy()
        for c, j, i, k in top[pick.choice(len(top), 4, replace=False)]:
            plane = (obuf.r, obuf.g, obuf.b)[c]
            v0 = plane[j, i, k]
            vals = []
            for v in (v0 + h, v0 - h):
                plane[j, i, k] = v
                vals.append(O.rms(O.reconstruct(obuf, ost, op)[0], gt))
            plane[j, i, k] = v0
            ref = (vals[0] - vals[1]) / (2 * h) / F
            got = float(gcol[c, k, j, i])
            tol = 1e-4 * abs(ref) + 2 * dg * pi_sum[c, j, i, k]
            print(f"  colour ({c},{k},{j},{i}): gpu {got:.6e} fd {ref:.6e}", flush=True)
            assert abs(got - ref) <= tol
            worst = max(worst, abs(got - ref) / abs(ref))
    print(f"gpu {g_gpu} fd {fd}; worst colour rel {worst:.3g}", flush=True)
    np.testing.assert_allclose(g_gpu, fd, rtol=1e-4)


def test_autograd_function_matches_backward_and_reaches_stream_colours():
    torch = torch_mod()
    afr = afr_mod()
    wl = S.make_workload("c1")
    xs = [torch.from_numpy(a).to(DEV) for a in wl.stream.arrays()]
    buf, _ = afr.build_deep_buffer(*xs, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    p = afr.Params(t_now=wl.t_now)
    gt = torch.from_numpy(S.ground_truth(wl.scene, wl.width, wl.height, wl.t_now, 4)).float().to(DEV)
    sig = torch.tensor(1.2, device=DEV, requires_grad=True)
    tau = torch.tensor(0.4, device=DEV, requires_grad=True)
    # stream colours -> slot colours by the build's src map; autograd scatters back by index
    col = torch.stack(xs[3:6]).requires_grad_(True)
    src = buf.src.long()
    slot = torch.where(src[None] >= 0, col[:, src.clamp(min=0)], torch.zeros((), device=DEV))
    rgb = afr.reconstruct_differentiable(buf, p, sig, tau, colours=slot.contiguous())
    loss = torch.sqrt(((rgb - gt) ** 2).mean())
    loss.backward()
    ob, _ = O.build_buffer(wl.stream, wl.width, wl.height, wl.k, "fp32", wl.t_ref)
    op = O.Params(t_now=wl.t_now, sigma=1.2, tau=0.4)
    orgb, _, ost = O.forward(ob, op)
    og = O.rms_grad(orgb, gt.cpu().numpy().astype(np.float64))
    oslot, opar = O.backward(ob, ost, op, og)
    # End to end, the upstream gradient comes from the GPU's own forward output, which differs from
    # the reference's by dC; |d(dl/dC)| <= max|dC| / (N RMS) per pixel, and it reaches a slot
    # through sum_p pi_s(p) (the reference adjoint of a ones image).
    dC = float(np.abs(rgb.detach().cpu().numpy() - orgb).max())
    dg = dC / (orgb.size * O.rms(orgb, gt.cpu().numpy()))
    aslot, _ = O.backward(ob, ost, op, np.abs(og) + 2 * dg / 1e-5)
    np.testing.assert_allclose([sig.grad.item(), tau.grad.item()], opar, rtol=1e-4)
    # stream-colour gradient = slot gradient scattered by src (each sample sits in at most one slot)
    ref = np.zeros((3, len(wl.stream)))
    aref = np.zeros((3, len(wl.stream)))
    s = ob.src.reshape(-1)  # reference layout [H, W, K]
    for c in range(3):
        ref[c, s[s >= 0]] = oslot[c].reshape(-1)[s >= 0]
        aref[c, s[s >= 0]] = aslot[c].reshape(-1)[s >= 0]
    _check_slots(col.grad.cpu().numpy().astype(np.float64), ref, aref)


def _adjoint_case(stream, w, h, k, precision, t_now, radius, edit_stats=None, seed=0):
    """GPU forward (tiled) + adjoint against the FP64 reference adjoint on the same statistics."""
    torch = torch_mod()
    afr = afr_mod()
    gbuf, _ = gpu_build(stream, w, h, k, precision, t_now)
    obuf, _ = O.build_buffer(stream, w, h, k, precision, t_now)
    gp, op = params(t_now, radius=radius)
    ost = O.estimate(obuf, op)
    if edit_stats is not None:
        edit_stats(ost)
    ost32 = stats_f32_as_f64(ost)
    gst = stats_to_gpu(ost)
    rgb, aux = afr.reconstruct(gbuf, gst, gp)
    orgb, _ = O.reconstruct(obuf, ost32, op)
    assert np.abs(rgb.cpu().numpy() - orgb).max() <= 1e-5
    og = np.random.default_rng(seed).standard_normal(orgb.shape) * 1e-3
    g = torch.from_numpy(og).float().to(DEV)
    gslot, gpar = afr.reconstruct_backward(gbuf, gst, gp, rgb, aux, g)
    oslot, opar = O.backward(obuf, ost32, op, og)
    aslot, _ = O.backward(obuf, ost32, op, np.abs(og))
    print(f"  d(sigma, tau) gpu {gpar.cpu().numpy()} ref {opar}", flush=True)
    np.testing.assert_allclose(gpar.cpu().numpy(), opar, rtol=1e-4)
    _check_slots(slots_to_reference_layout(gslot.cpu().numpy()).astype(np.float64), oslot, aslot)
    return aux.cpu().numpy()


@pytest.mark.parametrize("radius,precision", [(0, "fp32"), (1, "fp16"), (3, "fp32"), (4, "fp16")])
def test_backward_every_radius(radius, precision):
    """The tiled adjoint (one template per radius) against the reference on a ragged 44x27 image."""
    w, h, k = 44, 27, 3
    rng = np.random.default_rng(40 + radius)
    scene = S.DiscScene(w, h, rng, 8, 50.0, speed=0.3, radius=(2.0, 7.0))
    s = S.stratified_stream(scene, w, h, k, 50.0, 50.0, rng)
    print(f"backward radius {radius} {precision} {w}x{h} K={k}", flush=True)
    _adjoint_case(s, w, h, k, precision, 50.0, radius, seed=radius)


def test_backward_pixels_evaluated_directly():
    """One brand-new sample in the corner and a large temporal sensitivity (kt2 = 2 per ms^2 in every
    tile): the corner tile's age reference is ~0, so its pixels whose blocks hold only older samples
    (ages 15..40 ms) have shifted weights far below float32 range. The forward evaluates those pixels
    directly (their aux shift is their own maximum exponent), and the adjoint must use the exact
    path for them; both are checked against the reference."""
    w, h, k = 24, 16, 2
    rng = np.random.default_rng(77)
    t_now = 100.0
    ys, xs = np.mgrid[0:h, 0:w]
    px = np.repeat(xs.ravel(), 2).astype(np.float64)
    py = np.repeat(ys.ravel(), 2).astype(np.float64)
    n = px.size
    x = (px + rng.random(n)).astype(np.float32)
    y = (py + rng.random(n)).astype(np.float32)
    t = (t_now - 15.0 - 25.0 * rng.random(n)).astype(np.float32)
    x = np.append(x, np.float32(0.3))
    y = np.append(y, np.float32(0.6))
    t = np.append(t, np.float32(t_now))
    c = rng.random((3, n + 1)).astype(np.float32)
    s = S.Stream(x, y, t, c[0], c[1], c[2])

    def big_kt2(ost):
        ost[O.STAT["kt2"]] = 2.0

    aux = _adjoint_case(s, w, h, k, "fp32", t_now, 2, edit_stats=big_kt2, seed=9)
    # pixels of the corner tile evaluated directly carry their own (very negative) maximum exponent
    assert (aux[0][:8, :8] < -80.0).sum() > 10


@pytest.mark.parametrize("sx2,sy2,kt2,precision", [(0.01, 0.02, None, "fp32"), (0.015, 0.01, None, "fp16"),
                                                   (0.0625, 0.0625, 0.05, "fp32"),
                                                   (0.0625, 0.09, 0.05, "fp16")])
def test_narrow_widths(sx2, sy2, kt2, precision):
    """Spatial standard deviations of 0.1 to 0.3 px (statistics supplied by the caller, below the
    default width floor): the weights of the far offsets fall far below float32's range while the
    near ones stay large, so the separable factors cannot be carried upward from the smallest one.
    With a temporal sensitivity on top, old samples get small but non-negligible weights. The tiled
    forward and adjoint must still match the reference."""
    w, h, k = 40, 24, 4
    rng = np.random.default_rng(91)
    scene = S.DiscScene(w, h, rng, 8, 40.0, speed=0.3, radius=(2.0, 7.0))
    s = S.stratified_stream(scene, w, h, k, 40.0, 40.0, rng)
    print(f"narrow widths sx2={sx2} sy2={sy2} kt2={kt2} {precision}", flush=True)

    def narrow(ost):
        ost[O.STAT["sx2"]] = sx2
        ost[O.STAT["sy2"]] = sy2
        if kt2 is not None:
            ost[O.STAT["kt2"]] = kt2

    _adjoint_case(s, w, h, k, precision, 40.0, 2, edit_stats=narrow, seed=5)
