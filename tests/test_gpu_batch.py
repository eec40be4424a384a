"""Batched persistent launch (many uneven reconstructions in one launch, capturable in a graph).

Checks: every item equals afr_estimate_gradients + afr_reconstruct on that item bit for bit (the
batch runs the same per-tile code), every item matches the FP64 reference to 1e-5 on its FP16
buffer, the launch shape chosen by the tuner changes no output bit, and a captured graph replays to
the eager result every time, with eager work and synchronisation between replays.
"""
import numpy as np
import pytest

import afr_scenes as S
import oracle as O
from helpers import afr_mod, gpu_build, torch_mod

pytestmark = pytest.mark.gpu

SIZES = ((64, 64), (96, 80), (128, 128), (200, 120), (37, 53))
KS = (4, 8, 16)


def _items(n=10, seed=7, precision="fp16"):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        w, h = SIZES[int(rng.integers(len(SIZES)))]
        k = KS[int(rng.integers(len(KS)))]
        srng = np.random.default_rng(100 + i)
        scene = S.DiscScene(w, h, srng, 12, 64.0, highlights=bool(i % 2))
        stream = S.stratified_stream(scene, w, h, k, 64.0, 64.0, srng)
        out.append((stream, w, h, k))
    return out


def _build_all(items, precision="fp16"):
    afr = afr_mod()
    bufs = []
    for stream, w, h, k in items:
        buf, _ = gpu_build(stream, w, h, k, precision, 64.0)
        bufs.append((buf, afr.Params(t_now=64.0 + 0.25 * (k % 3))))
    return bufs


def test_batch_equals_separate_calls_and_reference():
    torch = torch_mod()
    afr = afr_mod()
    items = _items()
    bufs = _build_all(items)
    batch = afr.Batch(bufs)
    batch.run()
    torch.cuda.synchronize()
    for i, ((buf, p), (stream, w, h, k)) in enumerate(zip(bufs, items)):
        print(f"batch item {i}: {w}x{h} K={k}", flush=True)
        st = afr.estimate_gradients(buf, p)
        rgb, aux = afr.reconstruct(buf, st, p)
        assert torch.equal(batch.stats[i], st)
        assert torch.equal(batch.rgb[i], rgb)
        assert torch.equal(batch.aux[i], aux)
        ob, _ = O.build_buffer(stream, w, h, k, "fp16", 64.0)
        orgb, _, _ = O.forward(ob, O.Params(t_now=p.t_now))
        assert np.abs(batch.rgb[i].cpu().numpy() - orgb).max() <= 1e-5
    batch.close()


@pytest.mark.parametrize("radius,precision", [(0, "fp16"), (1, "fp16"), (3, "fp16"), (4, "fp16"),
                                              (2, "fp32"), (1, "fp32")])
def test_batch_every_radius_and_precision(radius, precision):
    """The batch kernel's instantiations for other radii and binary32 storage (other register
    budgets and group sizes) give each item's separate statistics and gather bit for bit, for every
    launch shape the radius allows."""
    torch = torch_mod()
    afr = afr_mod()
    items = _items(n=5, seed=31 + radius, precision=precision)
    bufs = [(buf, p.with_(radius=radius)) for buf, p in _build_all(items, precision=precision)]
    refs = []
    for buf, p in bufs:
        st = afr.estimate_gradients(buf, p)
        rgb, aux = afr.reconstruct(buf, st, p)
        refs.append((st, rgb, aux))
    for tpw in ((1, 2, 4) if radius <= 2 else (1, 2)):
        print(f"batch R={radius} {precision} tiles per wave {tpw}", flush=True)
        batch = afr.Batch(bufs, tiles_per_wave=tpw)
        batch.run()
        torch.cuda.synchronize()
        for i, (st, rgb, aux) in enumerate(refs):
            assert torch.equal(batch.stats[i], st), (tpw, i)
            assert torch.equal(batch.rgb[i], rgb), (tpw, i)
            assert torch.equal(batch.aux[i], aux), (tpw, i)
        batch.close()


def test_launch_shapes_and_tuner_change_no_bit():
    torch = torch_mod()
    afr = afr_mod()
    bufs = _build_all(_items(n=6, seed=11))
    ref = None
    for tpw in (1, 2, 4):
        batch = afr.Batch(bufs, tiles_per_wave=tpw)
        batch.run()
        torch.cuda.synchronize()
        outs = [r.clone() for r in batch.rgb]
        if ref is None:
            ref = outs
        else:
            assert all(torch.equal(a, b) for a, b in zip(ref, outs)), f"tiles_per_wave={tpw}"
        batch.close()
    batch = afr.Batch(bufs)
    best, ms = batch.tune()
    assert best in (1, 2, 4) and ms > 0 and batch.tiles_per_wave == best
    batch.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ref, batch.rgb))
    # single-frame tuner: recorded shape, same output
    buf, p = bufs[0]
    st = afr.estimate_gradients(buf, p)
    a, _ = afr.reconstruct(buf, st, p)
    tpw, _ = afr.reconstruct_tune(buf, st, p)
    b, _ = afr.reconstruct(buf, st, p)
    assert tpw in (1, 2, 4) and torch.equal(a, b)
    batch.close()


def test_graph_capture_replays_match_eager():
    torch = torch_mod()
    afr = afr_mod()
    bufs = _build_all(_items(n=8, seed=23))
    batch = afr.Batch(bufs)
    batch.run()
    torch.cuda.synchronize()
    eager = [r.clone() for r in batch.rgb]
    eager_stats = [s.clone() for s in batch.stats]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm the capture stream
        batch.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run()
    for rep in range(4):
        for r in batch.rgb:  # eager work between replays
            r.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(eager, batch.rgb)):
            assert torch.equal(a, b), f"replay {rep} item {i}"
        for a, b in zip(eager_stats, batch.stats):
            assert torch.equal(a, b)
    batch.close()


def test_plan_free_call_equals_plan_and_replays():
    """afr_batch_reconstruct (no plan: the item table written by the call's own kernels) gives the
    plan's outputs bit for bit for every launch shape, on a side stream too, and replays of a graph
    that captured it (with eager work between them) give them again."""
    torch = torch_mod()
    afr = afr_mod()
    bufs = _build_all(_items(n=7, seed=29))
    batch = afr.Batch(bufs)
    batch.run()
    torch.cuda.synchronize()
    eager = [r.clone() for r in batch.rgb] + [s.clone() for s in batch.stats]
    eager += [a.clone() for a in batch.aux]
    outs = lambda: list(batch.rgb) + list(batch.stats) + list(batch.aux)
    for tpw in (0, 1, 2, 4):
        print(f"plan-free batch, tiles per wave {tpw}", flush=True)
        for o in outs():
            o.fill_(float("nan"))
        batch.reconstruct(tiles_per_wave=tpw)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(eager, outs())), tpw
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.reconstruct(tiles_per_wave=2, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(eager, outs()))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.reconstruct(tiles_per_wave=4)
    for rep in range(3):
        for o in outs():
            o.fill_(float("nan"))
        batch.run()  # eager work between replays, which also rewrites the outputs
        for o in outs():
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(eager, outs())), rep
    batch.close()


@pytest.mark.timeout(900)
def test_c5_recipe_equals_separate_calls_and_reference():
    """The C5 batch as configured: 64 items drawn from {128x128, 320x240, 640x480, 1024x768} x
    K {4, 8, 16}, FP16 storage, R = 2. Every item of the batched launch (default shape, then the
    tuned one) equals its separate estimate + gather calls bit for bit, and the largest items (both
    1024x768 K=16 drawn first) match the FP64 reference on the same buffers to 1e-5."""
    torch = torch_mod()
    afr = afr_mod()
    recipe = S.c5_recipe()
    largest = [i for i, r in enumerate(recipe) if r == (1024, 768, 16)][:2]
    items, kept = [], {}
    for i in range(len(recipe)):
        wl = S.make_c5_batch(instances=[i])[0]
        if i % 8 == 0:
            print(f"c5 item {i}: {wl.width}x{wl.height} K={wl.k}", flush=True)
        buf, _ = gpu_build(wl.stream, wl.width, wl.height, wl.k, "fp16", wl.t_ref)
        items.append((buf, afr.Params(t_now=wl.t_now)))
        if i in largest:
            kept[i] = wl
    batch = afr.Batch(items)
    for label in ("default", "tuned"):
        if label == "tuned":
            tpw, _ = batch.tune()
            print(f"tuned tiles_per_wave {tpw}", flush=True)
        batch.run()
        torch.cuda.synchronize()
        for i, (buf, p) in enumerate(items):
            st = afr.estimate_gradients(buf, p)
            rgb, aux = afr.reconstruct(buf, st, p)
            assert torch.equal(batch.stats[i], st), (label, i)
            assert torch.equal(batch.rgb[i], rgb), (label, i)
            assert torch.equal(batch.aux[i], aux), (label, i)
    for i in largest:
        wl = kept[i]
        print(f"c5 item {i} against the reference", flush=True)
        ob, _ = O.build_buffer(wl.stream, wl.width, wl.height, wl.k, "fp16", wl.t_ref)
        orgb, _, _ = O.forward(ob, O.Params(t_now=wl.t_now))
        err = float(np.abs(batch.rgb[i].cpu().numpy() - orgb).max())
        print(f"  max |C - C_ref| = {err:.3g}", flush=True)
        assert err <= 1e-5
    batch.close()
