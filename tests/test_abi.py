"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function that
include/afr.h declares, and validates arguments before launching anything."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def afr():
    import paper_2510_15876_amd as afr
    if not os.path.exists(afr.lib_path()):
        from paper_2510_15876_amd import _build
        _build.build()
    afr.library()
    return afr


def _declared():
    src = open(os.path.join(ROOT, "include", "afr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(afr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("afr_build_deep_buffer", "afr_estimate_gradients", "afr_reconstruct",
              "afr_reconstruct_backward"):
        assert n in names


def test_library_exports_every_declared_symbol(afr):
    lib = afr.library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_no_torch_types_in_the_header():
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "afr.h")).read(), flags=re.S)
    for bad in ("torch", "at::", "c10", "Tensor"):
        assert bad not in src


def test_status_strings_and_sizes(afr):
    lib = afr.library()
    assert lib.afr_status_string(0) == b"ok"
    assert lib.afr_status_string(4) == b"workspace too small"
    assert lib.afr_version().startswith(b"afr")
    a = lib.afr_build_workspace_bytes(1000, 64, 64, 4)
    b = lib.afr_build_workspace_bytes(2000, 64, 64, 4)
    assert b - a >= 1000 * 32 - 256 and a >= 1000 * 32  # one 32-byte record per sample
    assert lib.afr_build_workspace_bytes(-1, 64, 64, 4) == 0
    assert lib.afr_backward_workspace_bytes(512, 512, 8, 2) >= 3 * 512 * 512 * 4
    # tiled adjoint: per-pixel (g', k') and per-tile partials of every region slot and plane
    assert lib.afr_backward_workspace_bytes(512, 512, 8, 2) >= 4096 * 8 * 3 * 144 * 4
    assert lib.afr_backward_workspace_bytes(0, 5, 8, 2) == 0
    assert lib.afr_backward_workspace_bytes(5, 5, 0, 2) == 0
    assert lib.afr_backward_workspace_bytes(5, 5, 8, 5) == 0


def _fake_buffer(afr, w=16, h=8, k=4, prec=0, t_ref=10.0, null_plane=False):
    # host addresses only: every call below must fail validation before touching them. A binary16
    # buffer's field pointers address one 12-byte record (ox, oy, r, g, b, age): the struct's order
    # ox, oy, tage, r, g, b sits at byte offsets 0, 2, 10, 4, 6, 8.
    d = 0x1000
    f = (d, d + 2, d + 10, d + 4, d + 6, d + 8) if prec == 1 else (d,) * 6
    return afr._DeepBuffer(w, h, k, prec, t_ref, None if null_plane else f[0], *f[1:], d, None)


@pytest.mark.parametrize("mutate,expect", [
    (dict(), None),
    (dict(k=0), 2), (dict(k=256), 2), (dict(w=0), 2), (dict(prec=3), 2),
    (dict(null_plane=True), 1), (dict(w=1 << 16, h=1 << 12, k=16), 2),
    (dict(prec=1), None),
    # one slot plane must stay below 2^31 bytes: 2^29 float32 pixels are too many even at K = 1
    (dict(w=1 << 15, h=1 << 14, k=1), 2), (dict(w=1 << 15, h=(1 << 14) - 1, k=1), None),
    # binary16 records are 12 bytes: 2^31 / 12 pixels
    (dict(w=1 << 14, h=10923, k=1, prec=1), 2), (dict(w=1 << 14, h=10922, k=1, prec=1), None),
])
def test_buffer_validation(afr, mutate, expect):
    lib = afr.library()
    kw = dict(w=16, h=8, k=4, prec=0, t_ref=10.0)
    kw.update(mutate)
    b = _fake_buffer(afr, **kw)
    p = afr.Params(t_now=11.0)._c()
    # NULL stats pointer: a valid buffer gets as far as the statistics check (invalid = 1)
    st = lib.afr_estimate_gradients(ctypes.byref(b), ctypes.byref(p), None, None)
    assert st == (1 if expect is None else expect)


@pytest.mark.parametrize("field,value,expect", [
    ("t_now", 9.0, 2),          # t_now < t_ref
    ("radius", 5, 2), ("radius", -1, 2), ("tile", 0, 2), ("tile", 17, 2),
    ("e_min", 0.0, 2), ("e_max", 0.0, 2), ("sigma", -1.0, 2), ("tau", float("nan"), 2),
    ("dt_floor", 0.0, 2), ("age_floor", -1.0, 2), ("alpha", float("inf"), 2),
    ("g_floor", 0.0, 2), ("g_floor", -1e-3, 2),
])
def test_param_validation(afr, field, value, expect):
    lib = afr.library()
    b = _fake_buffer(afr)
    p = afr.Params(t_now=11.0).with_(**{field: value})._c()
    s = afr._TileStats(8, 2, 1, 0x1000)
    assert lib.afr_estimate_gradients(ctypes.byref(b), ctypes.byref(p), ctypes.byref(s), None) == expect


def test_stats_geometry_and_workspace_checks(afr):
    lib = afr.library()
    b = _fake_buffer(afr, w=17, h=9)
    p = afr.Params(t_now=11.0)._c()
    bad = afr._TileStats(8, 2, 2, 0x1000)   # needs 3 x 2 tiles
    assert lib.afr_reconstruct(ctypes.byref(b), ctypes.byref(bad), ctypes.byref(p), 0x2000, None, None) == 1
    wrong_tile = afr._TileStats(4, 5, 3, 0x1000)
    assert lib.afr_reconstruct(ctypes.byref(b), ctypes.byref(wrong_tile), ctypes.byref(p), 0x2000, None, None) == 1
    ok = afr._TileStats(8, 3, 2, 0x1000)
    assert lib.afr_reconstruct(ctypes.byref(b), ctypes.byref(ok), ctypes.byref(p), None, None, None) == 1
    # backward: tau must be positive, workspace must be large enough
    p0 = afr.Params(t_now=11.0, tau=0.0)._c()
    args = [0x2000] * 6
    assert lib.afr_reconstruct_backward(ctypes.byref(b), ctypes.byref(ok), ctypes.byref(p0), *args[:5], 0x3000, 1 << 30, None) == 2
    small = lib.afr_backward_workspace_bytes(17, 9, 2, 2) - 1
    assert lib.afr_reconstruct_backward(ctypes.byref(b), ctypes.byref(ok), ctypes.byref(p), *args[:5], 0x3000, small, None) == 4
    # build: negative n, too small a workspace
    s = afr._Samples(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, -1)
    assert lib.afr_build_deep_buffer(ctypes.byref(s), ctypes.byref(b), 0x4000, 1 << 30, None, None) == 1
    s = afr._Samples(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 1000)
    assert lib.afr_build_deep_buffer(ctypes.byref(s), ctypes.byref(b), 0x4000, 16, None, None) == 4
    s = afr._Samples(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 1 << 31)
    assert lib.afr_build_deep_buffer(ctypes.byref(s), ctypes.byref(b), 0x4000, 1 << 40, None, None) == 2
    # reprojection velocities come in pairs
    s = afr._Samples(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 1000, 0x1000, None)
    assert lib.afr_build_deep_buffer(ctypes.byref(s), ctypes.byref(b), 0x4000, 1 << 30, None, None) == 1
    s = afr._Samples(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 1000, None, 0x1000)
    assert lib.afr_build_deep_buffer(ctypes.byref(s), ctypes.byref(b), 0x4000, 1 << 30, None, None) == 1
    # staged build: four stage events, none of them NULL
    assert lib.afr_build_stage_count() == 4
    s = afr._Samples(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 1000)
    evs = (ctypes.c_void_p * 4)(0x10, 0x20, None, 0x40)
    assert lib.afr_build_deep_buffer_staged(ctypes.byref(s), ctypes.byref(b), 0x4000, 1 << 30, None, None, evs) == 1
    assert lib.afr_build_deep_buffer_staged(ctypes.byref(s), ctypes.byref(b), 0x4000, 1 << 30, None, None, None) == 1


def test_fp16_record_layout_is_checked(afr):
    """Binary16 slots are 12-byte records: field pointers that do not address one record array
    (separate planes, a misaligned base) are rejected (AFR_E_INVALID) before anything is launched;
    a consistent record array passes on to the next check (here a radius out of range,
    AFR_E_RANGE)."""
    lib = afr.library()
    p = afr.Params(t_now=11.0, radius=9)._c()
    st = afr._TileStats(8, 2, 1, 0x7000)
    ok = _fake_buffer(afr, prec=1)
    assert lib.afr_estimate_gradients(ctypes.byref(ok), ctypes.byref(p), ctypes.byref(st), None) == 2
    planes = afr._DeepBuffer(16, 8, 4, 1, 10.0, 0x1000, 0x2000, 0x3000, 0x4000, 0x5000, 0x6000,
                             0x1000, None)
    assert lib.afr_estimate_gradients(ctypes.byref(planes), ctypes.byref(p), ctypes.byref(st), None) == 1
    d = 0x1002  # not 4-byte aligned
    odd = afr._DeepBuffer(16, 8, 4, 1, 10.0, d, d + 2, d + 10, d + 4, d + 6, d + 8, 0x1000, None)
    assert lib.afr_estimate_gradients(ctypes.byref(odd), ctypes.byref(p), ctypes.byref(st), None) == 1
    swapped = afr._DeepBuffer(16, 8, 4, 1, 10.0, 0x1000, 0x1002, 0x1004, 0x1006, 0x1008, 0x100a,
                              0x1000, None)  # planar field order, not the record's
    assert lib.afr_estimate_gradients(ctypes.byref(swapped), ctypes.byref(p), ctypes.byref(st), None) == 1


def test_crosshair_validation(afr):
    """The crosshair calls fail validation before anything is launched: FP16 queues, missing index
    arrays, a small workspace, and a queue whose geometry differs from the sample buffer."""
    lib = afr.library()
    p = afr.Params(t_now=11.0)._c()
    s = afr._Samples(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 1000)
    xh = afr._Crosshairs(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 500)
    need = lib.afr_crosshair_workspace_bytes(500, 16, 8)
    assert need >= 6 * 500 * 4 + lib.afr_build_workspace_bytes(500, 16, 8, 4)
    b16 = _fake_buffer(afr, prec=1)
    assert lib.afr_build_crosshair_buffer(ctypes.byref(s), ctypes.byref(xh), ctypes.byref(p), ctypes.byref(b16), 0x4000, need, None, None) == 5
    b = _fake_buffer(afr)
    assert lib.afr_build_crosshair_buffer(ctypes.byref(s), ctypes.byref(xh), ctypes.byref(p), ctypes.byref(b), 0x4000, need - 1, None, None) == 4
    no_old = afr._Crosshairs(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, None, 500)
    assert lib.afr_build_crosshair_buffer(ctypes.byref(s), ctypes.byref(no_old), ctypes.byref(p), ctypes.byref(b), 0x4000, need, None, None) == 1
    neg = afr._Crosshairs(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, -1)
    assert lib.afr_build_crosshair_buffer(ctypes.byref(s), ctypes.byref(neg), ctypes.byref(p), ctypes.byref(b), 0x4000, need, None, None) == 1
    bad_p = afr.Params(t_now=11.0, dt_floor=0.0)._c()
    assert lib.afr_build_crosshair_buffer(ctypes.byref(s), ctypes.byref(xh), ctypes.byref(bad_p), ctypes.byref(b), 0x4000, need, None, None) == 2
    # estimate: the queue must be FP32 and of the sample buffer's size
    st = afr._TileStats(8, 2, 1, 0x1000)
    other = _fake_buffer(afr, w=24)
    assert lib.afr_estimate_gradients_crosshair(ctypes.byref(b), ctypes.byref(other), ctypes.byref(p), ctypes.byref(st), None) == 1
    assert lib.afr_estimate_gradients_crosshair(ctypes.byref(b), ctypes.byref(b16), ctypes.byref(p), ctypes.byref(st), None) == 5
    late = afr.Params(t_now=9.0)._c()   # before the buffers' t_ref
    assert lib.afr_estimate_gradients_crosshair(ctypes.byref(b), ctypes.byref(b), ctypes.byref(late), ctypes.byref(st), None) == 2


def test_scatter_validation(afr):
    lib = afr.library()
    sp = afr.SplatParams()
    assert lib.afr_splat_sizes(16, 8, None, ctypes.byref(sp._c()), None, None) == 1
    for bad in (dict(size_min=0.0), dict(size_default=0.5), dict(size_max=65.0),
                dict(grow=0.5), dict(shrink=0.0), dict(shrink=1.5), dict(n_low=40),
                dict(size_max=float("nan"))):
        b = afr.SplatParams(**{**sp.__dict__, **bad})
        assert lib.afr_splat_sizes(16, 8, None, ctypes.byref(b._c()), 0x1000, None) == 2, bad
    assert lib.afr_splat_sizes(0, 8, None, ctypes.byref(sp._c()), 0x1000, None) == 2
    b = _fake_buffer(afr)
    p = afr.Params(t_now=11.0)._c()
    st = afr._TileStats(8, 2, 1, 0x1000)
    for m in (0.0, 65.0, float("inf"), float("nan")):
        assert lib.afr_reconstruct_scatter(ctypes.byref(b), ctypes.byref(st), ctypes.byref(p), 0x2000, m, 0x3000, None, None, None) == 2
    assert lib.afr_reconstruct_scatter(ctypes.byref(b), ctypes.byref(st), ctypes.byref(p), None, 5.0, 0x3000, None, None, None) == 1
    assert lib.afr_reconstruct_scatter(ctypes.byref(b), ctypes.byref(st), ctypes.byref(p), 0x2000, 5.0, None, None, None, None) == 1


def test_sampler_validation(afr):
    lib = afr.library()
    b = _fake_buffer(afr)
    p = afr.Params(t_now=11.0)._c()
    st = afr._TileStats(8, 2, 1, 0x1000)
    need = lib.afr_sampler_workspace_bytes(2)
    assert need > 0 and lib.afr_sampler_workspace_bytes(0) == 0
    ok = afr.SamplerParams()
    args = (0x2000, 0x3000, 0x4000, 0x5000)
    for bad in (dict(kappa=-0.1), dict(kappa=0.8, lam=0.3), dict(m=-1.0), dict(gain=0.0),
                dict(gain=float("inf"))):
        sp = afr.SamplerParams(**{**ok.__dict__, **bad})
        assert lib.afr_sampler_stats(ctypes.byref(b), ctypes.byref(st), ctypes.byref(p), ctypes.byref(sp._c()), *args, need, None) == 2, bad
    assert lib.afr_sampler_stats(ctypes.byref(b), ctypes.byref(st), ctypes.byref(p), ctypes.byref(ok._c()), *args, need - 1, None) == 4
    assert lib.afr_sampler_stats(ctypes.byref(b), ctypes.byref(st), ctypes.byref(p), ctypes.byref(ok._c()), None, 0x3000, 0x4000, 0x5000, need, None) == 1
    # selection: at most 65536 tiles, a large enough workspace, arrays for n > 0
    big = lib.afr_sampler_workspace_bytes(1 << 20)
    assert lib.afr_sampler_select(4096, 4096, 8, 0x1000, 10, 0x2000, 0x3000, 0x4000, None, 0x5000, big, None) == 2
    assert lib.afr_sampler_select(64, 64, 8, 0x1000, 10, 0x2000, 0x3000, 0x4000, None, 0x5000, 16, None) == 4
    assert lib.afr_sampler_select(64, 64, 8, 0x1000, 10, None, 0x3000, 0x4000, None, 0x5000, big, None) == 1
    assert lib.afr_sampler_select(64, 64, 0, 0x1000, 10, 0x2000, 0x3000, 0x4000, None, 0x5000, big, None) == 2
    # the allocation-free variant: the same checks, up to 65536 tiles (its fixed array), no workspace
    assert lib.afr_sampler_select_noalloc(4096, 4096, 8, 0x1000, 10, 0x2000, 0x3000, 0x4000, None, None) == 2
    assert lib.afr_sampler_select_noalloc(2049, 2048, 8, 0x1000, 10, 0x2000, 0x3000, 0x4000, None, None) == 2
    assert lib.afr_sampler_select_noalloc(64, 64, 8, None, 10, 0x2000, 0x3000, 0x4000, None, None) == 1
    assert lib.afr_sampler_select_noalloc(64, 64, 8, 0x1000, 10, None, 0x3000, 0x4000, None, None) == 1
    assert lib.afr_sampler_select_noalloc(64, 64, 8, 0x1000, -1, 0x2000, 0x3000, 0x4000, None, None) == 1
    assert lib.afr_sampler_select_noalloc(64, 64, 0, 0x1000, 10, 0x2000, 0x3000, 0x4000, None, None) == 2
    assert lib.afr_sampler_select_noalloc(64, 64, 8, 0x1000, 1 << 31, 0x2000, 0x3000, 0x4000, None, None) == 2


def test_sampler_tile_weights_validation(afr):
    lib = afr.library()
    need = lib.afr_sampler_workspace_bytes(64)
    assert lib.afr_sampler_tile_weights(64, 64, 8, 0x1000, None, 0, 0x2000, 0x3000, need, None) == 1
    assert lib.afr_sampler_tile_weights(64, 64, 8, 0x1000, 0x4000, 0, 0x2000, 0x3000, need - 1, None) == 4
    assert lib.afr_sampler_tile_weights(4096, 4096, 4, 0x1000, None, 3, 0x2000, 0x3000, 1 << 30, None) == 2
    assert lib.afr_sampler_tile_weights(64, 64, 8, None, None, 3, 0x2000, 0x3000, need, None) == 1


def test_rms_loss_validation(afr):
    lib = afr.library()
    need = lib.afr_rms_workspace_bytes()
    assert need > 0
    assert lib.afr_rms_loss(0x1000, 0x2000, -1, 1.0, None, None, 0x3000, need, None) == 1
    assert lib.afr_rms_loss(None, 0x2000, 10, 1.0, None, None, 0x3000, need, None) == 1
    assert lib.afr_rms_loss(0x1000, 0x2000, 10, 1.0, None, None, None, need, None) == 1
    assert lib.afr_rms_loss(0x1000, 0x2000, 10, float("nan"), None, None, 0x3000, need, None) == 2
    assert lib.afr_rms_loss(0x1000, 0x2000, 10, 1.0, None, None, 0x3000, need - 1, None) == 4


def _batch_item(afr, w=16, h=8, k=4, tile=8, radius=2, prec=0):
    buf = _fake_buffer(afr, w=w, h=h, k=k, prec=prec)
    p = afr.Params(t_now=11.0).with_(tile=tile, radius=radius)._c()
    s = afr._TileStats(tile, (w + tile - 1) // tile, (h + tile - 1) // tile, 0x1000)
    return afr._BatchItem(buf, s, p, 0x1000, None)


def test_batch_plan_validation(afr):
    """The batch plan (afr_batch_create / run / tune / destroy) validates every item on the host
    before it uploads anything, and the plan calls reject a NULL plan."""
    lib = afr.library()
    assert lib.afr_batch_workspace_bytes(0) == 0
    assert lib.afr_batch_workspace_bytes(64) >= 64 * 8 * 8
    ws_ok = lib.afr_batch_workspace_bytes(2)
    plan = ctypes.c_void_p()

    def create(items, tpw=0, ws=0x1000, nbytes=ws_ok):
        arr = (afr._BatchItem * max(1, len(items)))(*items)
        return lib.afr_batch_create(arr if items else None, len(items), tpw, ws, nbytes,
                                    ctypes.byref(plan))

    good = [_batch_item(afr), _batch_item(afr, w=24, h=16)]
    assert create([]) == 1                                   # no items
    assert create(good, ws=None) == 1                        # no workspace
    assert create(good, nbytes=ws_ok - 1) == 4               # workspace too small
    assert create(good, tpw=3) == 2                          # launch shape outside 0, 1, 2, 4
    bad_k = [_batch_item(afr), _batch_item(afr, k=0)]
    assert create(bad_k) == 2                                # an invalid buffer
    assert create([_batch_item(afr, tile=4)]) == 5           # statistics tiles other than 8 px
    assert create([_batch_item(afr), _batch_item(afr, radius=1)]) == 5   # mixed radius
    assert create([_batch_item(afr), _batch_item(afr, prec=1)]) == 5     # mixed precision
    no_rgb = _batch_item(afr)
    no_rgb.rgb = None
    assert create([no_rgb]) == 1                             # no output image
    assert create([_batch_item(afr, radius=3)], tpw=4) == 2  # four tiles per group need R <= 2
    assert not plan.value
    assert lib.afr_batch_run(None, None) == 1
    assert lib.afr_batch_tune(None, None, None, None) == 1
    assert lib.afr_batch_tiles_per_wave(None) == 0
    lib.afr_batch_destroy(None)


def test_batch_reconstruct_validation(afr):
    """The plan-free batch call (afr_batch_reconstruct) validates the items and its tune struct on
    the host before it enqueues anything, with afr_batch_create's status codes."""
    lib = afr.library()
    ws_ok = lib.afr_batch_workspace_bytes(2)

    def call(items, tpw=0, ws=0x1000, nbytes=ws_ok, tune=True):
        arr = (afr._BatchItem * max(1, len(items)))(*items)
        t = afr._Tune(tpw, ws, nbytes)
        return lib.afr_batch_reconstruct(arr if items else None, len(items),
                                         ctypes.byref(t) if tune else None, None)

    good = [_batch_item(afr), _batch_item(afr, w=24, h=16)]
    assert call([]) == 1                                     # no items
    assert call(good, tune=False) == 1                       # no tune struct
    assert call(good, ws=None) == 1                          # no workspace
    assert call(good, nbytes=ws_ok - 1) == 4                 # workspace too small
    assert call(good, tpw=3) == 2                            # launch shape outside 0, 1, 2, 4
    assert call([_batch_item(afr), _batch_item(afr, k=0)]) == 2           # an invalid buffer
    assert call([_batch_item(afr, tile=4)]) == 5             # statistics tiles other than 8 px
    assert call([_batch_item(afr), _batch_item(afr, radius=1)]) == 5      # mixed radius
    assert call([_batch_item(afr), _batch_item(afr, prec=1)]) == 5        # mixed precision
    assert call([_batch_item(afr, radius=3)], tpw=4) == 2    # four tiles per group need R <= 2
