"""FP64 reference ("oracle") for adaptive frameless reconstruction.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps the plain C reference in ``afr_oracle.c`` (built
with gcc into ``_liboracle.so``) and shares nothing with the GPU library: no code, headers, tables
or constants. Inputs come from ``afr_scenes`` (random draws and analytic scenes only).

Layouts follow the C file: slot planes ``[H, W, K]`` (slot 0 newest), ``count [H, W]``, tile
statistics ``[NSTAT, Ty, Tx]``, images ``[3, H, W]``, ``aux [2, H, W] = (E_max, W')``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "afr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")

STAT_NAMES = ("gx", "gy", "gt", "vol", "var", "lmean", "ex2", "ey2", "sx2", "sy2", "kt2")
NSTAT = len(STAT_NAMES)
STAT = {n: i for i, n in enumerate(STAT_NAMES)}


# gcc flags of the reference: no fast-math, no FP contraction; OpenMP over rows (every output
# element is computed by one thread in the single-thread order, so results do not depend on the
# thread count).
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile the C reference with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def source_path() -> str:
    return _SRC


def num_threads() -> int:
    """Threads the reference's parallel loops use (OMP_NUM_THREADS, else the host's cores)."""
    return int(_lib().or_num_threads())


def set_num_threads(n: int) -> None:
    _lib().or_set_num_threads(int(n))


class _Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("tau", ctypes.c_double), ("alpha", ctypes.c_double),
                ("e_min", ctypes.c_double), ("e_max", ctypes.c_double),
                ("g_floor", ctypes.c_double), ("dt_floor", ctypes.c_double),
                ("age_floor", ctypes.c_double), ("t_now", ctypes.c_double),
                ("radius", ctypes.c_int), ("tile", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)


class _Buffer(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("height", ctypes.c_int), ("k", ctypes.c_int),
                ("fp16", ctypes.c_int), ("t_ref", ctypes.c_double),
                ("ox", _dp), ("oy", _dp), ("ta", _dp), ("r", _dp), ("g", _dp), ("b", _dp),
                ("count", ctypes.POINTER(ctypes.c_uint8)), ("src", ctypes.POINTER(ctypes.c_int32))]


class _Splat(ctypes.Structure):
    _fields_ = [("size_default", ctypes.c_float), ("size_min", ctypes.c_float),
                ("size_max", ctypes.c_float), ("grow", ctypes.c_float), ("shrink", ctypes.c_float),
                ("n_low", ctypes.c_int), ("n_high", ctypes.c_int)]


class _Sampler(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("lambda_", ctypes.c_double), ("m", ctypes.c_double),
                ("gain", ctypes.c_double)]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        path = os.environ.get("AFR_ORACLE_LIB")  # another build of afr_oracle.c (sanitizers)
        if not path:
            path = _LIB_PATH
            if not os.path.exists(path):
                build(force=False)
        lib = ctypes.CDLL(path)
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_num_threads.argtypes = []
        lib.or_set_num_threads.restype = None
        lib.or_set_num_threads.argtypes = [ctypes.c_int]
        fp = ctypes.POINTER(ctypes.c_float)
        lib.or_f16_round.restype = ctypes.c_double
        lib.or_f16_round.argtypes = [ctypes.c_double]
        lib.or_build.restype = ctypes.c_int
        lib.or_build.argtypes = [ctypes.c_int64, fp, fp, fp, fp, fp, fp, fp, fp,
                                 ctypes.POINTER(_Buffer), ctypes.POINTER(ctypes.c_int64)]
        lib.or_pixel_stats.restype = ctypes.c_int
        lib.or_pixel_stats.argtypes = [ctypes.POINTER(_Buffer), ctypes.POINTER(_Params)] + [_dp] * 5
        lib.or_extents.restype = None
        lib.or_extents.argtypes = [ctypes.c_double] * 4 + [ctypes.POINTER(_Params), _dp]
        lib.or_estimate.restype = ctypes.c_int
        lib.or_estimate.argtypes = [ctypes.POINTER(_Buffer), ctypes.POINTER(_Params), _dp]
        lib.or_reconstruct.restype = ctypes.c_int
        lib.or_reconstruct.argtypes = [ctypes.POINTER(_Buffer), _dp, ctypes.POINTER(_Params), _dp, _dp]
        lib.or_backward.restype = ctypes.c_int
        lib.or_backward.argtypes = [ctypes.POINTER(_Buffer), _dp, ctypes.POINTER(_Params), _dp, _dp, _dp]
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.or_crosshair_records.restype = ctypes.c_int
        lib.or_crosshair_records.argtypes = ([ctypes.c_int64] + [fp] * 6 + [ctypes.c_int64]
                                             + [ip] * 6 + [ctypes.c_double] + [fp] * 3 + [_dp] * 3)
        lib.or_crosshair_tiles.restype = ctypes.c_int
        lib.or_crosshair_tiles.argtypes = [ctypes.POINTER(_Buffer), ctypes.POINTER(_Params), _dp]
        lib.or_scatter.restype = ctypes.c_int
        lib.or_scatter.argtypes = [ctypes.POINTER(_Buffer), _dp, ctypes.POINTER(_Params), fp,
                                   ctypes.c_float, _dp, _dp, fp, fp]
        lib.or_splat_sizes.restype = None
        lib.or_splat_sizes.argtypes = [ctypes.c_int, ctypes.c_int, fp, fp,
                                       ctypes.POINTER(_Splat), fp]
        lib.or_sampler_stats.restype = ctypes.c_int
        lib.or_sampler_stats.argtypes = [ctypes.POINTER(_Buffer), _dp, ctypes.POINTER(_Params),
                                         ctypes.POINTER(_Sampler), _dp, _dp, _dp]
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.or_sampler_select.restype = ctypes.c_int
        lib.or_sampler_select.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, fp,
                                          ctypes.c_int64, u32p, fp, fp,
                                          ctypes.POINTER(ctypes.c_int32)]
        lib.or_sampler_tile_weights.restype = ctypes.c_int
        lib.or_sampler_tile_weights.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, fp,
                                                ctypes.c_double, ctypes.c_int, fp]
        _lib_handle = lib
    return _lib_handle


@dataclass
class Params:
    """Filter constants. ``alpha`` is 3.47 per second (Sec. 4), expressed per millisecond."""
    sigma: float = 1.0
    tau: float = 0.5
    alpha: float = 3.47e-3
    e_min: float = 0.5
    e_max: float = 1.0
    g_floor: float = 1e-3
    dt_floor: float = 1e-3
    age_floor: float = 1e-3
    t_now: float = 0.0
    radius: int = 2
    tile: int = 8

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)

    def _c(self) -> _Params:
        return _Params(float(self.sigma), float(self.tau), float(self.alpha), float(self.e_min),
                       float(self.e_max), float(self.g_floor), float(self.dt_floor),
                       float(self.age_floor), float(self.t_now), int(self.radius), int(self.tile))


@dataclass
class Buffer:
    """Per-pixel deep buffer in FP64 (FP16 mode holds binary16-rounded values)."""
    width: int
    height: int
    k: int
    fp16: bool
    t_ref: float
    ox: np.ndarray
    oy: np.ndarray
    ta: np.ndarray
    r: np.ndarray
    g: np.ndarray
    b: np.ndarray
    count: np.ndarray
    src: np.ndarray

    @staticmethod
    def empty(width, height, k, fp16=False, t_ref=0.0) -> "Buffer":
        z = lambda: np.zeros((height, width, k), np.float64)
        return Buffer(width, height, k, bool(fp16), float(t_ref), z(), z(), z(), z(), z(), z(),
                      np.zeros((height, width), np.uint8), np.full((height, width, k), -1, np.int32))

    def colours(self) -> np.ndarray:
        return np.stack([self.r, self.g, self.b])

    def with_colours(self, rgb) -> "Buffer":
        rgb = np.asarray(rgb, np.float64)
        return replace(self, r=rgb[0].copy(), g=rgb[1].copy(), b=rgb[2].copy())

    def _c(self) -> _Buffer:
        for a in (self.ox, self.oy, self.ta, self.r, self.g, self.b):
            assert a.dtype == np.float64 and a.flags.c_contiguous
            assert a.shape == (self.height, self.width, self.k)
        assert self.count.dtype == np.uint8 and self.count.flags.c_contiguous
        assert self.src.dtype == np.int32 and self.src.flags.c_contiguous
        d = lambda a: a.ctypes.data_as(_dp)
        return _Buffer(self.width, self.height, self.k, int(self.fp16), float(self.t_ref),
                       d(self.ox), d(self.oy), d(self.ta), d(self.r), d(self.g), d(self.b),
                       self.count.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                       self.src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def f16_round(v) -> np.ndarray:
    lib = _lib()
    v = np.asarray(v, np.float64)
    return np.array([lib.or_f16_round(float(a)) for a in v.reshape(-1)]).reshape(v.shape)


def build_buffer(stream, width, height, k, precision="fp32", t_ref=None, reproject=False):
    """Per-pixel deep buffer from a stream; returns ``(Buffer, dropped)``. With ``reproject`` the
    stream's velocities advance every sample to ``t_ref`` first (see or_build)."""
    x, y, t, r, g, b = (np.ascontiguousarray(a, np.float32) for a in stream.arrays())
    vel = stream.motion() if reproject else None
    if reproject and vel is None:
        raise ValueError("reproject=True needs a stream with velocities")
    vx, vy = (None, None) if vel is None else (np.ascontiguousarray(a, np.float32) for a in vel)
    if t_ref is None:
        t_ref = float(t.max()) if t.size else 0.0
    buf = Buffer.empty(width, height, k, precision == "fp16", float(np.float32(t_ref)))
    bc = buf._c()
    dropped = ctypes.c_int64(0)
    fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    fpn = lambda a: None if a is None else fp(a)
    rc = _lib().or_build(len(x), fp(x), fp(y), fp(t), fp(r), fp(g), fp(b), fpn(vx), fpn(vy),
                         ctypes.byref(bc), ctypes.byref(dropped))
    if rc:
        raise ValueError(f"or_build failed ({rc})")
    return buf, int(dropped.value)


def pixel_stats(buf: Buffer, params: Params) -> dict:
    hw = (buf.height, buf.width)
    outs = [np.zeros(hw, np.float64) for _ in range(5)]
    rc = _lib().or_pixel_stats(ctypes.byref(buf._c()), ctypes.byref(params._c()),
                               *(o.ctypes.data_as(_dp) for o in outs))
    if rc:
        raise ValueError(f"or_pixel_stats failed ({rc})")
    return dict(zip(("lbar", "omega", "gx", "gy", "gt"), outs))


def extents(gx, gy, gt, vol, params: Params) -> dict:
    out = np.zeros(5, np.float64)
    _lib().or_extents(float(gx), float(gy), float(gt), float(vol), ctypes.byref(params._c()),
                      out.ctypes.data_as(_dp))
    return dict(zip(("ex2", "ey2", "sx2", "sy2", "kt2"), out))


def tiles_shape(width, height, tile):
    return (-(-height // tile), -(-width // tile))


def estimate(buf: Buffer, params: Params) -> np.ndarray:
    ty, tx = tiles_shape(buf.width, buf.height, params.tile)
    stats = np.zeros((NSTAT, ty, tx), np.float64)
    rc = _lib().or_estimate(ctypes.byref(buf._c()), ctypes.byref(params._c()),
                            stats.ctypes.data_as(_dp))
    if rc:
        raise ValueError(f"or_estimate failed ({rc})")
    return stats


def reconstruct(buf: Buffer, stats: np.ndarray, params: Params):
    stats = np.ascontiguousarray(stats, np.float64)
    rgb = np.zeros((3, buf.height, buf.width), np.float64)
    aux = np.zeros((2, buf.height, buf.width), np.float64)
    rc = _lib().or_reconstruct(ctypes.byref(buf._c()), stats.ctypes.data_as(_dp),
                               ctypes.byref(params._c()), rgb.ctypes.data_as(_dp),
                               aux.ctypes.data_as(_dp))
    if rc:
        raise ValueError(f"or_reconstruct failed ({rc})")
    return rgb, aux


def backward(buf: Buffer, stats: np.ndarray, params: Params, grad_rgb):
    stats = np.ascontiguousarray(stats, np.float64)
    grad_rgb = np.ascontiguousarray(grad_rgb, np.float64)
    gslot = np.zeros((3, buf.height, buf.width, buf.k), np.float64)
    gpar = np.zeros(2, np.float64)
    rc = _lib().or_backward(ctypes.byref(buf._c()), stats.ctypes.data_as(_dp),
                            ctypes.byref(params._c()), grad_rgb.ctypes.data_as(_dp),
                            gslot.ctypes.data_as(_dp), gpar.ctypes.data_as(_dp))
    if rc:
        raise ValueError(f"or_backward failed ({rc})")
    return gslot, gpar


def forward(buf: Buffer, params: Params):
    """Estimate then reconstruct: ``(rgb, aux, stats)``."""
    stats = estimate(buf, params)
    rgb, aux = reconstruct(buf, stats, params)
    return rgb, aux, stats


def rms(img, gt) -> float:
    """Root-mean-square error over pixels and channels (the gold-standard comparison of Sec. 7)."""
    d = np.asarray(img, np.float64) - np.asarray(gt, np.float64)
    return float(np.sqrt(np.mean(d * d)))


def rms_grad(img, gt, scale=1.0):
    """d(scale * RMS)/d img."""
    d = np.asarray(img, np.float64) - np.asarray(gt, np.float64)
    e = float(np.sqrt(np.mean(d * d)))
    if e == 0.0:
        return np.zeros_like(d)
    return scale * d / (d.size * e)


# ---- crosshair gradients (Sec. 4.1) --------------------------------------------------------------

_XH_FIELDS = ("centre", "xm", "xp", "ym", "yp", "old")


def crosshair_records(stream, xh, dt_floor=1e-3):
    """Per-crosshair records: ``(cx, cy, ct)`` float32 (NaN position for a dropped crosshair) and
    ``(gx, gy, gt)`` in FP64 (-1 where undefined); see or_crosshair_records."""
    x, y, t, r, g, b = (np.ascontiguousarray(a, np.float32) for a in stream.arrays())
    idx = [np.ascontiguousarray(getattr(xh, f), np.int32) for f in _XH_FIELDS]
    n = int(idx[0].shape[0])
    assert all(int(a.shape[0]) == n for a in idx)
    c3 = [np.zeros(n, np.float32) for _ in range(3)]
    g3 = [np.zeros(n, np.float64) for _ in range(3)]
    fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    rc = _lib().or_crosshair_records(len(x), fp(x), fp(y), fp(t), fp(r), fp(g), fp(b), n,
                                     *(ip(a) for a in idx), float(dt_floor), *(fp(a) for a in c3),
                                     *(a.ctypes.data_as(_dp) for a in g3))
    if rc != 0:
        raise ValueError(f"or_crosshair_records failed ({rc})")
    return c3, g3


def crosshair_buffer(stream, xh, width, height, k, t_ref, dt_floor=1e-3):
    """The sampler's per-pixel crosshair queues (Sec. 4.1): each crosshair's record is pushed into
    the queue of its centre pixel, which keeps the ``k`` newest (FP32; gradients in r, g, b).
    Returns ``(Buffer, dropped)``."""
    from afr_scenes import Stream
    (cx, cy, ct), g3 = crosshair_records(stream, xh, dt_floor)
    rec = Stream(cx, cy, ct, *(a.astype(np.float32) for a in g3))
    return build_buffer(rec, width, height, k, "fp32", t_ref)


def estimate_crosshair(buf: Buffer, xbuf: Buffer, params: Params) -> np.ndarray:
    """Tile statistics with the gradient planes taken from the crosshair queues ``xbuf`` and the
    extents recomputed from them (volume, variance and mean luminance from ``buf``)."""
    stats = estimate(buf, params)
    rc = _lib().or_crosshair_tiles(ctypes.byref(xbuf._c()), ctypes.byref(params._c()),
                                   stats.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError(f"or_crosshair_tiles failed ({rc})")
    return stats


# ---- scatter form and adaptive splat size (Sec. 5.2, 6.2) ----------------------------------------

@dataclass
class SplatParams:
    """Adaptive splat size (Sec. 6.2): grow 4x below 4 splats per pixel, shrink 0.7x above 32.
    Sizes are splat edge lengths in px; the defaults start at the gather's 5 x 5 block."""
    size_default: float = 5.0
    size_min: float = 1.0
    size_max: float = 16.0
    grow: float = 4.0
    shrink: float = 0.7
    n_low: int = 4
    n_high: int = 32

    def _c(self) -> _Splat:
        return _Splat(self.size_default, self.size_min, self.size_max, self.grow, self.shrink,
                      int(self.n_low), int(self.n_high))


def splat_sizes(width, height, coverage, sp: SplatParams) -> np.ndarray:
    """Per-pixel splat size [H, W] float32 for the next image from this image's coverage map
    ``(n, mean size)`` (each [H, W] float32), or from nothing (``coverage=None``: the first image)."""
    fp = lambda a: None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    n = sz = None
    if coverage is not None:
        n, sz = (np.ascontiguousarray(a, np.float32) for a in coverage)
    out = np.zeros((height, width), np.float32)
    _lib().or_splat_sizes(int(width), int(height), fp(n), fp(sz), ctypes.byref(sp._c()), fp(out))
    return out


def scatter(buf: Buffer, stats: np.ndarray, params: Params, size, max_size: float):
    """Scatter-form image: ``(rgb [3,H,W], aux [2,H,W], (n, mean size))`` with per-source-pixel splat
    sizes ``size`` [H, W] (see or_scatter)."""
    stats = np.ascontiguousarray(stats, np.float64)
    size = np.ascontiguousarray(size, np.float32)
    H, W = buf.height, buf.width
    rgb = np.zeros((3, H, W), np.float64)
    aux = np.zeros((2, H, W), np.float64)
    n = np.zeros((H, W), np.float32)
    ms = np.zeros((H, W), np.float32)
    fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    rc = _lib().or_scatter(ctypes.byref(buf._c()), stats.ctypes.data_as(_dp),
                           ctypes.byref(params._c()), fp(size), float(max_size),
                           rgb.ctypes.data_as(_dp), aux.ctypes.data_as(_dp), fp(n), fp(ms))
    if rc:
        raise ValueError(f"or_scatter failed ({rc})")
    return rgb, aux, (n, ms)


# ---- sampler feedback statistics and tile selection (Sec. 4, 4.1, 6.1) ---------------------------

SAMPLER_GLOBALS = ("sum_v", "sum_u", "mean_empty", "dcds", "dcdt", "mean_age", "S", "target_tiles")


@dataclass
class SamplerParams:
    """Tile error weights (Sec. 6.1: kappa for variation, lambda for undersampling; the occlusion
    share 1 - kappa - lambda has no term here), the undersampling factor m and the gain constant i
    of Sec. 4.1."""
    kappa: float = 0.7
    lam: float = 0.3
    m: float = 2.0
    gain: float = 4.0

    def _c(self) -> _Sampler:
        return _Sampler(float(self.kappa), float(self.lam), float(self.m), float(self.gain))


def sampler_stats(buf: Buffer, stats: np.ndarray, params: Params, sp: SamplerParams):
    """``(E [Ty, Tx], u [Ty, Tx], globals dict)`` from the sampler's buffer and its statistics."""
    ty, tx = tiles_shape(buf.width, buf.height, params.tile)
    stats = np.ascontiguousarray(stats, np.float64)
    E = np.zeros((ty, tx))
    u = np.zeros((ty, tx))
    g = np.zeros(len(SAMPLER_GLOBALS))
    rc = _lib().or_sampler_stats(ctypes.byref(buf._c()), stats.ctypes.data_as(_dp),
                                 ctypes.byref(params._c()), ctypes.byref(sp._c()),
                                 E.ctypes.data_as(_dp), u.ctypes.data_as(_dp), g.ctypes.data_as(_dp))
    if rc:
        raise ValueError(f"or_sampler_stats failed ({rc})")
    return E, u, dict(zip(SAMPLER_GLOBALS, g))


def sampler_select(width, height, tile, E, rnd):
    """Sample spots for the next samples: ``(x, y, tile index)`` for ``n = len(rnd) // 3`` draws;
    ``E`` is the float32 tile error [Ty, Tx], ``rnd`` uint32 [3 n] (see or_sampler_select)."""
    E = np.ascontiguousarray(E, np.float32)
    rnd = np.ascontiguousarray(rnd, np.uint32)
    n = rnd.size // 3
    x = np.zeros(n, np.float32)
    y = np.zeros(n, np.float32)
    t = np.zeros(n, np.int32)
    fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    rc = _lib().or_sampler_select(int(width), int(height), int(tile), fp(E), n,
                                  rnd.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), fp(x), fp(y),
                                  t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise ValueError(f"or_sampler_select failed ({rc})")
    return x, y, t


def sampler_tile_weights(width, height, tile, E, target=1.0, n_parts=0):
    """Equal-error tile weights [Ty, Tx] float32 (see or_sampler_tile_weights): ``n_parts`` parts,
    or the gain-control ``target`` tile count rounded and clamped when ``n_parts`` is 0."""
    E = np.ascontiguousarray(E, np.float32)
    out = np.zeros(E.shape, np.float32)
    fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    rc = _lib().or_sampler_tile_weights(int(width), int(height), int(tile), fp(E), float(target),
                                        int(n_parts), fp(out))
    if rc:
        raise ValueError(f"or_sampler_tile_weights failed ({rc})")
    return out
