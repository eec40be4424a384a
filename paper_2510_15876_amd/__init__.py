"""Adaptive frameless reconstruction on MI355X: Python binding of ``libafr.so``.

The binding only marshals arguments: every step of the reconstruction path runs in the HIP kernels
behind the C ABI declared in ``include/afr.h``. PyTorch supplies device memory and the current HIP
stream. There is no CPU fallback: calls fail loudly when the library is missing or no GPU is present.

Function names follow the C ABI: ``build_deep_buffer``, ``estimate_gradients``, ``reconstruct``,
``reconstruct_plain``, ``reconstruct_backward``; ``ReconstructFn`` wraps forward and adjoint as a
``torch.autograd.Function`` with gradients for the sample colours and for ``sigma`` and ``tau``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, replace
from typing import Optional

import torch

__all__ = [
    "AfrError", "Params", "DeepBuffer", "STAT_NAMES", "NSTAT", "STAT", "library", "lib_path",
    "build_deep_buffer", "estimate_gradients", "forward", "reconstruct", "reconstruct_plain",
    "reconstruct_launch",
    "reconstruct_backward", "ReconstructFn", "reconstruct_differentiable", "tiles_shape",
    "reconstruct_tune", "Batch", "build_crosshair_buffer", "estimate_gradients_crosshair",
    "SplatParams", "splat_sizes", "reconstruct_scatter", "SamplerParams", "sampler_stats",
    "sampler_select", "sampler_select_noalloc", "sampler_tile_weights", "SAMPLER_GLOBALS",
    "rms_loss",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libafr.so")

STAT_NAMES = ("gx", "gy", "gt", "vol", "var", "lmean", "ex2", "ey2", "sx2", "sy2", "kt2")
NSTAT = len(STAT_NAMES)
STAT = {n: i for i, n in enumerate(STAT_NAMES)}
PRECISIONS = {"fp32": 0, "fp16": 1}


class AfrError(RuntimeError):
    pass


# ---- C structs (mirror include/afr.h) ------------------------------------------------------------

class _Samples(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("g", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("vx", ctypes.c_void_p), ("vy", ctypes.c_void_p)]


class _Tune(ctypes.Structure):
    _fields_ = [("tiles_per_wave", ctypes.c_int32), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t)]


class _Crosshairs(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_void_p), ("xm", ctypes.c_void_p), ("xp", ctypes.c_void_p),
                ("ym", ctypes.c_void_p), ("yp", ctypes.c_void_p), ("old", ctypes.c_void_p),
                ("n", ctypes.c_int64)]


class _DeepBuffer(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("k", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("t_ref", ctypes.c_float),
                ("ox", ctypes.c_void_p), ("oy", ctypes.c_void_p), ("tage", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("g", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("src", ctypes.c_void_p)]


class _TileStats(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("tiles_x", ctypes.c_int32),
                ("tiles_y", ctypes.c_int32), ("data", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_float), ("tau", ctypes.c_float), ("alpha", ctypes.c_float),
                ("e_min", ctypes.c_float), ("e_max", ctypes.c_float),
                ("g_floor", ctypes.c_float), ("dt_floor", ctypes.c_float),
                ("age_floor", ctypes.c_float), ("radius", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("t_now", ctypes.c_float)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("buf", _DeepBuffer), ("stats", _TileStats), ("params", _Params),
                ("rgb", ctypes.c_void_p), ("aux", ctypes.c_void_p)]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def library():
    """Load libafr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise AfrError(f"{_LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    vp, st = ctypes.c_void_p, ctypes.c_int
    lib.afr_status_string.restype = ctypes.c_char_p
    lib.afr_status_string.argtypes = [st]
    lib.afr_version.restype = ctypes.c_char_p
    lib.afr_version.argtypes = []
    lib.afr_build_workspace_bytes.restype = ctypes.c_size_t
    lib.afr_build_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32]
    lib.afr_build_deep_buffer.restype = st
    lib.afr_build_deep_buffer.argtypes = [P(_Samples), P(_DeepBuffer), vp, ctypes.c_size_t, vp, vp]
    lib.afr_build_stage_count.restype = ctypes.c_int32
    lib.afr_build_stage_count.argtypes = []
    lib.afr_build_deep_buffer_staged.restype = st
    lib.afr_build_deep_buffer_staged.argtypes = [P(_Samples), P(_DeepBuffer), vp, ctypes.c_size_t,
                                                 vp, vp, P(vp)]
    lib.afr_estimate_gradients.restype = st
    lib.afr_estimate_gradients.argtypes = [P(_DeepBuffer), P(_Params), P(_TileStats), vp]
    lib.afr_rms_workspace_bytes.restype = ctypes.c_size_t
    lib.afr_rms_workspace_bytes.argtypes = []
    lib.afr_rms_loss.restype = st
    lib.afr_rms_loss.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, vp, vp, vp,
                                 ctypes.c_size_t, vp]
    lib.afr_sampler_workspace_bytes.restype = ctypes.c_size_t
    lib.afr_sampler_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.afr_sampler_stats.restype = st
    lib.afr_sampler_stats.argtypes = [P(_DeepBuffer), P(_TileStats), P(_Params), P(_SamplerParams),
                                      vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.afr_sampler_tile_weights.restype = st
    lib.afr_sampler_tile_weights.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                             ctypes.c_int32, vp, vp, ctypes.c_size_t, vp]
    lib.afr_sampler_select.restype = st
    lib.afr_sampler_select.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                       ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.afr_splat_sizes.restype = st
    lib.afr_splat_sizes.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, P(_SplatParams), vp, vp]
    lib.afr_reconstruct_scatter.restype = st
    lib.afr_reconstruct_scatter.argtypes = [P(_DeepBuffer), P(_TileStats), P(_Params), vp,
                                            ctypes.c_float, vp, vp, vp, vp]
    lib.afr_crosshair_workspace_bytes.restype = ctypes.c_size_t
    lib.afr_crosshair_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    lib.afr_build_crosshair_buffer.restype = st
    lib.afr_build_crosshair_buffer.argtypes = [P(_Samples), P(_Crosshairs), P(_Params),
                                               P(_DeepBuffer), vp, ctypes.c_size_t, vp, vp]
    lib.afr_estimate_gradients_crosshair.restype = st
    lib.afr_estimate_gradients_crosshair.argtypes = [P(_DeepBuffer), P(_DeepBuffer), P(_Params),
                                                     P(_TileStats), vp]
    for name in ("afr_reconstruct", "afr_reconstruct_plain"):
        f = getattr(lib, name)
        f.restype = st
        f.argtypes = [P(_DeepBuffer), P(_TileStats), P(_Params), vp, vp, vp]
    lib.afr_reconstruct_tune.restype = st
    lib.afr_reconstruct_tune.argtypes = [P(_DeepBuffer), P(_TileStats), P(_Params), vp,
                                         P(ctypes.c_int32), P(ctypes.c_float), vp]
    lib.afr_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.afr_batch_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.afr_batch_create.restype = st
    lib.afr_batch_create.argtypes = [P(_BatchItem), ctypes.c_int32, ctypes.c_int32, vp,
                                     ctypes.c_size_t, P(vp)]
    lib.afr_batch_run.restype = st
    lib.afr_batch_run.argtypes = [vp, vp]
    lib.afr_batch_tune.restype = st
    lib.afr_batch_tune.argtypes = [vp, vp, P(ctypes.c_int32), P(ctypes.c_float)]
    lib.afr_batch_tiles_per_wave.restype = ctypes.c_int32
    lib.afr_batch_tiles_per_wave.argtypes = [vp]
    lib.afr_batch_reconstruct.restype = st
    lib.afr_batch_reconstruct.argtypes = [P(_BatchItem), ctypes.c_int32, P(_Tune), vp]
    lib.afr_batch_destroy.restype = None
    lib.afr_batch_destroy.argtypes = [vp]
    lib.afr_sampler_select_noalloc.restype = st
    lib.afr_sampler_select_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                               ctypes.c_int64, vp, vp, vp, vp, vp]
    lib.afr_reconstruct_launch.restype = st
    lib.afr_reconstruct_launch.argtypes = [P(_DeepBuffer), P(_TileStats), P(_Params), ctypes.c_int32,
                                           vp, vp, vp]
    lib.afr_forward.restype = st
    lib.afr_forward.argtypes = [P(_DeepBuffer), P(_Params), P(_TileStats), vp, vp, vp]
    lib.afr_backward_workspace_bytes.restype = ctypes.c_size_t
    lib.afr_backward_workspace_bytes.argtypes = [ctypes.c_int32] * 4
    lib.afr_reconstruct_backward.restype = st
    lib.afr_reconstruct_backward.argtypes = [P(_DeepBuffer), P(_TileStats), P(_Params), vp, vp, vp,
                                             vp, vp, vp, ctypes.c_size_t, vp]
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        msg = library().afr_status_string(status).decode()
        raise AfrError(f"{what}: {msg} (status {status})")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise AfrError("libafr takes device tensors")
    if not t.is_contiguous():
        raise AfrError("libafr takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ---- Python-side containers ----------------------------------------------------------------------

@dataclass
class Params:
    """Filter constants (see ``afr_params`` in include/afr.h)."""
    sigma: float = 1.0
    tau: float = 0.5
    alpha: float = 3.47e-3
    e_min: float = 0.5
    e_max: float = 1.0
    g_floor: float = 1e-3
    dt_floor: float = 1e-3
    age_floor: float = 1e-3
    radius: int = 2
    tile: int = 8
    t_now: float = 0.0

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)

    def _c(self) -> _Params:
        return _Params(self.sigma, self.tau, self.alpha, self.e_min, self.e_max, self.g_floor,
                       self.dt_floor, self.age_floor, int(self.radius), int(self.tile),
                       self.t_now)


class _SplatParams(ctypes.Structure):
    _fields_ = [("size_default", ctypes.c_float), ("size_min", ctypes.c_float),
                ("size_max", ctypes.c_float), ("grow", ctypes.c_float), ("shrink", ctypes.c_float),
                ("n_low", ctypes.c_int32), ("n_high", ctypes.c_int32)]


@dataclass
class SplatParams:
    """Adaptive splat size (see ``afr_splat_params`` in include/afr.h)."""
    size_default: float = 5.0
    size_min: float = 1.0
    size_max: float = 16.0
    grow: float = 4.0
    shrink: float = 0.7
    n_low: int = 4
    n_high: int = 32

    def _c(self) -> _SplatParams:
        return _SplatParams(self.size_default, self.size_min, self.size_max, self.grow,
                            self.shrink, int(self.n_low), int(self.n_high))


class _SamplerParams(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_float), ("lambda_", ctypes.c_float), ("m", ctypes.c_float),
                ("gain", ctypes.c_float)]


@dataclass
class SamplerParams:
    """Sampler feedback weights (see ``afr_sampler_params`` in include/afr.h)."""
    kappa: float = 0.7
    lam: float = 0.3
    m: float = 2.0
    gain: float = 4.0

    def _c(self) -> _SamplerParams:
        return _SamplerParams(self.kappa, self.lam, self.m, self.gain)


SAMPLER_GLOBALS = ("sum_v", "sum_u", "mean_empty", "dcds", "dcdt", "mean_age", "S", "target_tiles")


def tiles_shape(width: int, height: int, tile: int):
    return (-(-height // tile), -(-width // tile))


class DeepBuffer:
    """Per-pixel deep buffer in device memory (plane k holds every pixel's k-th newest sample),
    ``count[H, W]`` (uint8) and ``src[K, H, W]`` (int32 stream index, -1 when empty).

    ``planes`` is ``[6, K, H, W]`` float32 (ox, oy, tage, r, g, b) for FP32 storage, and for FP16
    storage ``[K, H, W, 6]`` binary16 slot records in the order (ox, oy, r, g, b, tage), the layout
    of afr.h. ``field(name)`` returns a ``[K, H, W]`` view of one field either way."""

    FIELDS = ("ox", "oy", "tage", "r", "g", "b")
    RECORD = ("ox", "oy", "r", "g", "b", "tage")  # binary16 slot record order

    def __init__(self, width: int, height: int, k: int, precision: str = "fp32",
                 t_ref: float = 0.0, device="cuda", with_src: bool = True):
        if precision not in PRECISIONS:
            raise AfrError(f"precision must be one of {tuple(PRECISIONS)}")
        self.width, self.height, self.k = int(width), int(height), int(k)
        self.precision = precision
        self.t_ref = float(t_ref)
        if precision == "fp16":
            self.planes = torch.empty((self.k, self.height, self.width, 6), dtype=torch.float16,
                                      device=device)
        else:
            self.planes = torch.empty((6, self.k, self.height, self.width), dtype=torch.float32,
                                      device=device)
        self.count = torch.empty((self.height, self.width), dtype=torch.uint8, device=device)
        self.src = (torch.empty((self.k, self.height, self.width), dtype=torch.int32, device=device)
                    if with_src else None)

    def field(self, name: str) -> torch.Tensor:
        if self.precision == "fp16":
            return self.planes[..., self.RECORD.index(name)]
        return self.planes[self.FIELDS.index(name)]

    def colours(self) -> torch.Tensor:
        """The colour fields as ``[3, K, H, W]`` (a view; not contiguous for FP16 records)."""
        if self.precision == "fp16":
            return self.planes[..., 2:5].permute(3, 0, 1, 2)
        return self.planes[3:6]

    def clone(self) -> "DeepBuffer":
        o = DeepBuffer.__new__(DeepBuffer)
        o.width, o.height, o.k, o.precision, o.t_ref = (self.width, self.height, self.k,
                                                         self.precision, self.t_ref)
        o.planes = self.planes.clone()
        o.count = self.count.clone()
        o.src = None if self.src is None else self.src.clone()
        return o

    def _c(self, colours: Optional[torch.Tensor] = None) -> _DeepBuffer:
        p = self.planes
        src = None if self.src is None else _ptr(self.src).value
        if self.precision == "fp16":
            if colours is not None:
                raise AfrError("replacement colours need an FP32 buffer (FP16 slots are records)")
            b = p.data_ptr()  # record fields 2 bytes apart: ox, oy, r, g, b, tage
            return _DeepBuffer(self.width, self.height, self.k, PRECISIONS[self.precision],
                               self.t_ref, b, b + 2, b + 10, b + 4, b + 6, b + 8,
                               _ptr(self.count).value, src)
        c = p[3:6] if colours is None else colours
        if colours is not None and (colours.dtype != p.dtype or tuple(colours.shape) != tuple(p[3:6].shape)):
            raise AfrError("replacement colours must match the buffer's colour planes")
        if colours is not None and not colours.is_contiguous():
            raise AfrError("replacement colours must be contiguous")
        base = c.data_ptr()
        step = c[0].numel() * c.element_size()
        return _DeepBuffer(self.width, self.height, self.k, PRECISIONS[self.precision],
                           self.t_ref, p[0].data_ptr(), p[1].data_ptr(), p[2].data_ptr(),
                           base, base + step, base + 2 * step, _ptr(self.count).value, src)


def _stats_c(stats: torch.Tensor, tile: int) -> _TileStats:
    if stats.dtype != torch.float32 or stats.dim() != 3 or stats.shape[0] != NSTAT:
        raise AfrError(f"tile statistics must be float32 [{NSTAT}, Ty, Tx]")
    return _TileStats(int(tile), int(stats.shape[2]), int(stats.shape[1]), _ptr(stats).value)


_ws_cache = {}
_WS_CACHE_MAX = 64  # entries (kind x device x stream); the oldest go first beyond this


def _workspace(nbytes: int, device, key: str, stream=None) -> torch.Tensor:
    """Scratch memory for one kind of call, kept per device and per stream: calls on different
    streams may run at the same time and must not share a workspace. It is allocated on the stream
    that uses it, so the allocator never hands it to other work while that stream still runs."""
    s = torch.cuda.current_stream(device) if stream is None else stream
    k = (key, str(device), s.cuda_stream)
    t = _ws_cache.pop(k, None)
    if t is None or t.numel() < nbytes:
        with torch.cuda.stream(s):
            t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    _ws_cache[k] = t  # most recently used last
    while len(_ws_cache) > _WS_CACHE_MAX:
        # a dropped workspace returns to its own stream's pool, so work queued on that stream
        # still finishes before the memory is handed out again
        _ws_cache.pop(next(iter(_ws_cache)))
    return t


# ---- entry points --------------------------------------------------------------------------------

def build_deep_buffer(x, y, t, r, g, b, width: int, height: int, k: int, precision: str = "fp32",
                      t_ref: Optional[float] = None, out: Optional[DeepBuffer] = None,
                      stream=None, dropped: Optional[torch.Tensor] = None, stage_events=None,
                      vx=None, vy=None):
    """Build the per-pixel deep buffer from a device sample stream (float32 SoA).

    ``vx``, ``vy``: optional per-sample image-space velocities (px/ms); when given, every sample is
    reprojected to ``t_ref`` before binning (see afr_samples in afr.h).
    ``stage_events``: optional list of ``build_stage_count()`` timing-enabled ``torch.cuda.Event``
    objects, recorded on the stream after the count, scan, scatter and select stages.
    Returns ``(buffer, dropped)`` where ``dropped`` is a device int64 tensor of one element."""
    lib = library()
    if (vx is None) != (vy is None):
        raise AfrError("vx and vy go together")
    xs = [x, y, t, r, g, b]
    vel = [] if vx is None else [vx, vy]
    n = int(x.shape[0])
    for a in xs + vel:
        if a.dtype != torch.float32 or not a.is_cuda or a.dim() != 1 or not a.is_contiguous():
            raise AfrError("sample arrays must be contiguous 1-D float32 device tensors")
        if int(a.shape[0]) != n or a.device != x.device:
            raise AfrError("sample arrays must have one length and one device")
    if t_ref is None:
        raise AfrError("t_ref is required (every sample with t > t_ref is dropped)")
    dev = x.device
    if out is None:
        out = DeepBuffer(width, height, k, precision, t_ref, device=dev)
    else:
        out.t_ref = float(t_ref)
    if dropped is None:
        dropped = torch.zeros(1, dtype=torch.int64, device=dev)
    s = _Samples(*(a.data_ptr() if n else None for a in xs), n,
                 *((a.data_ptr() if n else None) for a in vel))
    wsb = lib.afr_build_workspace_bytes(n, width, height, k)
    ws = _workspace(wsb, dev, "build", stream)
    bc = out._c()
    if stage_events is None:
        _check(lib.afr_build_deep_buffer(ctypes.byref(s), ctypes.byref(bc), _ptr(ws), wsb,
                                         _ptr(dropped), _stream(stream)), "afr_build_deep_buffer")
        return out, dropped
    ns = lib.afr_build_stage_count()
    if len(stage_events) != ns:
        raise AfrError(f"stage_events needs {ns} events")
    handles = []
    for ev in stage_events:
        if not ev.cuda_event:  # torch creates the event at its first record
            ev.record()
        handles.append(ev.cuda_event)
    arr = (ctypes.c_void_p * ns)(*handles)
    _check(lib.afr_build_deep_buffer_staged(ctypes.byref(s), ctypes.byref(bc), _ptr(ws), wsb,
                                            _ptr(dropped), _stream(stream), arr),
           "afr_build_deep_buffer_staged")
    return out, dropped


def build_stage_count() -> int:
    return int(library().afr_build_stage_count())


def estimate_gradients(buf: DeepBuffer, params: Params, out: Optional[torch.Tensor] = None,
                       stream=None, colours=None) -> torch.Tensor:
    """Per-tile statistics ``[NSTAT, Ty, Tx]`` float32 (planes in ``STAT_NAMES`` order)."""
    lib = library()
    ty, tx = tiles_shape(buf.width, buf.height, params.tile)
    if out is None:
        out = torch.empty((NSTAT, ty, tx), dtype=torch.float32, device=buf.planes.device)
    bc, pc, sc = buf._c(colours), params._c(), _stats_c(out, params.tile)
    _check(lib.afr_estimate_gradients(ctypes.byref(bc), ctypes.byref(pc), ctypes.byref(sc),
                                      _stream(stream)), "afr_estimate_gradients")
    return out


def rms_loss(img: torch.Tensor, ref: torch.Tensor, scale: float = 1.0, want_grad: bool = True,
             loss: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None,
             stream=None):
    """``(loss, grad)``: ``scale * RMS(img - ref)`` as a float64 device scalar tensor and its
    gradient with respect to ``img`` (or None), see afr_rms_loss."""
    lib = library()
    if (img.dtype != torch.float32 or ref.dtype != torch.float32 or not img.is_contiguous()
            or not ref.is_contiguous() or img.shape != ref.shape or img.device != ref.device):
        raise AfrError("img and ref must be contiguous float32 device tensors of one shape")
    dev = img.device
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=dev)
    if grad is None and want_grad:
        grad = torch.empty_like(img)
    wsb = lib.afr_rms_workspace_bytes()
    ws = _workspace(wsb, dev, "rms", stream)
    n = img.numel()
    _check(lib.afr_rms_loss(_ptr(img) if n else None, _ptr(ref) if n else None, n, float(scale),
                            _ptr(loss), _ptr(grad) if (grad is not None and n) else None, _ptr(ws),
                            wsb, _stream(stream)), "afr_rms_loss")
    return loss, grad


def sampler_stats(buf: DeepBuffer, stats: torch.Tensor, params: Params, sp: SamplerParams,
                  stream=None):
    """Sampler feedback from the sampler's buffer and its statistics: ``(E [Ty,Tx], u [Ty,Tx],
    globals float64 [8])`` (globals in ``SAMPLER_GLOBALS`` order)."""
    lib = library()
    dev = buf.planes.device
    ty, tx = tiles_shape(buf.width, buf.height, params.tile)
    E = torch.empty((ty, tx), dtype=torch.float32, device=dev)
    u = torch.empty((ty, tx), dtype=torch.float32, device=dev)
    g = torch.empty(8, dtype=torch.float64, device=dev)
    wsb = lib.afr_sampler_workspace_bytes(ty * tx)
    ws = _workspace(wsb, dev, "sampler", stream)
    bc, sc, pc = buf._c(), _stats_c(stats, params.tile), params._c()
    _check(lib.afr_sampler_stats(ctypes.byref(bc), ctypes.byref(sc), ctypes.byref(pc),
                                 ctypes.byref(sp._c()), _ptr(E), _ptr(u), _ptr(g), _ptr(ws), wsb,
                                 _stream(stream)), "afr_sampler_stats")
    return E, u, g


def sampler_tile_weights(width: int, height: int, tile: int, E: torch.Tensor,
                         globals_: Optional[torch.Tensor] = None, n_parts: int = 0,
                         out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Equal-error tile weights [Ty, Tx] (see afr_sampler_tile_weights): ``n_parts`` parts, or the
    gain-control target count in ``globals_`` (from ``sampler_stats``) when ``n_parts`` is 0."""
    lib = library()
    ty, tx = tiles_shape(width, height, tile)
    if E.dtype != torch.float32 or not E.is_contiguous() or tuple(E.shape) != (ty, tx):
        raise AfrError("E must be a contiguous float32 [tiles_y, tiles_x] tensor")
    if globals_ is not None and (globals_.dtype != torch.float64 or globals_.numel() != 8):
        raise AfrError("globals_ must be the float64 [8] tensor of sampler_stats")
    if out is None:
        out = torch.empty_like(E)
    wsb = lib.afr_sampler_workspace_bytes(ty * tx)
    ws = _workspace(wsb, E.device, "sampler", stream)
    _check(lib.afr_sampler_tile_weights(width, height, tile, _ptr(E), _ptr(globals_), int(n_parts),
                                        _ptr(out), _ptr(ws), wsb, _stream(stream)),
           "afr_sampler_tile_weights")
    return out


def sampler_select(width: int, height: int, tile: int, E: torch.Tensor, rnd: torch.Tensor,
                   want_tile: bool = True, stream=None):
    """Spots ``(x, y, tile or None)`` for ``n = rnd.numel() // 3`` new samples, tiles drawn in
    proportion to ``E`` [Ty, Tx] (see afr_sampler_select)."""
    lib = library()
    dev = E.device
    ty, tx = tiles_shape(width, height, tile)
    if E.dtype != torch.float32 or not E.is_contiguous() or tuple(E.shape) != (ty, tx):
        raise AfrError("E must be a contiguous float32 [tiles_y, tiles_x] tensor")
    if rnd.dtype != torch.int32 or not rnd.is_contiguous() or rnd.dim() != 1 or rnd.numel() % 3:
        raise AfrError("rnd must be a contiguous 1-D int32 tensor (uint32 bits) of length 3 n")
    n = rnd.numel() // 3
    x = torch.empty(n, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    t = torch.empty(n, dtype=torch.int32, device=dev) if want_tile else None
    wsb = lib.afr_sampler_workspace_bytes(ty * tx)
    ws = _workspace(wsb, dev, "sampler", stream)
    _check(lib.afr_sampler_select(width, height, tile, _ptr(E), n, _ptr(rnd) if n else None,
                                  _ptr(x) if n else None, _ptr(y) if n else None,
                                  _ptr(t) if (t is not None and n) else None, _ptr(ws), wsb,
                                  _stream(stream)), "afr_sampler_select")
    return x, y, t


def sampler_select_noalloc(width: int, height: int, tile: int, E: torch.Tensor, rnd: torch.Tensor,
                           x: torch.Tensor, y: torch.Tensor, tile_out: Optional[torch.Tensor] = None,
                           stream=None):
    """``sampler_select`` into caller-provided ``x``, ``y`` (float32 [n]) and ``tile_out`` (int32 [n]
    or None) through afr_sampler_select_noalloc: no workspace, nothing allocated by the call."""
    lib = library()
    ty, tx = tiles_shape(width, height, tile)
    if E.dtype != torch.float32 or not E.is_contiguous() or tuple(E.shape) != (ty, tx):
        raise AfrError("E must be a contiguous float32 [tiles_y, tiles_x] tensor")
    if rnd.dtype != torch.int32 or not rnd.is_contiguous() or rnd.dim() != 1 or rnd.numel() % 3:
        raise AfrError("rnd must be a contiguous 1-D int32 tensor (uint32 bits) of length 3 n")
    n = rnd.numel() // 3
    for name, t, dt in (("x", x, torch.float32), ("y", y, torch.float32),
                        ("tile_out", tile_out, torch.int32)):
        if t is not None and (t.dtype != dt or not t.is_contiguous() or t.numel() < n):
            raise AfrError(f"{name} must be a contiguous {dt} tensor of at least {n} elements")
    _check(lib.afr_sampler_select_noalloc(width, height, tile, _ptr(E), n, _ptr(rnd) if n else None,
                                          _ptr(x) if n else None, _ptr(y) if n else None,
                                          _ptr(tile_out) if (tile_out is not None and n) else None,
                                          _stream(stream)), "afr_sampler_select_noalloc")
    return x, y, tile_out


def splat_sizes(width: int, height: int, coverage: Optional[torch.Tensor], sp: SplatParams,
                out: Optional[torch.Tensor] = None, device=None, stream=None) -> torch.Tensor:
    """Per-pixel splat size [H, W] for the next image from this image's coverage map [2, H, W]
    (``None``: the first image)."""
    lib = library()
    dev = coverage.device if coverage is not None else (out.device if out is not None else device)
    if dev is None:
        raise AfrError("splat_sizes needs a device when there is no coverage map or output")
    if coverage is not None and (coverage.dtype != torch.float32 or not coverage.is_contiguous()
                                 or tuple(coverage.shape) != (2, height, width)):
        raise AfrError("coverage must be a contiguous float32 [2, H, W] tensor")
    if out is None:
        out = torch.empty((height, width), dtype=torch.float32, device=dev)
    _check(lib.afr_splat_sizes(width, height, _ptr(coverage), ctypes.byref(sp._c()), _ptr(out),
                               _stream(stream)), "afr_splat_sizes")
    return out


def reconstruct_scatter(buf: DeepBuffer, stats: torch.Tensor, params: Params, size: torch.Tensor,
                        max_size: float, rgb: Optional[torch.Tensor] = None, want_aux: bool = True,
                        coverage: Optional[torch.Tensor] = None, want_coverage: bool = True,
                        stream=None):
    """Scatter-form image ``(rgb [3,H,W], aux [2,H,W] or None, coverage [2,H,W] or None)`` with the
    per-source-pixel splat sizes ``size`` [H, W]."""
    lib = library()
    dev = buf.planes.device
    H, W = buf.height, buf.width
    if size.dtype != torch.float32 or not size.is_contiguous() or tuple(size.shape) != (H, W):
        raise AfrError("size must be a contiguous float32 [H, W] tensor")
    if rgb is None:
        rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    aux = torch.empty((2, H, W), dtype=torch.float32, device=dev) if want_aux else None
    if coverage is None and want_coverage:
        coverage = torch.empty((2, H, W), dtype=torch.float32, device=dev)
    bc, pc, sc = buf._c(), params._c(), _stats_c(stats, params.tile)
    _check(lib.afr_reconstruct_scatter(ctypes.byref(bc), ctypes.byref(sc), ctypes.byref(pc),
                                       _ptr(size), float(max_size), _ptr(rgb), _ptr(aux),
                                       _ptr(coverage), _stream(stream)), "afr_reconstruct_scatter")
    return rgb, aux, coverage


def build_crosshair_buffer(samples, crosshairs, width: int, height: int, k: int, params: Params,
                           t_ref: float, out: Optional[DeepBuffer] = None, stream=None,
                           dropped: Optional[torch.Tensor] = None):
    """The sampler's per-pixel crosshair queues (FP32; gradients gx, gy, gt in the r, g, b planes).

    ``samples``: the six float32 device arrays (x, y, t, r, g, b) of the stream; ``crosshairs``:
    six int32 device arrays (centre, xm, xp, ym, yp, old) of stream indices, -1 where absent.
    Returns ``(buffer, dropped)``."""
    lib = library()
    xs = list(samples)
    ids = list(crosshairs)
    if len(xs) != 6 or len(ids) != 6:
        raise AfrError("samples are (x, y, t, r, g, b) and crosshairs (centre, xm, xp, ym, yp, old)")
    n = int(xs[0].shape[0])
    nx = int(ids[0].shape[0])
    dev = xs[0].device
    for a in xs:
        if (a.dtype != torch.float32 or not a.is_cuda or a.dim() != 1 or not a.is_contiguous()
                or int(a.shape[0]) != n or a.device != dev):
            raise AfrError("sample arrays must be contiguous 1-D float32 device tensors of one length")
    for a in ids:
        if (a.dtype != torch.int32 or not a.is_cuda or a.dim() != 1 or not a.is_contiguous()
                or int(a.shape[0]) != nx or a.device != dev):
            raise AfrError("crosshair arrays must be contiguous 1-D int32 device tensors of one length")
    if out is None:
        out = DeepBuffer(width, height, k, "fp32", t_ref, device=dev)
    else:
        out.t_ref = float(t_ref)
    if dropped is None:
        dropped = torch.zeros(1, dtype=torch.int64, device=dev)
    sc = _Samples(*(a.data_ptr() if n else None for a in xs), n)
    xc = _Crosshairs(*(a.data_ptr() if nx else None for a in ids), nx)
    wsb = lib.afr_crosshair_workspace_bytes(nx, width, height)
    ws = _workspace(wsb, dev, "crosshair", stream)
    bc, pc = out._c(), params._c()
    _check(lib.afr_build_crosshair_buffer(ctypes.byref(sc), ctypes.byref(xc), ctypes.byref(pc),
                                          ctypes.byref(bc), _ptr(ws), wsb, _ptr(dropped),
                                          _stream(stream)), "afr_build_crosshair_buffer")
    return out, dropped


def estimate_gradients_crosshair(buf: DeepBuffer, xbuf: DeepBuffer, params: Params,
                                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Tile statistics of ``buf`` with the gradient planes (and the extents) taken from the
    crosshair queues ``xbuf``."""
    lib = library()
    ty, tx = tiles_shape(buf.width, buf.height, params.tile)
    if out is None:
        out = torch.empty((NSTAT, ty, tx), dtype=torch.float32, device=buf.planes.device)
    bc, xc, pc, sc = buf._c(), xbuf._c(), params._c(), _stats_c(out, params.tile)
    _check(lib.afr_estimate_gradients_crosshair(ctypes.byref(bc), ctypes.byref(xc),
                                                ctypes.byref(pc), ctypes.byref(sc),
                                                _stream(stream)),
           "afr_estimate_gradients_crosshair")
    return out


def _reconstruct(name, buf, stats, params, rgb, aux, want_aux, stream, colours=None):
    lib = library()
    dev = buf.planes.device
    if rgb is None:
        rgb = torch.empty((3, buf.height, buf.width), dtype=torch.float32, device=dev)
    if aux is None and want_aux:
        aux = torch.empty((2, buf.height, buf.width), dtype=torch.float32, device=dev)
    bc, pc, sc = buf._c(colours), params._c(), _stats_c(stats, params.tile)
    _check(getattr(lib, name)(ctypes.byref(bc), ctypes.byref(sc), ctypes.byref(pc), _ptr(rgb),
                              _ptr(aux), _stream(stream)), name)
    return rgb, aux


def reconstruct(buf: DeepBuffer, stats: torch.Tensor, params: Params, rgb=None, aux=None,
                want_aux: bool = True, stream=None, colours=None):
    """LDS-tiled gather. Returns ``(rgb [3,H,W], aux [2,H,W] or None)``."""
    return _reconstruct("afr_reconstruct", buf, stats, params, rgb, aux, want_aux, stream, colours)


def forward(buf: DeepBuffer, params: Params, stats: Optional[torch.Tensor] = None, rgb=None,
            aux=None, want_aux: bool = True, stream=None):
    """Statistics and gather in one launch (afr_forward): ``(stats, rgb, aux or None)``, equal bit
    for bit to ``estimate_gradients`` followed by ``reconstruct``."""
    lib = library()
    dev = buf.planes.device
    ty, tx = tiles_shape(buf.width, buf.height, params.tile)
    if stats is None:
        stats = torch.empty((NSTAT, ty, tx), dtype=torch.float32, device=dev)
    if rgb is None:
        rgb = torch.empty((3, buf.height, buf.width), dtype=torch.float32, device=dev)
    if aux is None and want_aux:
        aux = torch.empty((2, buf.height, buf.width), dtype=torch.float32, device=dev)
    bc, pc, sc = buf._c(), params._c(), _stats_c(stats, params.tile)
    _check(lib.afr_forward(ctypes.byref(bc), ctypes.byref(pc), ctypes.byref(sc), _ptr(rgb),
                           _ptr(aux), _stream(stream)), "afr_forward")
    return stats, rgb, aux


def reconstruct_launch(buf: DeepBuffer, stats: torch.Tensor, params: Params, tiles_per_wave: int,
                       rgb=None, aux=None, want_aux: bool = True, stream=None, colours=None):
    """LDS-tiled gather with an explicit launch shape (bit-identical output for every shape)."""
    lib = library()
    dev = buf.planes.device
    if rgb is None:
        rgb = torch.empty((3, buf.height, buf.width), dtype=torch.float32, device=dev)
    if aux is None and want_aux:
        aux = torch.empty((2, buf.height, buf.width), dtype=torch.float32, device=dev)
    bc, pc, sc = buf._c(colours), params._c(), _stats_c(stats, params.tile)
    _check(lib.afr_reconstruct_launch(ctypes.byref(bc), ctypes.byref(sc), ctypes.byref(pc),
                                      int(tiles_per_wave), _ptr(rgb), _ptr(aux), _stream(stream)),
           "afr_reconstruct_launch")
    return rgb, aux


def reconstruct_tune(buf: DeepBuffer, stats: torch.Tensor, params: Params, stream=None):
    """Time every launch shape of the tiled gather on these inputs (blocking), record the fastest
    for this buffer class, and return ``(tiles_per_wave, ms)``."""
    lib = library()
    rgb = torch.empty((3, buf.height, buf.width), dtype=torch.float32, device=buf.planes.device)
    best, ms = ctypes.c_int32(0), ctypes.c_float(0.0)
    bc, pc, sc = buf._c(), params._c(), _stats_c(stats, params.tile)
    _check(lib.afr_reconstruct_tune(ctypes.byref(bc), ctypes.byref(sc), ctypes.byref(pc), _ptr(rgb),
                                    ctypes.byref(best), ctypes.byref(ms), _stream(stream)),
           "afr_reconstruct_tune")
    return int(best.value), float(ms.value)


class Batch:
    """Many independent estimate + gather pipelines in one persistent launch (``afr_batch_*``).

    ``items`` is a list of ``(DeepBuffer, Params)``; every item must use 8 px tiles, one radius and
    one storage precision. Outputs (``rgb``, ``aux``, ``stats`` per item) are allocated here. ``run``
    enqueues the whole batch on the current stream and can be captured in a CUDA/HIP graph."""

    def __init__(self, items, tiles_per_wave: int = 0, want_aux: bool = True):
        lib = library()
        if not items:
            raise AfrError("empty batch")
        self.items = list(items)
        self.rgb, self.aux, self.stats = [], [], []
        arr = (_BatchItem * len(items))()
        for i, (buf, p) in enumerate(self.items):
            dev = buf.planes.device
            ty, tx = tiles_shape(buf.width, buf.height, p.tile)
            st = torch.empty((NSTAT, ty, tx), dtype=torch.float32, device=dev)
            rgb = torch.empty((3, buf.height, buf.width), dtype=torch.float32, device=dev)
            aux = (torch.empty((2, buf.height, buf.width), dtype=torch.float32, device=dev)
                   if want_aux else None)
            self.stats.append(st)
            self.rgb.append(rgb)
            self.aux.append(aux)
            arr[i] = _BatchItem(buf._c(), _stats_c(st, p.tile), p._c(), _ptr(rgb).value,
                                None if aux is None else _ptr(aux).value)
        n = len(items)
        nbytes = lib.afr_batch_workspace_bytes(n)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.items[0][0].planes.device)
        plan = ctypes.c_void_p()
        _check(lib.afr_batch_create(arr, n, int(tiles_per_wave), _ptr(self.ws), nbytes,
                                    ctypes.byref(plan)), "afr_batch_create")
        self._plan = plan
        self._arr = arr

    def run(self, stream=None):
        _check(library().afr_batch_run(self._plan, _stream(stream)), "afr_batch_run")

    def reconstruct(self, tiles_per_wave: int = 0, stream=None):
        """The same batch through the plan-free call (afr_batch_reconstruct): the item table is
        written into a workspace of its own by the call's kernels, so this can be captured."""
        lib = library()
        n = len(self.items)
        nbytes = lib.afr_batch_workspace_bytes(n)
        if getattr(self, "_ws1", None) is None:
            self._ws1 = torch.empty(nbytes, dtype=torch.uint8, device=self.ws.device)
        t = _Tune(int(tiles_per_wave), _ptr(self._ws1).value, nbytes)
        _check(lib.afr_batch_reconstruct(self._arr, n, ctypes.byref(t), _stream(stream)),
               "afr_batch_reconstruct")

    def tune(self, stream=None):
        best, ms = ctypes.c_int32(0), ctypes.c_float(0.0)
        _check(library().afr_batch_tune(self._plan, _stream(stream), ctypes.byref(best),
                                        ctypes.byref(ms)), "afr_batch_tune")
        return int(best.value), float(ms.value)

    @property
    def tiles_per_wave(self) -> int:
        return int(library().afr_batch_tiles_per_wave(self._plan))

    def close(self):
        if getattr(self, "_plan", None):
            library().afr_batch_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct_plain(buf: DeepBuffer, stats: torch.Tensor, params: Params, rgb=None, aux=None,
                      want_aux: bool = True, stream=None, colours=None):
    """Direct gather (one thread per pixel, one exponential per pair)."""
    return _reconstruct("afr_reconstruct_plain", buf, stats, params, rgb, aux, want_aux, stream,
                        colours)


def reconstruct_backward(buf: DeepBuffer, stats: torch.Tensor, params: Params, rgb, aux, grad_rgb,
                         grad_slot=None, grad_params=None, stream=None, colours=None):
    """Adjoint of the gather: ``(grad_slot [3,K,H,W] float32, grad_params [2] = (d sigma, d tau))``."""
    lib = library()
    dev = buf.planes.device
    if grad_slot is None:
        grad_slot = torch.empty((3, buf.k, buf.height, buf.width), dtype=torch.float32, device=dev)
    if grad_params is None:
        grad_params = torch.empty(2, dtype=torch.float32, device=dev)
    wsb = lib.afr_backward_workspace_bytes(buf.width, buf.height, buf.k, params.radius)
    ws = _workspace(wsb, dev, "backward", stream)
    bc, pc, sc = buf._c(colours), params._c(), _stats_c(stats, params.tile)
    grad_rgb = grad_rgb.contiguous().float()
    _check(lib.afr_reconstruct_backward(ctypes.byref(bc), ctypes.byref(sc), ctypes.byref(pc),
                                        _ptr(rgb), _ptr(aux), _ptr(grad_rgb), _ptr(grad_slot),
                                        _ptr(grad_params), _ptr(ws), wsb, _stream(stream)),
           "afr_reconstruct_backward")
    return grad_slot, grad_params


class ReconstructFn(torch.autograd.Function):
    """Differentiable gather.

    Inputs: slot colours ``[3, K, H, W]`` (a replacement for the colours of an FP32 buffer, or, with
    ``own`` set, the buffer's own colours, which are then read from the buffer), ``sigma`` and
    ``tau`` (0-d float tensors). The tile statistics are estimated from the buffer's stored samples
    at the given sigma and tau and are constants of the gather (stop-gradient), as in
    ``afr_reconstruct_backward``: the forward is exactly the gather the adjoint differentiates, and
    gradients flow to the colours and to sigma and tau.
    """

    @staticmethod
    def forward(ctx, colours, sigma, tau, buf: DeepBuffer, params: Params, form: str = "tiled",
                own: bool = False):
        p = params.with_(sigma=float(sigma), tau=float(tau))
        ctx.colour_dtype = colours.dtype
        colours = None if own else colours.detach().contiguous()
        stats = estimate_gradients(buf, p)
        fn = reconstruct if form == "tiled" else reconstruct_plain
        rgb, aux = fn(buf, stats, p, colours=colours)
        ctx.save_for_backward(rgb, aux, stats, *(() if colours is None else (colours,)))
        ctx.buf, ctx.params, ctx.own = buf, p, own
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        rgb, aux, stats = ctx.saved_tensors[:3]
        colours = None if ctx.own else ctx.saved_tensors[3]
        gslot, gpar = reconstruct_backward(ctx.buf, stats, ctx.params, rgb, aux, grad_rgb,
                                           colours=colours)
        gc = gslot.to(ctx.colour_dtype) if ctx.needs_input_grad[0] else None
        gs = gpar[0] if ctx.needs_input_grad[1] else None
        gt = gpar[1] if ctx.needs_input_grad[2] else None
        return gc, gs, gt, None, None, None, None


def reconstruct_differentiable(buf: DeepBuffer, params: Params, sigma, tau, colours=None,
                               form: str = "tiled"):
    """``rgb = ReconstructFn(colours, sigma, tau)``; colours default to the buffer's own."""
    if colours is None:
        return ReconstructFn.apply(buf.colours(), sigma, tau, buf, params, form, True)
    return ReconstructFn.apply(colours, sigma, tau, buf, params, form, False)
