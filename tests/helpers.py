"""Shared helpers for the GPU parity tests: run the same seeded workload through the HIP library (via
its C ABI binding) and through the FP64 reference, and compare."""
from __future__ import annotations

import functools

import numpy as np

import afr_scenes as S
import oracle as O

DEV = "cuda"


def torch_mod():
    import torch
    return torch


def afr_mod():
    import paper_2510_15876_amd as afr
    return afr


@functools.lru_cache(maxsize=None)
def workload(name: str):
    return S.make_workload(name)


def dev_stream(stream):
    torch = torch_mod()
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in stream.arrays()]


def gpu_build(stream, w, h, k, precision, t_ref, reproject=False):
    afr = afr_mod()
    vel = {}
    if reproject:
        torch = torch_mod()
        vx, vy = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in stream.motion())
        vel = dict(vx=vx, vy=vy)
    buf, dropped = afr.build_deep_buffer(*dev_stream(stream), w, h, k, precision, t_ref, **vel)
    return buf, int(dropped.item())


@functools.lru_cache(maxsize=None)
def oracle_build_cached(name: str, precision: str, k: int):
    wl = workload(name)
    return O.build_buffer(wl.stream, wl.width, wl.height, k, precision, wl.t_ref)


def params(t_now, **kw):
    afr = afr_mod()
    return afr.Params(t_now=float(t_now), **kw), O.Params(t_now=float(np.float32(t_now)), **kw)


def buffer_np(buf):
    """GPU deep buffer as float64 numpy planes (dict), plus count and src."""
    d = {f: np.ascontiguousarray(buf.field(f).float().cpu().numpy().astype(np.float64)
                                 .transpose(1, 2, 0)) for f in buf.FIELDS}
    d["count"] = buf.count.cpu().numpy()
    d["src"] = None if buf.src is None else buf.src.cpu().numpy().transpose(1, 2, 0)
    return d


def slots_to_reference_layout(a):
    """GPU slot-major [..., K, H, W] -> reference [..., H, W, K]."""
    a = np.asarray(a)
    return np.ascontiguousarray(np.moveaxis(a, -3, -1))


def assert_buffers_equal(gbuf, obuf):
    g = buffer_np(gbuf)
    np.testing.assert_array_equal(g["count"], obuf.count)
    if g["src"] is not None:
        np.testing.assert_array_equal(g["src"], obuf.src)
    for f, of in (("ox", "ox"), ("oy", "oy"), ("tage", "ta"), ("r", "r"), ("g", "g"), ("b", "b")):
        np.testing.assert_array_equal(g[f], getattr(obuf, of), err_msg=f"plane {f}")


def stats_to_gpu(ost):
    """Reference statistics rounded to float32 on the device (reference output -> GPU input)."""
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(ost, np.float32)).to(DEV)


def stats_f32_as_f64(ost):
    return np.ascontiguousarray(ost, np.float32).astype(np.float64)


def reconstruct(form, buf, stats, p, **kw):
    afr = afr_mod()
    fn = afr.reconstruct if form == "tiled" else afr.reconstruct_plain
    return fn(buf, stats, p, **kw)


def log_weight_sum(aux):
    """log(sum_s exp(E_s)) from an aux pair (shift m, W_m = sum exp(E_s - m)); -inf where empty."""
    m, w = aux[0], aux[1]
    with np.errstate(divide="ignore"):
        return np.where(w > 0, m + np.log(np.where(w > 0, w, 1.0)), -np.inf)
