"""Seeded synthetic scenes and space-time sample streams.

The paper evaluates on animated ray-traced scenes from the BART testbed (Sec. 7); none of them is
available here, so seeded analytic 2-D scenes stand in for them. A "sample" is what the paper's
sampler streams to its reconstructor (Sec. 4.2, Sec. 5.2): a colour taken at one sub-pixel image
position at one instant. Every workload below draws such samples from an analytic scene.

This module only draws random numbers and evaluates scene colour at given space-time points. It holds
none of the reconstruction arithmetic: the FP64 reference in ``oracle/`` and the GPU library both
consume the arrays it returns, and neither is imported here.

Units: positions in pixels (pixel ``(i, j)`` covers ``[i, i+1) x [j, j+1)``), time in milliseconds.
Streams are float32 structure-of-arrays, ordered by ascending time unless ``sort=False``.
Seeds follow ``1000 * config + instance`` with NumPy's PCG64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Stream", "Workload", "CheckerDiscScene", "DiscScene", "stratified_stream", "uniform_stream",
    "ground_truth", "make_workload", "make_c4_sequence", "make_c5_batch", "CONFIG_NAMES",
    "Crosshairs", "crosshair_stream", "make_crosshair_workload", "shade_samples",
]

OMEGA_RAD_PER_MS = 1e-3   # background ramp rotation, 1 rad/s
FRAME_MS = 1000.0 / 60.0  # 60 Hz display refresh


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Stream:
    """A stream of space-time samples: float32 SoA arrays of equal length. ``vx``, ``vy`` (px/ms,
    optional) are the image-space velocities of the surfaces the samples hit, for reprojection."""
    x: np.ndarray
    y: np.ndarray
    t: np.ndarray
    r: np.ndarray
    g: np.ndarray
    b: np.ndarray
    vx: Optional[np.ndarray] = None
    vy: Optional[np.ndarray] = None

    def __len__(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return (self.x, self.y, self.t, self.r, self.g, self.b)

    def motion(self):
        """(vx, vy), or None when the stream carries no velocities."""
        return None if self.vx is None else (self.vx, self.vy)

    def select(self, mask_or_index) -> "Stream":
        m = self.motion()
        extra = () if m is None else tuple(a[mask_or_index] for a in m)
        return Stream(*(a[mask_or_index] for a in self.arrays()), *extra)

    def copy(self) -> "Stream":
        m = self.motion()
        extra = () if m is None else tuple(a.copy() for a in m)
        return Stream(*(a.copy() for a in self.arrays()), *extra)


# --------------------------------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------------------------------

class CheckerDiscScene:
    """Static 8-px black/white checkerboard with one red disc of radius 10 moving +x at 0.2 px/ms.

    White where ``floor(x/8) + floor(y/8)`` is even. The disc centre is ``(22 + 0.2 t, 32)``.
    """

    def __init__(self, cell: float = 8.0, radius: float = 10.0, speed: float = 0.2,
                 x0: float = 22.0, y0: float = 32.0):
        self.cell, self.radius, self.speed, self.x0, self.y0 = cell, radius, speed, x0, y0

    def color(self, x, y, t):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        t = np.asarray(t, np.float64)
        white = ((np.floor(x / self.cell) + np.floor(y / self.cell)) % 2 == 0).astype(np.float64)
        r, g, b = white.copy(), white.copy(), white.copy()
        cx = self.x0 + self.speed * t
        inside = (x - cx) ** 2 + (y - self.y0) ** 2 <= self.radius ** 2
        r[inside], g[inside], b[inside] = 1.0, 0.0, 0.0
        return r, g, b

    def shade(self, x, y, t):
        """Colour and image-space velocity (px/ms) of the surface at (x, y, t)."""
        r, g, b = self.color(x, y, t)
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        cx = self.x0 + self.speed * np.asarray(t, np.float64)
        inside = (x - cx) ** 2 + (y - self.y0) ** 2 <= self.radius ** 2
        vx = np.where(inside, self.speed, 0.0)
        return r, g, b, vx, np.zeros_like(vx)


class DiscScene:
    """Moving discs over a rotating grey ramp; painter's order (later discs on top), no wrap.

    Disc ``d`` has radius ``U[r_lo, r_hi]``, colour ``U[0,1]^3``, centre uniform over the image at
    time ``t_centre`` and velocity ``U[-speed, speed]^2`` px/ms. The background is the grey level
    ``0.5 + 0.5 * ((x - W/2) cos wt + (y - H/2) sin wt) / (hypot(W, H) / 2)``, clipped to [0, 1].
    With ``highlights`` each disc also carries a Gaussian highlight (sigma 3 px, peak 1.0) centred at
    ``centre + (-r/3, -r/3)``, added to all three channels inside the disc and clipped at 1.
    With ``checker > 0`` the background is instead a static checkerboard of that cell size in px,
    rotated by ``checker_angle`` radians: with ``u = x cos a + y sin a``, ``v = y cos a - x sin a``,
    grey 0.8 where ``floor(u/c) + floor(v/c)`` is even and 0.2 elsewhere.
    """

    def __init__(self, width: int, height: int, rng: np.random.Generator, n_discs: int,
                 t_centre: float, highlights: bool = False, speed: float = 0.5,
                 radius: tuple = (4.0, 24.0), omega: float = OMEGA_RAD_PER_MS,
                 highlight_sigma: float = 3.0, highlight_peak: float = 1.0,
                 checker: float = 0.0, checker_angle: float = 0.0):
        self.checker = float(checker)
        self.checker_angle = float(checker_angle)
        self.width, self.height = int(width), int(height)
        self.t_centre = float(t_centre)
        self.omega = float(omega)
        self.highlights = bool(highlights)
        self.hl_sigma, self.hl_peak = float(highlight_sigma), float(highlight_peak)
        n = int(n_discs)
        self.radius = rng.uniform(radius[0], radius[1], n)
        self.rgb = rng.uniform(0.0, 1.0, (n, 3))
        self.cx = rng.uniform(0.0, width, n)
        self.cy = rng.uniform(0.0, height, n)
        self.vel = rng.uniform(-speed, speed, (n, 2))

    def background(self, x, y, t):
        if self.checker > 0.0:  # static checkerboard, grey levels 0.2 and 0.8
            c, ca, sa = self.checker, np.cos(self.checker_angle), np.sin(self.checker_angle)
            u, v = x * ca + y * sa, y * ca - x * sa
            even = (np.floor(u / c) + np.floor(v / c)) % 2 == 0
            return np.where(even, 0.8, 0.2) + 0.0 * t
        w, h = self.width, self.height
        half_diag = 0.5 * np.hypot(w, h)
        proj = (x - 0.5 * w) * np.cos(self.omega * t) + (y - 0.5 * h) * np.sin(self.omega * t)
        return np.clip(0.5 + 0.5 * proj / half_diag, 0.0, 1.0)

    def centre(self, d: int, t):
        dt = t - self.t_centre
        return self.cx[d] + self.vel[d, 0] * dt, self.cy[d] + self.vel[d, 1] * dt

    def color(self, x, y, t):
        return self.shade(x, y, t)[:3]

    def shade(self, x, y, t):
        """Colour and image-space velocity (px/ms) of the surface at (x, y, t): the top disc's
        velocity, 0 on the background (its shading changes, its points do not move)."""
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        t = np.asarray(t, np.float64)
        grey = self.background(x, y, t)
        r, g, b = grey.copy(), grey.copy(), grey.copy()
        vx, vy = np.zeros_like(grey), np.zeros_like(grey)
        if x.size == 0:
            return r, g, b, vx, vy
        t_lo, t_hi = float(t.min()), float(t.max())
        for d in range(self.radius.shape[0]):
            rad = self.radius[d]
            c0 = self.centre(d, t_lo)
            c1 = self.centre(d, t_hi)
            x_lo, x_hi = min(c0[0], c1[0]) - rad, max(c0[0], c1[0]) + rad
            y_lo, y_hi = min(c0[1], c1[1]) - rad, max(c0[1], c1[1]) + rad
            cand = np.nonzero((x >= x_lo) & (x <= x_hi) & (y >= y_lo) & (y <= y_hi))[0]
            if cand.size == 0:
                continue
            cx, cy = self.centre(d, t[cand])
            ddx, ddy = x[cand] - cx, y[cand] - cy
            inside = ddx * ddx + ddy * ddy <= rad * rad
            idx = cand[inside]
            if idx.size == 0:
                continue
            cr, cg, cb = self.rgb[d]
            vx[idx], vy[idx] = self.vel[d, 0], self.vel[d, 1]
            if self.highlights:
                hx = ddx[inside] + rad / 3.0
                hy = ddy[inside] + rad / 3.0
                hl = self.hl_peak * np.exp(-(hx * hx + hy * hy) / (2.0 * self.hl_sigma ** 2))
                r[idx] = np.minimum(1.0, cr + hl)
                g[idx] = np.minimum(1.0, cg + hl)
                b[idx] = np.minimum(1.0, cb + hl)
            else:
                r[idx], g[idx], b[idx] = cr, cg, cb
        return r, g, b, vx, vy


# --------------------------------------------------------------------------------------------------
# Streams and ground truth
# --------------------------------------------------------------------------------------------------

def _shade_to_stream(scene, x32, y32, t32, sort: bool) -> Stream:
    r, g, b, vx, vy = scene.shade(x32.astype(np.float64), y32.astype(np.float64),
                                  t32.astype(np.float64))
    f = lambda a: a.astype(np.float32)
    s = Stream(x32, y32, t32, f(r), f(g), f(b), f(vx), f(vy))
    if sort:
        order = np.argsort(t32, kind="stable")
        s = s.select(order)
    return s


def shade_samples(scene, x, y, t, sort: bool = True) -> Stream:
    """A stream of samples of ``scene`` taken at the given float32 spots and times."""
    return _shade_to_stream(scene, np.asarray(x, np.float32), np.asarray(y, np.float32),
                            np.asarray(t, np.float32), sort)


def stratified_stream(scene, width: int, height: int, m, t_now: float, t_win: float,
                      rng: np.random.Generator, sort: bool = True) -> Stream:
    """``m`` samples per pixel (an int, or an ``[H, W]`` int array), each at a uniform sub-pixel
    position ``(i + U, j + U)`` and time ``t_now - U[0, t_win)``.

    Draw order: x offsets, y offsets, then time offsets, each as an ``[H, W, max m]`` array.
    """
    m_arr = np.broadcast_to(np.asarray(m, np.int64), (height, width))
    m_max = int(m_arr.max()) if m_arr.size else 0
    shape = (height, width, m_max)
    ux = rng.random(shape)
    uy = rng.random(shape)
    ut = rng.random(shape)
    jj, ii = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                         indexing="ij")
    x = (ii[:, :, None] + ux).astype(np.float32)
    y = (jj[:, :, None] + uy).astype(np.float32)
    t = (t_now - t_win * ut).astype(np.float32)
    keep = np.arange(m_max)[None, None, :] < m_arr[:, :, None]
    return _shade_to_stream(scene, x[keep], y[keep], t[keep], sort)


def uniform_stream(scene, width: int, height: int, n: int, t_now: float, t_win: float,
                   rng: np.random.Generator, sort: bool = True) -> Stream:
    """``n`` samples at uniform positions over the whole image (not stratified: occupancy varies
    and pixels can be empty) and times ``t_now - U[0, t_win)``. Draw order: x, y, t."""
    x = (width * rng.random(n)).astype(np.float32)
    y = (height * rng.random(n)).astype(np.float32)
    t = (t_now - t_win * rng.random(n)).astype(np.float32)
    # float32 rounding can land exactly on the far image edge; such samples stay in the stream
    # (the build drops them as outside the image) so that the recipe is unchanged.
    return _shade_to_stream(scene, x, y, t, sort)


def ground_truth(scene, width: int, height: int, t: float, ss: int = 16) -> np.ndarray:
    """Antialiased zero-delay ideal image at time ``t``: the ``ss x ss`` box-supersampled pixel
    mean of the analytic scene, FP64, shape ``[3, H, W]`` (the gold standard of Sec. 7)."""
    off = (np.arange(ss, dtype=np.float64) + 0.5) / ss
    out = np.zeros((3, height, width), np.float64)
    rows_per_chunk = max(1, (1 << 22) // max(1, width * ss * ss))
    for j0 in range(0, height, rows_per_chunk):
        j1 = min(height, j0 + rows_per_chunk)
        jj = np.arange(j0, j1, dtype=np.float64)
        ii = np.arange(width, dtype=np.float64)
        px = ii[None, :, None, None] + off[None, None, None, :]
        py = jj[:, None, None, None] + off[None, None, :, None]
        px, py = np.broadcast_arrays(px, py)
        px = px.reshape(-1)
        py = py.reshape(-1)
        r, g, b = scene.color(px, py, np.full(px.shape, t))
        for c, v in enumerate((r, g, b)):
            out[c, j0:j1] = v.reshape(j1 - j0, width, ss * ss).mean(axis=2)
    return out


# --------------------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    stream: Stream
    width: int
    height: int
    k: int
    precision: str          # "fp32" or "fp16": storage precision of the deep buffer
    t_ref: float            # stream reference time: every sample has t <= t_ref
    t_now: float            # reconstruction time
    scene: object = field(repr=False, default=None)
    radius: int = 2
    tile: int = 8
    description: str = ""

    @property
    def pixels(self) -> int:
        return self.width * self.height


CONFIG_NAMES = ("c0", "c1", "c2", "c3", "c4", "c5")


def _c2_density(scene, width, height, k, t_now, t_win, tile=32, frac=0.25):
    """Per-pixel sample counts for C2: ``2K`` in the quarter of 32x32 tiles whose pixel-centre
    colour changes most over the window, ``K`` elsewhere."""
    jj, ii = np.meshgrid(np.arange(height) + 0.5, np.arange(width) + 0.5, indexing="ij")
    px, py = ii.reshape(-1), jj.reshape(-1)
    now = np.stack(scene.color(px, py, np.full(px.shape, t_now)))
    then = np.stack(scene.color(px, py, np.full(px.shape, t_now - t_win)))
    change = np.abs(now - then).mean(axis=0).reshape(height, width)
    ty, tx = -(-height // tile), -(-width // tile)
    score = np.zeros((ty, tx))
    for a in range(ty):
        for c in range(tx):
            score[a, c] = change[a * tile:(a + 1) * tile, c * tile:(c + 1) * tile].mean()
    n_top = (ty * tx) // int(round(1 / frac))
    order = np.argsort(-score.reshape(-1), kind="stable")[:n_top]
    m = np.full((height, width), k, np.int64)
    for flat in order:
        a, c = divmod(int(flat), tx)
        m[a * tile:(a + 1) * tile, c * tile:(c + 1) * tile] = 2 * k
    return m


def make_workload(name: str, instance: int = 0, sort: bool = True, **over) -> Workload:
    """Build one named synthetic workload.

    c0  256x256, 400K samples uniform over the image (unstratified; empty pixels possible), 1 s
        window, K=16, 16 discs at U[-0.05, 0.05] px/ms. Shaped like the paper's 256x256, N=400K
        reconstruction (Sec. 5.2).
    c1  64x64, K=4, 4 samples/px over 40 ms, checkerboard + moving red disc, FP32.
    c2  256x256, K=8, 16 discs over a rotating ramp, 64 ms window, density doubled in the quarter
        of 32x32 tiles with the most temporal change, FP32.
    c3  640x480, K=16, 64 discs with specular-like highlights, 64 ms window, FP16 storage.
    c4  512x512, K=8, 64 discs, FP32; the first frame of the sequence from ``make_c4_sequence``.
    """
    cfg = CONFIG_NAMES.index(name)
    rng = _rng(1000 * cfg + instance)
    if name == "c0":
        w, h, k, t_win, t_now = 256, 256, 16, 1000.0, 1000.0
        scene = DiscScene(w, h, rng, 16, t_now, speed=0.05)
        s = uniform_stream(scene, w, h, 400_000, t_now, t_win, rng, sort)
        wl = Workload(name, s, w, h, k, "fp32", t_now, t_now, scene,
                      description="256x256 N=400K uniform, K=16, 1 s window")
    elif name == "c1":
        w, h, k, t_win, t_now = 64, 64, 4, 40.0, 40.0
        scene = CheckerDiscScene()
        s = stratified_stream(scene, w, h, 4, t_now, t_win, rng, sort)
        wl = Workload(name, s, w, h, k, "fp32", t_now, t_now, scene,
                      description="64x64 K=4 checkerboard + moving disc, FP32")
    elif name == "c2":
        w, h, k, t_win, t_now = 256, 256, 8, 64.0, 64.0
        scene = DiscScene(w, h, rng, 16, t_now)
        m = _c2_density(scene, w, h, k, t_now, t_win)
        s = stratified_stream(scene, w, h, m, t_now, t_win, rng, sort)
        wl = Workload(name, s, w, h, k, "fp32", t_now, t_now, scene,
                      description="256x256 K=8 16 discs, density doubled in top-quarter tiles, FP32")
    elif name == "c3":
        w, h, k, t_win, t_now = 640, 480, 16, 64.0, 64.0
        scene = DiscScene(w, h, rng, 64, t_now, highlights=True)
        s = stratified_stream(scene, w, h, k, t_now, t_win, rng, sort)
        wl = Workload(name, s, w, h, k, "fp16", t_now, t_now, scene,
                      description="640x480 K=16 64 discs + highlights, FP16 storage")
    elif name == "c4":
        seq = make_c4_sequence(n_frames=1, instance=instance)
        return seq.frame_workload(0)
    else:
        raise ValueError(f"unknown workload {name!r}; c5 is a batch, see make_c5_batch")
    for key, val in over.items():
        setattr(wl, key, val)
    return wl


@dataclass
class C4Sequence:
    """512x512, K=8 frame sequence at 60 Hz: frame ``f`` is reconstructed at
    ``t_now = 64 + f * 16.667`` ms from a stream that keeps arriving at 8 samples per 64 ms per
    pixel (one sample at a uniform time and sub-pixel position in each 8 ms interval)."""
    stream: Stream
    scene: DiscScene
    width: int
    height: int
    k: int
    frame_times: np.ndarray

    def frame_stream(self, f: int) -> Stream:
        t_now = float(self.frame_times[f])
        mask = (self.stream.t <= np.float32(t_now)) & (self.stream.t > np.float32(t_now - 72.0))
        return self.stream.select(mask)

    def frame_workload(self, f: int) -> Workload:
        t_now = float(np.float32(self.frame_times[f]))
        return Workload("c4", self.frame_stream(f), self.width, self.height, self.k, "fp32",
                        t_now, t_now, self.scene,
                        description=f"512x512 K=8 64 discs, frame {f} at t={t_now:.3f} ms, FP32")


def make_c4_sequence(n_frames: int = 32, instance: int = 0, width: int = 512, height: int = 512,
                     k: int = 8) -> C4Sequence:
    rng = _rng(4000 + instance)
    t0, period = 64.0, 64.0 / k
    frame_times = np.array([np.float32(t0 + f * FRAME_MS) for f in range(n_frames)], np.float64)
    t_end = float(frame_times[-1])
    n_iv = int(np.ceil(t_end / period))
    scene = DiscScene(width, height, rng, 64, t0)
    shape = (height, width, n_iv)
    ux = rng.random(shape)
    uy = rng.random(shape)
    ut = rng.random(shape)
    jj, ii = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                         indexing="ij")
    x = (ii[:, :, None] + ux).astype(np.float32)
    y = (jj[:, :, None] + uy).astype(np.float32)
    t = ((np.arange(n_iv)[None, None, :] + ut) * period).astype(np.float32)
    parts = []
    for q in range(n_iv):  # shade one 8 ms interval at a time: disc sweeps stay small
        parts.append(_shade_to_stream(scene, x[:, :, q].reshape(-1), y[:, :, q].reshape(-1),
                                      t[:, :, q].reshape(-1), sort=False))
    s = Stream(*(np.concatenate([getattr(p, f) for p in parts])
                 for f in ("x", "y", "t", "r", "g", "b", "vx", "vy")))
    s = s.select(np.argsort(s.t, kind="stable"))
    return C4Sequence(s, scene, width, height, k, frame_times)


C5_SIZES = ((128, 128), (320, 240), (640, 480), (1024, 768))
C5_KS = (4, 8, 16)


def make_c5_batch(n: int = 64, sizes=C5_SIZES, ks=C5_KS, sort: bool = False, instances=None):
    """``n`` independent FP16-storage workloads of uneven size: each draws a size from ``sizes`` and
    a depth from ``ks`` (seed 5999 draws the recipe), then its own seeded 64-disc scene (seed
    ``5000 + i``), stratified at ``K`` samples per pixel over 64 ms."""
    recipe = _rng(5999)
    size_idx = recipe.integers(0, len(sizes), n)
    k_idx = recipe.integers(0, len(ks), n)
    out = []
    for i in range(n) if instances is None else instances:
        w, h = sizes[int(size_idx[i])]
        k = ks[int(k_idx[i])]
        rng = _rng(5000 + i)
        scene = DiscScene(w, h, rng, 64, 64.0)
        s = stratified_stream(scene, w, h, k, 64.0, 64.0, rng, sort)
        out.append(Workload("c5", s, w, h, k, "fp16", 64.0, 64.0, scene,
                            description=f"batch item {i}: {w}x{h} K={k}, FP16 storage"))
    return out


def c5_recipe(n: int = 64, sizes=C5_SIZES, ks=C5_KS):
    """(width, height, K) of each batch item without generating the streams."""
    recipe = _rng(5999)
    size_idx = recipe.integers(0, len(sizes), n)
    k_idx = recipe.integers(0, len(ks), n)
    return [(sizes[int(a)][0], sizes[int(a)][1], ks[int(b)]) for a, b in zip(size_idx, k_idx)]


# --------------------------------------------------------------------------------------------------
# Crosshair sampling (Sec. 4.1, 4.2)
# --------------------------------------------------------------------------------------------------

@dataclass
class Crosshairs:
    """Crosshairs as int32 indices into a sample stream, one entry per crosshair: the centre
    ``(x, y, t)``, the four samples one pixel away at the same instant (``xm``, ``xp`` at x -/+ 1,
    ``ym``, ``yp`` at y -/+ 1) and the earlier sample ``old`` at the same sub-pixel spot. -1 marks
    a sample that does not exist (a neighbour outside the image)."""
    centre: np.ndarray
    xm: np.ndarray
    xp: np.ndarray
    ym: np.ndarray
    yp: np.ndarray
    old: np.ndarray

    def __len__(self) -> int:
        return int(self.centre.shape[0])

    def arrays(self):
        return (self.centre, self.xm, self.xp, self.ym, self.yp, self.old)


def crosshair_stream(scene, width: int, height: int, visits: int, t_now: float, t_win: float,
                     rng: np.random.Generator):
    """A sample stream made by crosshair sampling, and its crosshairs.

    Every pixel is visited ``visits`` times at uniform times in ``(t_now - t_win, t_now]``. At each
    visit the sampler completes the crosshair started at the previous visit to that pixel (five new
    samples at the visit time: the centre at the spot chosen then, and its four neighbours one pixel
    away, those outside the image omitted; the earlier sample is the one taken at that spot) and
    starts the next one with a single sample at a new uniform sub-pixel spot (Sec. 4.2, with the
    tile of the paper's sampler narrowed to one pixel). Every sample goes into the stream, which is
    sorted by time; the crosshair indices refer to the sorted stream, and crosshairs are listed in
    the order they were completed.

    Draw order: spot offsets x, y as ``[H, W, visits]``, then visit-time offsets ``[H, W, visits]``.
    """
    shape = (height, width, visits)
    ux = rng.random(shape)
    uy = rng.random(shape)
    ut = np.sort(rng.random(shape), axis=2)
    jj, ii = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                         indexing="ij")
    sx = (ii[:, :, None] + ux).astype(np.float32)                # spot of the sample started
    sy = (jj[:, :, None] + uy).astype(np.float32)
    tv = (t_now - t_win * (1.0 - ut)).astype(np.float32)        # visit times, ascending
    # the starting samples: one per visit
    xs, ys, ts = [sx.reshape(-1)], [sy.reshape(-1)], [tv.reshape(-1)]
    n_start = sx.size
    start_id = np.arange(n_start, dtype=np.int64).reshape(shape)
    # completed crosshairs: visit v >= 1 completes the one started at v - 1
    cxh = sx[:, :, :-1].reshape(-1)
    cyh = sy[:, :, :-1].reshape(-1)
    tc = tv[:, :, 1:].reshape(-1)
    old = start_id[:, :, :-1].reshape(-1)
    nx = cxh.size
    ids = {}
    base = n_start
    one = np.float32(1.0)
    for name, dx, dy in (("centre", 0, 0), ("xm", -1, 0), ("xp", 1, 0), ("ym", 0, -1),
                         ("yp", 0, 1)):
        px = cxh if dx == 0 else (cxh - one if dx < 0 else cxh + one)
        py = cyh if dy == 0 else (cyh - one if dy < 0 else cyh + one)
        inside = (px >= 0) & (px < width) & (py >= 0) & (py < height)
        k = np.nonzero(inside)[0]
        idx = np.full(nx, -1, np.int64)
        idx[k] = base + np.arange(k.size)
        base += k.size
        xs.append(px[k]); ys.append(py[k]); ts.append(tc[k])
        ids[name] = idx
    x = np.concatenate(xs).astype(np.float32)
    y = np.concatenate(ys).astype(np.float32)
    t = np.concatenate(ts).astype(np.float32)
    s = _shade_to_stream(scene, x, y, t, sort=False)
    order = np.argsort(t, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    remap = lambda a: np.where(a >= 0, rank[np.maximum(a, 0)], -1).astype(np.int32)
    xh = Crosshairs(remap(ids["centre"]), remap(ids["xm"]), remap(ids["xp"]), remap(ids["ym"]),
                    remap(ids["yp"]), remap(old))
    # crosshairs in completion order (the order the sampler makes them)
    by_time = np.argsort(xh.centre, kind="stable")
    xh = Crosshairs(*(a[by_time] for a in xh.arrays()))
    return s.select(order), xh


@dataclass
class CrosshairWorkload:
    workload: Workload
    crosshairs: Crosshairs
    k_xh: int               # depth of the sampler's per-pixel crosshair queue


def make_crosshair_workload(instance: int = 0, width: int = 256, height: int = 256,
                            visits: int = 4, k: int = 16, k_xh: int = 4) -> CrosshairWorkload:
    """256x256 crosshair-sampled workload: a static 8-px checkerboard (grey 0.2 / 0.8, rotated by
    0.3 rad so that its edges cross pixels at every sub-pixel offset) under 16 discs
    moving at up to 0.2 px/ms, every pixel visited ``visits`` times over a 64 ms window (about 19
    samples per pixel), reconstructor depth ``k`` (FP32), sampler queue depth ``k_xh`` (Sec. 4 uses
    4). Seed 6000 + instance."""
    rng = _rng(6000 + instance)
    t_now, t_win = 64.0, 64.0
    scene = DiscScene(width, height, rng, 16, t_now, speed=0.2, checker=8.0, checker_angle=0.3)
    s, xh = crosshair_stream(scene, width, height, visits, t_now, t_win, rng)
    t_ref = float(np.float32(t_now))
    wl = Workload("crosshair", s, width, height, k, "fp32", t_ref, t_ref, scene,
                  description="256x256 crosshair sampling, checkerboard + 16 discs, FP32")
    return CrosshairWorkload(wl, xh, k_xh)
