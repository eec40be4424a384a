"""GPU deep-buffer build against the FP64 reference: bit-exact (integer selection, exact float32
offsets, round-to-nearest-even binary16)."""
import numpy as np
import pytest

import afr_scenes as S
import oracle as O
from helpers import assert_buffers_equal, gpu_build, oracle_build_cached, workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,precision", [("c1", "fp32"), ("c1", "fp16"), ("c2", "fp32"),
                                            ("c0", "fp32"), ("c3", "fp16")])
def test_build_matches_reference(name, precision):
    wl = workload(name)
    print(f"build parity {name} {precision} {wl.width}x{wl.height} K={wl.k} n={len(wl.stream)}",
          flush=True)
    gbuf, gd = gpu_build(wl.stream, wl.width, wl.height, wl.k, precision, wl.t_ref)
    obuf, od = oracle_build_cached(name, precision, wl.k)
    assert gd == od
    assert_buffers_equal(gbuf, obuf)


@pytest.mark.parametrize("k", [1, 3, 17, 40, 100])
def test_build_depths_and_ties(k):
    """Depths on every selection path (register lists up to 64, scan selection above), a stream with
    many equal times (ties broken by stream index) and unstratified occupancy up to ~60 per pixel."""
    rng = np.random.default_rng(100 + k)
    w, h, n = 37, 23, 37 * 23 * 30
    x = (rng.random(n) ** 2 * w).astype(np.float32)  # skewed: dense columns on the left
    y = (rng.random(n) * h).astype(np.float32)
    t = rng.choice(np.arange(0, 50, 0.5, dtype=np.float32), n)
    c = rng.random((3, n)).astype(np.float32)
    s = S.Stream(x, y, t, c[0], c[1], c[2])
    print(f"build depth K={k} n={n}", flush=True)
    for precision in ("fp32", "fp16"):
        gbuf, gd = gpu_build(s, w, h, k, precision, 40.0)
        obuf, od = O.build_buffer(s, w, h, k, precision, 40.0)
        assert gd == od
        assert_buffers_equal(gbuf, obuf)


def test_build_drops_invalid_samples_and_handles_empty_streams():
    w, h = 9, 5
    x = np.array([0.0, 8.9999, 9.0, -1e-3, 4.5, np.nan, 4.5, 4.5, 2.5, 1.0, 3.0], np.float32)
    y = np.array([0.0, 4.9999, 1.0, 1.00, 5.0, 1.0, 1.5, 1.5, 0.5, np.inf, 2.0], np.float32)
    t = np.array([1.0, 2.0, 1.0, 1.0, 1.0, 1.0, 5.0, 1.0, 1.0, 1.0, -7e4], np.float32)
    r = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, np.inf, 0.9, 1.0, 0.5], np.float32)
    g = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 7e4, 1.0, 0.5], np.float32)
    s = S.Stream(x, y, t, r, g, r.copy())
    for precision, expect_dropped in (("fp32", 7), ("fp16", 9)):
        # fp16 additionally drops the colour 7e4 and the age 4 - (-7e4) > 65504
        gbuf, gd = gpu_build(s, w, h, 2, precision, 4.0)
        obuf, od = O.build_buffer(s, w, h, 2, precision, 4.0)
        assert gd == od == expect_dropped
        assert_buffers_equal(gbuf, obuf)
    empty = S.Stream(*(np.zeros(0, np.float32) for _ in range(6)))
    gbuf, gd = gpu_build(empty, w, h, 3, "fp32", 4.0)
    assert gd == 0 and int(gbuf.count.sum().item()) == 0
    assert bool((gbuf.src == -1).all().item()) and bool((gbuf.planes == 0).all().item())
