"""afr_sampler_select_noalloc (the selection with its prefix in a library-owned device array)
against afr_sampler_select (workspace from the caller), through the C ABI.

Both run the same two kernels on the same float32 tile errors and random bits, so the spots and
tiles must agree bit for bit. Calls come in a row on one stream, each smaller than the one before
(fewer tiles and fewer samples), so a result that read a stale prefix entry of the previous call
would differ; the first call uses the array's full 65 536 tiles.
"""
import numpy as np
import pytest

from helpers import DEV, afr_mod, torch_mod

pytestmark = pytest.mark.gpu


def _case(rng, w, h, tile, n, torch):
    ty, tx = -(-h // tile), -(-w // tile)
    E = (rng.random((ty, tx)) ** 3).astype(np.float32)
    E.reshape(-1)[::7] = 0.0
    r = rng.integers(0, 2 ** 32, 3 * n, dtype=np.uint64).astype(np.uint32)
    return torch.from_numpy(E).to(DEV), torch.from_numpy(r.view(np.int32)).to(DEV)


def test_noalloc_select_equals_workspace_select():
    torch = torch_mod()
    afr = afr_mod()
    rng = np.random.default_rng(355)
    # (width, height, tile, samples): 256x256 tiles = 65536 (the limit), then smaller ones
    for w, h, tile, n in ((2048, 2048, 8, 300_000), (640, 480, 8, 50_000), (250, 131, 8, 7_001),
                          (40, 30, 16, 33)):
        print(f"noalloc select {w}x{h} tile={tile} n={n}", flush=True)
        E, rnd = _case(rng, w, h, tile, n, torch)
        x = torch.full((n,), -1.0, device=DEV)
        y = torch.full((n,), -1.0, device=DEV)
        t = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        afr.sampler_select_noalloc(w, h, tile, E, rnd, x, y, t)
        rx, ry, rt = afr.sampler_select(w, h, tile, E, rnd)
        torch.cuda.synchronize()
        assert torch.equal(t, rt)
        assert torch.equal(x.view(torch.int32), rx.view(torch.int32))
        assert torch.equal(y.view(torch.int32), ry.view(torch.int32))
        assert bool(((x >= 0) & (x < w) & (y >= 0) & (y < h)).all())


def test_noalloc_select_limits():
    torch = torch_mod()
    afr = afr_mod()
    print("noalloc select limits", flush=True)
    E = torch.ones((2, 3), device=DEV)
    z = torch.zeros(0, device=DEV)
    x, y, t = afr.sampler_select_noalloc(20, 10, 8, E, torch.zeros(0, dtype=torch.int32, device=DEV),
                                         z, z, None)
    assert x.numel() == 0
    # one tile more than the array holds: rejected before any launch
    E = torch.ones((257, 256), device=DEV)
    rnd = torch.zeros(3, dtype=torch.int32, device=DEV)
    o = torch.zeros(1, device=DEV)
    with pytest.raises(afr.AfrError):
        afr.sampler_select_noalloc(2048, 2049, 8, E, rnd, o, o.clone(), None)
