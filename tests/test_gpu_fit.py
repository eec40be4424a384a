"""Fitting sigma and tau by descent on the per-frame RMS error against the analytic ground truth
(the adjoint kernel through ReconstructFn), and exact resume from a JSON checkpoint."""
import os

import pytest

import afr_scenes as S
from helpers import DEV, afr_mod, gpu_build, torch_mod

pytestmark = pytest.mark.gpu


def _frames(n=4, size=128, k=8):
    torch = torch_mod()
    afr = afr_mod()
    seq = S.make_c4_sequence(n_frames=n, width=size, height=size, k=k)
    out = []
    for f in range(n):
        wl = seq.frame_workload(f)
        buf, _ = gpu_build(wl.stream, size, size, k, "fp32", wl.t_ref)
        gt = torch.from_numpy(S.ground_truth(seq.scene, size, size, wl.t_now, 4)).float().to(DEV)
        out.append((buf, afr.Params(t_now=wl.t_now), gt))
    return out


def test_fit_reduces_rms_and_resumes_exactly(tmp_path):
    from paper_2510_15876_amd import fit as F
    frames = _frames()
    full = F.fit(frames, sigma0=1.0, tau0=0.5, steps=6, lr=0.1)
    losses = [h["loss"] for h in full.history]
    print("losses", losses, "sigma", full.sigma, "tau", full.tau, flush=True)
    assert losses[-1] < losses[0]
    ck = os.path.join(tmp_path, "fit.json")
    F.fit(frames, sigma0=1.0, tau0=0.5, steps=3, lr=0.1, checkpoint=ck)
    resumed = F.fit(frames, steps=6, lr=0.1, state=F.FitState.load(ck))
    assert resumed.log_sigma == full.log_sigma and resumed.log_tau == full.log_tau
    assert [h["loss"] for h in resumed.history] == losses
