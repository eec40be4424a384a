"""Fit the filter parameters sigma (spatial width scale) and tau (temporal sensitivity) by gradient
descent on the reconstruction error.

The loss is the mean over frames of the per-frame RMS error against a reference image, the error
measure of the paper's gold-standard evaluation (Sec. 7). Gradients come from the adjoint kernel
through ``ReconstructFn``; the tile statistics are held fixed within a step (they are inputs of the
gather). Parameters are optimised in log space, so both stay positive, with Adam.

A checkpoint is a small JSON file (parameters, step, optimiser moments, loss history); resuming from
it continues the same trajectory because every kernel on the path is deterministic.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

from . import DeepBuffer, Params, reconstruct_differentiable


@dataclass
class FitState:
    log_sigma: float
    log_tau: float
    step: int = 0
    m: List[float] = field(default_factory=lambda: [0.0, 0.0])
    v: List[float] = field(default_factory=lambda: [0.0, 0.0])
    history: List[dict] = field(default_factory=list)

    @property
    def sigma(self) -> float:
        return math.exp(self.log_sigma)

    @property
    def tau(self) -> float:
        return math.exp(self.log_tau)

    def save(self, path: str):
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.__dict__, f)
        os.replace(tmp, path)

    @staticmethod
    def load(path: str) -> "FitState":
        with open(path) as f:
            return FitState(**json.load(f))


def frame_loss(frames: Sequence[Tuple[DeepBuffer, Params, torch.Tensor]], sigma, tau,
               form: str = "tiled"):
    """Mean over frames of RMS(C_f - GT_f); differentiable in sigma and tau (0-d tensors)."""
    total = 0.0
    for buf, p, gt in frames:
        rgb = reconstruct_differentiable(buf, p, sigma, tau, form=form)
        total = total + torch.sqrt(((rgb - gt) ** 2).mean())
    return total / len(frames)


def fit(frames: Sequence[Tuple[DeepBuffer, Params, torch.Tensor]], sigma0: float = 1.0,
        tau0: float = 0.5, steps: int = 20, lr: float = 0.05, betas=(0.9, 0.999),
        eps: float = 1e-8, state: Optional[FitState] = None, checkpoint: Optional[str] = None,
        form: str = "tiled", log=None) -> FitState:
    """Adam on (log sigma, log tau). Returns the final state; writes ``checkpoint`` after each step
    when given (and resumes from ``state`` when given)."""
    st = state or FitState(math.log(sigma0), math.log(tau0))
    dev = frames[0][0].planes.device
    b1, b2 = betas
    while st.step < steps:
        ls = torch.tensor(st.log_sigma, dtype=torch.float64, device=dev, requires_grad=True)
        lt = torch.tensor(st.log_tau, dtype=torch.float64, device=dev, requires_grad=True)
        loss = frame_loss(frames, torch.exp(ls).float(), torch.exp(lt).float(), form)
        loss.backward()
        g = [float(ls.grad), float(lt.grad)]
        st.step += 1
        for i in range(2):
            st.m[i] = b1 * st.m[i] + (1 - b1) * g[i]
            st.v[i] = b2 * st.v[i] + (1 - b2) * g[i] * g[i]
        mhat = [m / (1 - b1 ** st.step) for m in st.m]
        vhat = [v / (1 - b2 ** st.step) for v in st.v]
        rec = {"step": st.step, "loss": float(loss), "sigma": st.sigma, "tau": st.tau,
               "grad_log_sigma": g[0], "grad_log_tau": g[1]}
        st.log_sigma -= lr * mhat[0] / (math.sqrt(vhat[0]) + eps)
        st.log_tau -= lr * mhat[1] / (math.sqrt(vhat[1]) + eps)
        st.history.append(rec)
        if log:
            log(rec)
        if checkpoint:
            st.save(checkpoint)
    return st
