"""Gradient-descent calibration of view positions and disparities (Sec. V-B).

``FDLCalibLoss`` exposes ``fdl_calib_grad`` to torch autograd: the forward
pass runs the kernel once and returns the loss, the gradient with respect to
(u, d) that the same kernel produced is what ``backward`` hands to autograd
(the hand-written adjoint; there is no autograd tape through the solve).

``calibrate`` runs the paper's loop -- fresh random frequency subset, layers
re-solved at the current (u, d), gradient, normalised step -- entirely on the
device; with ``graph=True`` all steps are captured once in a HIP graph and
replayed, so the host issues one launch for the whole run.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import calib_grad, calib_workspace_bytes, gd_step


class FDLCalibLoss(torch.autograd.Function):
    """loss = E(u, d) of ``fdl_calib_grad``; u [m,2] f32, d [n] f32 (leaves)."""

    @staticmethod
    def forward(ctx, u, d, view_spec, H, W, lam, eps, reg, mode, freq_idx=None):
        loss, gu, gd = calib_grad(view_spec, u.detach().contiguous(), d.detach().contiguous(), H, W, lam, eps,
                                  reg, mode, freq_idx)
        ctx.save_for_backward(gu, gd)
        ctx.dtypes = (u.dtype, d.dtype)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        gu, gd = ctx.saved_tensors
        tu, td = ctx.dtypes
        return (g * gu).to(tu), (g * gd).to(td), None, None, None, None, None, None, None, None


@dataclass
class CalibResult:
    u: torch.Tensor
    d: torch.Tensor
    loss_first: float
    loss_last: float
    losses: Optional[torch.Tensor] = None   # [steps] f64 on device


def calibrate(view_spec: torch.Tensor, u0: torch.Tensor, d0: torch.Tensor, H: int, W: int, lam: float, eps: float,
              reg: int, mode: int, steps: int = 200, Q: int = 4096, alpha: float = 0.2, eps_g: float = 1e-6,
              seed: int = 5, graph: bool = False, subsets: Optional[torch.Tensor] = None) -> CalibResult:
    """Run ``steps`` iterations of the Sec. V-B update on the device.

    Each step draws Q distinct bins uniformly from [1, F) (seeded; all subsets
    are generated up front so the loop has no host work), evaluates the loss
    and gradient there and applies the normalised step.  With ``graph=True``
    the whole loop is captured into one HIP graph and replayed once."""
    dev = view_spec.device
    m = u0.shape[0]
    n = d0.shape[0]
    F = H * (W // 2 + 1)
    Q = min(Q, F - 1)
    if subsets is None:
        rng = np.random.default_rng(seed)
        idx = np.stack([np.sort(rng.choice(np.arange(1, F), size=Q, replace=False)) for _ in range(steps)])
        subsets = torch.from_numpy(idx.astype(np.int32)).to(dev)
    u = u0.detach().clone().contiguous()
    d = d0.detach().clone().contiguous()
    losses = torch.empty(steps, dtype=torch.float64, device=dev)
    gu = torch.empty((m, 2), dtype=torch.float64, device=dev)
    gd = torch.empty(n, dtype=torch.float64, device=dev)
    ws = torch.empty(max(calib_workspace_bytes(m, n, Q), 1), dtype=torch.uint8, device=dev)

    def body():
        for s in range(steps):
            calib_grad(view_spec, u, d, H, W, lam, eps, reg, mode, subsets[s], out=(losses[s:s + 1], gu, gd), ws=ws)
            gd_step(u, d, gu, gd, alpha, eps_g)

    if graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                body()
        torch.cuda.current_stream(dev).wait_stream(side)
        # capture does not execute: restore the start point, then replay once
        u.copy_(u0)
        d.copy_(d0)
        g.replay()
        torch.cuda.current_stream(dev).synchronize()
    else:
        body()
    torch.cuda.synchronize(dev)
    return CalibResult(u, d, float(losses[0].item()), float(losses[-1].item()), losses)
