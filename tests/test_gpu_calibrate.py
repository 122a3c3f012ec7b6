"""Differentiation pattern: torch.autograd.Function over the hand-written
adjoint, and the 200-step gradient-descent calibration (7x7 views, 256^2,
16 layers, leave-one-out loss), eager and captured in a HIP graph."""
import numpy as np
import pytest
import torch

from oracle import fdl_oracle as O
from paper_1901_06919_amd import synth

pytestmark = pytest.mark.gpu


def _inputs():
    spec, u0, d0 = synth.lf_7x7_256_calib()
    views = O.forward_views(spec.layers.astype(np.float64), spec.u, spec.d) + spec.noise
    b = O.rfft2(views.astype(np.float32)).astype(np.complex64)
    return spec, torch.from_numpy(u0).cuda(), torch.from_numpy(d0).cuda(), torch.from_numpy(b).cuda()


def test_autograd_function_returns_the_adjoint():
    import paper_1901_06919_amd as fdl
    from paper_1901_06919_amd.calibrate import FDLCalibLoss
    spec, u0, d0, b = _inputs()
    H, W = spec.H, spec.W
    S = torch.from_numpy(synth.frequency_subset(H * (W // 2 + 1), 4096, np.random.default_rng(1))).cuda()
    u = u0.clone().requires_grad_(True)
    d = d0.clone().requires_grad_(True)
    loss = FDLCalibLoss.apply(u, d, b, H, W, spec.lam, spec.eps, spec.reg, 1, S)
    (3.0 * loss).backward()
    l2, gu, gd = fdl.calib_grad(b, u0, d0, H, W, spec.lam, spec.eps, spec.reg, 1, S)
    torch.cuda.synchronize()
    assert torch.allclose(u.grad.double(), 3.0 * gu, rtol=1e-6, atol=0)
    assert torch.allclose(d.grad.double(), 3.0 * gd, rtol=1e-6, atol=0)
    assert abs(loss.item() - l2.item()) == 0.0


def test_calibration_200_steps_eager_and_graph():
    from paper_1901_06919_amd.calibrate import calibrate
    spec, u0, d0, b = _inputs()
    H, W = spec.H, spec.W
    kw = dict(lam=spec.lam, eps=spec.eps, reg=spec.reg, mode=O.LOSS_LOO, steps=200, Q=4096, seed=5)
    e = calibrate(b, u0, d0, H, W, graph=False, **kw)
    g = calibrate(b, u0, d0, H, W, graph=True, **kw)
    L = e.losses.cpu().numpy()
    print(f"loss first 10 mean {L[:10].mean():.5e}  last 10 mean {L[-10:].mean():.5e}")
    assert L[-10:].mean() < L[:10].mean()
    assert torch.equal(e.u, g.u) and torch.equal(e.d, g.d)
    assert torch.equal(e.losses, g.losses)
