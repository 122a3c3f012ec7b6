"""The allocation-free calibration entry point (fdl_calib_grad_noalloc)
against fdl_calib_grad on the same inputs: two calls in a row on one GPU, the
second smaller, each bit-identical to the workspace entry point (same kernels
and launch shape), plus the rejection of a size beyond the static array."""
import numpy as np
import pytest
import torch

from oracle import fdl_oracle as O

pytestmark = pytest.mark.gpu


def fdl():
    import paper_1901_06919_amd as m
    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _case(seed, m, n, C, H, W):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-3, 3, (m, 2)).astype(np.float32)
    d = np.linspace(-2, 2, n).astype(np.float32)
    spec = O.rfft2(rng.standard_normal((m, C, H, W))).astype(np.complex64)
    return dev(spec), dev(u), dev(d)


def _outs(m, n):
    return (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty((m, 2), dtype=torch.float64, device="cuda"),
            torch.empty(n, dtype=torch.float64, device="cuda"))


def test_noalloc_matches_workspace_entry_point_twice():
    lam, eps = 1e-2, 1e-3
    # first call: 7x7 views, 16 layers, leave-one-out loss on 1500 sampled bins
    m, n, C, H, W = 49, 16, 1, 64, 64
    print(f"noalloc call 1: m={m} n={n} C={C} {H}x{W} LOO Q=1500", flush=True)
    spec, u, d = _case(901, m, n, C, H, W)
    F = H * (W // 2 + 1)
    idx = dev(np.random.default_rng(902).choice(np.arange(1, F), 1500, replace=False).astype(np.int32))
    ref = fdl().calib_grad(spec, u, d, H, W, lam, eps, O.REG_LAYER2, O.LOSS_LOO, idx)
    got = fdl().calib_grad_noalloc(spec, u, d, H, W, lam, eps, O.REG_LAYER2, O.LOSS_LOO, idx, out=_outs(m, n))
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    # second call, smaller: 3x3 views, 5 layers, 2 channels, paper loss on all bins,
    # with one out-of-range index counted in the status word
    m, n, C, H, W = 9, 5, 2, 16, 16
    print(f"noalloc call 2: m={m} n={n} C={C} {H}x{W} FIT", flush=True)
    spec, u, d = _case(903, m, n, C, H, W)
    F = H * (W // 2 + 1)
    raw = np.arange(F, dtype=np.int32)
    raw[5] = F + 3
    idx = dev(raw)
    st_ref = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = fdl().calib_grad(spec, u, d, H, W, lam, eps, O.REG_L2, O.LOSS_FIT, idx, status=st_ref)
    got = fdl().calib_grad_noalloc(spec, u, d, H, W, lam, eps, O.REG_L2, O.LOSS_FIT, idx, out=_outs(m, n), status=st)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
        assert torch.isfinite(a).all()
    assert int(st.item()) == 1 and int(st_ref.item()) == 1


def test_noalloc_rejects_sizes_beyond_the_static_array():
    m, n, C, H, W = 256, 32, 1, 8, 8
    print("noalloc: oversize request rejected on the host", flush=True)
    spec, u, d = _case(904, m, n, C, H, W)
    idx = dev(np.zeros(1000, dtype=np.int32))   # workspace 1000 x 545 doubles > 4 MiB
    with pytest.raises(RuntimeError, match="fdl_calib_grad_noalloc"):
        fdl().calib_grad_noalloc(spec, u, d, H, W, 1e-2, 1e-3, O.REG_L2, O.LOSS_FIT, idx, out=_outs(m, n))
