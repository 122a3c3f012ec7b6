"""GPU parity for layer construction with the second-order view regulariser
over a finite camera-plane square (Eq. GTG), against the FP64 oracle; both the
Toeplitz (uniform disparities) and the general Gram paths."""
import numpy as np
import pytest
import torch

from oracle import fdl_oracle as O
from paper_1901_06919_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


def fdl():
    import paper_1901_06919_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("grid,n,C,H,W,region,uniform", [(3, 5, 1, 24, 40, 2.0, True), (4, 20, 3, 16, 24, 4.5, False),
                                                         (5, 32, 4, 12, 16, 8.0, True), (1, 1, 1, 2, 2, 1.0, True),
                                                         (3, 12, 2, 20, 18, 0.5, False)])
def test_construct_region_matches_oracle(grid, n, C, H, W, region, uniform):
    print(f"construct_region grid={grid} n={n} C={C} H={H} W={W} r={region} uniform={uniform}", flush=True)
    rng = np.random.default_rng(900 + n + C)
    u = synth.centered_grid_positions(grid).astype(np.float32)
    if not uniform:
        u = u + rng.uniform(-0.3, 0.3, u.shape).astype(np.float32)
    m = u.shape[0]
    d = (np.linspace(-2, 2, n) if uniform else np.sort(rng.uniform(-2, 2, n))).astype(np.float32)
    spec = O.rfft2(rng.standard_normal((m, C, H, W))).astype(np.complex64)
    lam, eps = 0.05, 1e-3
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, lam, eps,
                      O.REG_VIEW2_REGION, region=region)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = fdl().construct_region(dev(spec), dev(u), torch.from_numpy(d), H, W, lam, eps, region, status=st)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 {err:.3e} status {st.item()}")
    assert err < TOL
    assert st.item() == 0


# one case per kernel instantiation: row slots (n <= 16 or not) x channel class
# (1, 2-3, 4) x disparity class (uniform on an exact grid, general on a
# jittered one)
REGION_CLASSES = [(n, C, uniform) for n in (12, 21) for C in (1, 3, 4) for uniform in (True, False)]


@pytest.mark.parametrize("n,C,uniform", REGION_CLASSES)
def test_construct_region_every_instantiation(n, C, uniform):
    print(f"construct_region class n={n} C={C} uniform={uniform}", flush=True)
    rng = np.random.default_rng(1200 + 7 * n + C)
    u = synth.centered_grid_positions(3).astype(np.float32)
    if not uniform:
        u = u + rng.uniform(-0.3, 0.3, u.shape).astype(np.float32)
    m = u.shape[0]
    H, W = 10, 12
    d = (np.linspace(-2, 2, n) if uniform else np.sort(rng.uniform(-2, 2, n))).astype(np.float32)
    spec = O.rfft2(rng.standard_normal((m, C, H, W))).astype(np.complex64)
    lam, eps, region = 0.05, 1e-3, 3.0
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, lam, eps,
                      O.REG_VIEW2_REGION, region=region)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = fdl().construct_region(dev(spec), dev(u), torch.from_numpy(d), H, W, lam, eps, region, status=st)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 {err:.3e} status {st.item()}")
    assert err < TOL
    assert st.item() == 0


def test_construct_region_large_side_is_the_view_regulariser():
    H, W = 32, 32
    rng = np.random.default_rng(910)
    u = synth.centered_grid_positions(5).astype(np.float32)
    d = np.linspace(-2, 2, 16).astype(np.float32)
    spec = dev(O.rfft2(rng.standard_normal((25, 1, H, W))).astype(np.complex64))
    a = fdl().construct_region(spec, dev(u), torch.from_numpy(d), H, W, 0.05, 1e-3, 1e6)
    b = fdl().construct(spec, dev(u), torch.from_numpy(d), H, W, 0.05, 1e-3, O.REG_VIEW2)
    torch.cuda.synchronize()
    err = O.rel_l2(a.cpu().numpy(), b.cpu().numpy())
    print(f"  r = 1e6 vs view regulariser rel_l2 {err:.3e}")
    assert err < 1e-5


def test_construct_region_rejects_bad_side():
    m = fdl()
    spec = dev(np.zeros((4, 1, 8, 5), np.complex64))
    u = dev(np.zeros((4, 2), np.float32))
    with pytest.raises(m.FDLError):
        m.construct_region(spec, u, torch.zeros(3), 8, 8, 0.1, 1e-3, 0.0)
