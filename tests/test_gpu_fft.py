"""GPU parity: fdl_rfft2 / fdl_irfft2 against numpy's FFT (the oracle's DFT
step), on seeded images of the supported sizes 2^a 3^b."""
import numpy as np
import pytest
import torch

from oracle import fdl_oracle as O

pytestmark = pytest.mark.gpu


def fdl():
    import paper_1901_06919_amd as m
    return m


SIZES = [(1, 2), (3, 4), (8, 8), (12, 16), (24, 36), (128, 128), (256, 256), (384, 384), (512, 512),
         (96, 512), (512, 96), (4096, 8), (2, 8192), (64, 64), (768, 24), (1024, 48), (512, 36), (8, 768), (6, 1024), (2, 2048)]


@pytest.mark.parametrize("H,W", SIZES)
def test_rfft2_matches_numpy(H, W):
    print(f"rfft2 H={H} W={W}", flush=True)
    rng = np.random.default_rng(H * 31 + W)
    batch = 3
    img = rng.standard_normal((batch, H, W)).astype(np.float32)
    ref = O.rfft2(img.astype(np.float64))
    got = fdl().rfft2(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 = {err:.3e}")
    assert err < 2e-6


@pytest.mark.parametrize("H,W", SIZES)
def test_irfft2_matches_numpy(H, W):
    print(f"irfft2 H={H} W={W}", flush=True)
    rng = np.random.default_rng(H * 37 + W)
    batch = 2
    spec = (rng.standard_normal((batch, H, W // 2 + 1)) + 1j * rng.standard_normal((batch, H, W // 2 + 1)))
    spec = spec.astype(np.complex64)
    ref = O.irfft2(spec.astype(np.complex128), H, W)
    got = fdl().irfft2(torch.from_numpy(spec).cuda().clone(), H, W)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 = {err:.3e}")
    assert err < 2e-6


def test_fft_rejects_unsupported_sizes():
    f = fdl()
    with pytest.raises(f.FDLError):
        f.rfft2(torch.zeros((1, 8, 10), device="cuda"))     # W/2 = 5
    with pytest.raises(f.FDLError):
        f.rfft2(torch.zeros((1, 7, 8), device="cuda"))      # H = 7
