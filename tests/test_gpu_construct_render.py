"""GPU parity: fdl_construct and fdl_render against the FP64 oracle, element by
element on identical seeded inputs (complex64 spectra, float32 positions and
disparities), bar: relative L2 <= 1e-4 over the whole output array."""
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rand_case(seed, m, n, C, H, W, uniform):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-3, 3, (m, 2)).astype(np.float32)
    if uniform:
        d = np.linspace(-2.5, 2.5, n).astype(np.float32)
    else:
        d = np.sort(rng.uniform(-2.5, 2.5, n)).astype(np.float32)
    img = rng.standard_normal((m, C, H, W)).astype(np.float32)
    spec = O.rfft2(img).astype(np.complex64)
    return u, d, spec


CASES = [
    # (m, n, C, H, W, uniform d, reg)
    (4, 3, 1, 8, 8, True, O.REG_VIEW2),
    (4, 3, 1, 8, 8, False, O.REG_VIEW2),
    (9, 16, 3, 16, 24, True, O.REG_VIEW2),
    (13, 17, 2, 12, 16, True, O.REG_LAYER2),
    (13, 17, 2, 12, 16, False, O.REG_L2),
    (81, 30, 3, 32, 32, True, O.REG_VIEW2),
    (81, 30, 3, 20, 18, False, O.REG_VIEW2),
    (7, 32, 4, 6, 10, True, O.REG_LAYER2),
    (1, 1, 1, 2, 2, True, O.REG_VIEW2),
    (2, 5, 1, 3, 4, False, O.REG_L2),
    (25, 8, 1, 5, 130, True, O.REG_VIEW2),
]


@pytest.mark.parametrize("m,n,C,H,W,uniform,reg", CASES)
def test_construct_matches_oracle(m, n, C, H, W, uniform, reg):
    print(f"construct case m={m} n={n} C={C} H={H} W={W} uniform={uniform} reg={reg}", flush=True)
    u, d, spec = _rand_case(1000 + m * 7 + n, m, n, C, H, W, uniform)
    lam, eps = 1e-2, 1e-3
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, lam, eps, reg)
    got = fdl().construct(dev(spec), dev(u), dev(d), H, W, lam, eps, reg)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 = {err:.3e}")
    assert err < TOL


# one case per kernel instantiation: every solved-row class (8, 16, 20, 24,
# 28, 30, 32 rows), channel class (1, 2-3, 4) and disparity class
SOLVER_CLASSES = [(n, C, uniform) for n in (5, 12, 19, 23, 27, 29, 31, 32) for C in (1, 2, 4)
                  for uniform in (True, False)]


@pytest.mark.parametrize("n,C,uniform", SOLVER_CLASSES)
def test_construct_every_solver_class(n, C, uniform):
    m, H, W = 6, 6, 8
    print(f"construct class case n={n} C={C} uniform={uniform}", flush=True)
    u, d, spec = _rand_case(7000 + 3 * n + C, m, n, C, H, W, uniform)
    reg = O.REG_VIEW2 if uniform else O.REG_L2
    lam, eps = 1e-2, 1e-3
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, lam, eps, reg)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = fdl().construct(dev(spec), dev(u), dev(d), H, W, lam, eps, reg, status=st)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 = {err:.3e} status {st.item()}")
    assert st.item() == 0
    assert err < TOL


def test_construct_5x5_128_full_size():
    """The 5x5-view light field at full size (128^2, 8 layers), views from the oracle's forward model."""
    spec_in = synth.lf_5x5_128()
    views = O.forward_views(spec_in.layers.astype(np.float64), spec_in.u, spec_in.d) + spec_in.noise
    H, W = spec_in.H, spec_in.W
    b = O.rfft2(views.astype(np.float32)).astype(np.complex64)
    ref = O.construct(b.astype(np.complex128), spec_in.u.astype(np.float64), spec_in.d.astype(np.float64), H, W,
                      spec_in.lam, spec_in.eps, spec_in.reg)
    got = fdl().construct(dev(b), dev(spec_in.u), dev(spec_in.d), H, W, spec_in.lam, spec_in.eps, spec_in.reg)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"5x5/128 construct rel_l2 = {err:.3e}")
    assert err < TOL


def test_construct_status_counts_singular_dc():
    """eps = 0 with the view regulariser leaves the DC system singular (rank 1)."""
    u, d, spec = _rand_case(5, 9, 4, 1, 8, 8, True)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    fdl().construct(dev(spec), dev(u), dev(d), 8, 8, 1e-2, 0.0, O.REG_VIEW2, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) >= 1


def test_construct_rejects_bad_arguments():
    f = fdl()
    u, d, spec = _rand_case(6, 4, 3, 1, 8, 8, True)
    with pytest.raises(f.FDLError):
        f.construct(dev(spec), dev(u), dev(np.zeros(40, np.float32)), 8, 8, 1e-2, 1e-3)   # n > 32
    with pytest.raises(f.FDLError):
        f.construct(dev(spec), dev(u), dev(d), 8, 8, -1.0, 1e-3)


def _views(seed, V, shapes, pos=3.0, rmax=2.0, frange=3.0):
    rng = np.random.default_rng(seed)
    return synth.render_requests(V, rng, pos, rmax, -frange, frange, shapes=shapes)


RCASES = [
    # (n, C, H, W, V, shapes)
    (8, 1, 16, 16, 1, (O.AP_PINHOLE,)),
    (8, 1, 24, 18, 17, (O.AP_DISK, O.AP_SQUARE, O.AP_PINHOLE)),
    (30, 3, 32, 32, 40, (O.AP_DISK,)),
    (30, 3, 20, 34, 9, (O.AP_SQUARE,)),
    (5, 2, 6, 8, 33, (O.AP_DISK, O.AP_SQUARE)),
    (32, 4, 12, 12, 11, (O.AP_DISK, O.AP_SQUARE)),
]


@pytest.mark.parametrize("n,C,H,W,V,shapes", RCASES)
def test_render_matches_oracle(n, C, H, W, V, shapes):
    print(f"render case n={n} C={C} H={H} W={W} V={V} shapes={shapes}", flush=True)
    rng = np.random.default_rng(77 + n + V)
    x = O.rfft2(rng.standard_normal((n, C, H, W))).astype(np.complex64)
    d = np.sort(rng.uniform(-3, 3, n)).astype(np.float32)
    views = _views(n * 100 + V, V, shapes)
    ref = O.render(x.astype(np.complex128), d.astype(np.float64), views.astype(np.float64), H, W)
    got = fdl().render(dev(x), dev(d), dev(views), H, W)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 = {err:.3e}")
    assert err < TOL


def test_render_wide_apertures():
    """Apertures wide enough that 2 pi rho |s - d| |w| runs past the tabulated
    range of the disk spectrum (up to about 470), so both the table and the
    direct asymptotic form are exercised, with square apertures alongside."""
    n, C, H, W, V = 12, 1, 32, 32, 20
    print(f"render wide apertures n={n} V={V}", flush=True)
    rng = np.random.default_rng(4242)
    x = O.rfft2(rng.standard_normal((n, C, H, W))).astype(np.complex64)
    d = np.sort(rng.uniform(-3, 3, n)).astype(np.float32)
    views = _views(99, V, (O.AP_DISK, O.AP_SQUARE), rmax=12.0, frange=6.0)
    ref = O.render(x.astype(np.complex128), d.astype(np.float64), views.astype(np.float64), H, W)
    got = fdl().render(dev(x), dev(d), dev(views), H, W)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 = {err:.3e}")
    assert err < TOL


def test_render_9x9_views_reduced_resolution():
    """The benchmark's render requests (81 disk views at the input positions, radius
    U[0,2], focus U[-3,3]) over 30 layers of 1/f images at 64^2."""
    spec_in = synth.lf_9x9_512_rgb(H=64, W=64)
    x = O.rfft2(spec_in.layers).astype(np.complex64)
    H, W = spec_in.H, spec_in.W
    ref = O.render(x.astype(np.complex128), spec_in.d.astype(np.float64), spec_in.views.astype(np.float64), H, W)
    got = fdl().render(dev(x), dev(spec_in.d), dev(spec_in.views), H, W)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"9x9 render (64^2) rel_l2 = {err:.3e}")
    assert err < TOL


def test_construct_and_render_at_the_size_limits():
    """The largest sizes the entry points accept: 4096 views, 32 layers and
    4 channels for construction (uniform and general disparities), 2000
    views of 4 channels over 32 layers for rendering, on a small image."""
    H, W = 8, 10
    rng = np.random.default_rng(990)
    m, n, C = 4096, 32, 4
    u = rng.uniform(-4, 4, (m, 2)).astype(np.float32)
    spec = O.rfft2(rng.standard_normal((m, C, H, W))).astype(np.complex64)
    for d in (np.linspace(-2, 2, n).astype(np.float32), np.sort(rng.uniform(-2, 2, n)).astype(np.float32)):
        print(f"construct m={m} n={n} C={C} uniform={bool(np.allclose(np.diff(d), np.diff(d)[0]))}", flush=True)
        ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, 1e-2, 1e-3,
                          O.REG_VIEW2, chunk=16)
        got = fdl().construct(dev(spec), dev(u), torch.from_numpy(d), H, W, 1e-2, 1e-3, O.REG_VIEW2)
        torch.cuda.synchronize()
        err = O.rel_l2(got.cpu().numpy(), ref)
        print(f"  rel_l2 = {err:.3e}")
        assert err < TOL
    V = 2000
    layers = O.rfft2(rng.standard_normal((n, C, H, W))).astype(np.complex64)
    d = np.linspace(-2, 2, n).astype(np.float32)
    views = _views(991, V, (O.AP_DISK, O.AP_SQUARE, O.AP_PINHOLE))
    print(f"render V={V} n={n} C={C}", flush=True)
    ref = O.render(layers.astype(np.complex128), d.astype(np.float64), views.astype(np.float64), H, W)
    got = fdl().render(dev(layers), dev(d), dev(views), H, W)
    torch.cuda.synchronize()
    err = O.rel_l2(got.cpu().numpy(), ref)
    print(f"  rel_l2 = {err:.3e}")
    assert err < TOL


def test_construct_in_bin_ranges_equals_one_construction():
    """fdl_construct_bins over three ranges (ragged ends, one crossing a row)
    writes exactly the bits of one fdl_construct, and leaves other bins alone."""
    rng = np.random.default_rng(77)
    m, n, C, H, W = 9, 20, 3, 24, 30
    u = rng.uniform(-2, 2, (m, 2)).astype(np.float32)
    d = np.linspace(-2, 2, n).astype(np.float32)
    spec = O.rfft2(rng.standard_normal((m, C, H, W))).astype(np.complex64)
    F = H * (W // 2 + 1)
    print(f"construct_bins m={m} n={n} C={C} F={F}", flush=True)
    full = fdl().construct(dev(spec), dev(u), torch.from_numpy(d), H, W, 1e-2, 1e-3, O.REG_VIEW2)
    out = torch.full_like(full, complex(7.0, -7.0))
    for b0, cnt in ((0, 37), (37, 150), (187, F - 187)):
        fdl().construct_bins(dev(spec), dev(u), torch.from_numpy(d), H, W, 1e-2, 1e-3, O.REG_VIEW2, b0, cnt, out)
    torch.cuda.synchronize()
    assert torch.equal(out, full)
    part = torch.full_like(full, complex(7.0, -7.0))
    fdl().construct_bins(dev(spec), dev(u), torch.from_numpy(d), H, W, 1e-2, 1e-3, O.REG_VIEW2, 40, 60, part)
    flat, ref = part.reshape(n, C, F), full.reshape(n, C, F)
    assert torch.equal(flat[:, :, 40:100], ref[:, :, 40:100])
    assert bool((flat[:, :, :40] == complex(7.0, -7.0)).all()) and bool((flat[:, :, 100:] == complex(7.0, -7.0)).all())
