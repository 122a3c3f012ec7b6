"""GPU parity of the construction on views that lie on a complete lattice in
raster order (u_j = o + a g1 + b g2, j = a B + b), where the Toeplitz view loop
steps each phase exp(2 pi i e_t p_j) from view to view by one complex product
instead of forming it from the phase table (Sec. V-A phases; the lattice
identity p_j = <o,w> + a <g1,w> + b <g2,w> is exact for these positions).

Every case is checked against the FP64 oracle (relative L2 <= 1e-4), and
against the same light field with its views in a shuffled order, which is
not a lattice in raster order and so takes the table path: the normal
equations are sums over views, so the two must agree to float32 output
rounding (relative L2 <= 2e-6).  Geometries cover the lattice row at its
largest (16 views), rows longer than 16 (table path), more than 8 lattice
rows (the row start is re-anchored every 8 rows), one-row and one-view
lattices, a skewed lattice, column-major order, and positions one float ulp
off the lattice (table path)."""
import numpy as np
import pytest
import torch

from oracle import fdl_oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL_PATHS = 2e-6


def fdl():
    import paper_1901_06919_amd as m
    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def lattice(A, B, o, g1, g2):
    """Raster-order positions o + a g1 + b g2 (float32, exact for dyadic inputs)."""
    a, b = np.divmod(np.arange(A * B), B)
    u = np.asarray(o, np.float64)[None, :] + a[:, None] * np.asarray(g1, np.float64) + \
        b[:, None] * np.asarray(g2, np.float64)
    u32 = u.astype(np.float32)
    assert np.array_equal(u32.astype(np.float64), u), "lattice positions must be exact in float32"
    return u32


GEOMETRIES = {
    "9x9 integer grid": lambda: lattice(9, 9, (-4, -4), (0, 1), (1, 0)),
    "3x5 rectangular": lambda: lattice(3, 5, (-2, -1), (0, 1), (1, 0)),
    "2x16 longest row": lambda: lattice(2, 16, (-7.5, -0.5), (0, 1), (1, 0)),
    "1x17 row too long": lambda: lattice(1, 17, (-8, 0), (0, 0), (1, 0)),
    "17x3 re-anchored rows": lambda: lattice(17, 3, (-1, -8), (0, 1), (1, 0)),
    "1x7 single row": lambda: lattice(1, 7, (-3, 0.5), (0, 0), (1, 0)),
    "skewed 4x6": lambda: lattice(4, 6, (-1.25, 0.75), (0.5, 0.25), (0.25, -0.5)),
    "column-major 5x5": lambda: lattice(5, 5, (-2, -2), (1, 0), (0, 1)),
}


def _case(seed, u, n, C, H, W):
    rng = np.random.default_rng(seed)
    m = u.shape[0]
    d = np.linspace(-2.0, 2.0, n).astype(np.float32)
    spec = O.rfft2(rng.standard_normal((m, C, H, W)).astype(np.float32)).astype(np.complex64)
    return d, spec


def _construct(spec, u, d, H, W, lam, eps, reg):
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = fdl().construct(dev(spec), dev(u), dev(d), H, W, lam, eps, reg, status=st)
    torch.cuda.synchronize()
    return got.cpu().numpy(), int(st.item())


@pytest.mark.parametrize("geom", list(GEOMETRIES))
@pytest.mark.parametrize("n,C", [(30, 3), (12, 1), (8, 4)])
def test_lattice_views_match_oracle_and_table_path(geom, n, C):
    u = GEOMETRIES[geom]()
    m = u.shape[0]
    H, W = 10, 12
    print(f"lattice case {geom} m={m} n={n} C={C}", flush=True)
    d, spec = _case(300 + m + n + C, u, n, C, H, W)
    lam, eps, reg = 1e-2, 1e-3, O.REG_VIEW2
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, lam, eps, reg)
    got, st = _construct(spec, u, d, H, W, lam, eps, reg)
    err = O.rel_l2(got, ref)
    # the same light field with its views shuffled: not a raster lattice
    perm = np.random.default_rng(m).permutation(m)
    if m > 2:
        while np.all(perm == np.arange(m)):
            perm = np.random.default_rng(int(perm[0]) + 1).permutation(m)
    got_p, st_p = _construct(spec[perm], u[perm], d, H, W, lam, eps, reg)
    err_p = O.rel_l2(got_p, ref)
    diff = O.rel_l2(got, got_p.astype(np.complex128))
    print(f"  rel_l2 lattice {err:.3e} shuffled {err_p:.3e} between {diff:.3e} status {st} {st_p}")
    assert st == st_p
    assert err < TOL and err_p < TOL
    assert diff < TOL_PATHS


def test_single_view_lattice():
    u = np.array([[0.5, -1.0]], np.float32)
    H, W, n, C = 6, 8, 3, 2
    d, spec = _case(17, u, n, C, H, W)
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, 1e-2, 1e-3,
                      O.REG_VIEW2)
    got, _ = _construct(spec, u, d, H, W, 1e-2, 1e-3, O.REG_VIEW2)
    err = O.rel_l2(got, ref)
    print(f"single view rel_l2 {err:.3e}")
    assert err < TOL


def test_positions_one_ulp_off_the_lattice_take_the_table_path():
    """One position moved by one float32 ulp breaks the lattice identity; the
    result still matches the oracle on the moved position."""
    u = lattice(9, 9, (-4, -4), (0, 1), (1, 0))
    u[40, 0] = np.nextafter(u[40, 0], np.float32(10))
    n, C, H, W = 30, 3, 10, 12
    d, spec = _case(23, u, n, C, H, W)
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, 1e-2, 1e-3,
                      O.REG_VIEW2)
    got, st = _construct(spec, u, d, H, W, 1e-2, 1e-3, O.REG_VIEW2)
    err = O.rel_l2(got, ref)
    print(f"one-ulp case rel_l2 {err:.3e} status {st}")
    assert err < TOL


def test_lattice_at_the_benchmark_geometry_matches_oracle_tightly():
    """9x9 views, 30 layers, 3 channels on a 32x32 spectrum: the lattice path's
    error against the oracle stays at the level of the table path's."""
    u = GEOMETRIES["9x9 integer grid"]()
    n, C, H, W = 30, 3, 32, 32
    d, spec = _case(99, u, n, C, H, W)
    ref = O.construct(spec.astype(np.complex128), u.astype(np.float64), d.astype(np.float64), H, W, 1e-2, 1e-3,
                      O.REG_VIEW2)
    got, st = _construct(spec, u, d, H, W, 1e-2, 1e-3, O.REG_VIEW2)
    perm = np.random.default_rng(5).permutation(u.shape[0])
    got_p, _ = _construct(spec[perm], u[perm], d, H, W, 1e-2, 1e-3, O.REG_VIEW2)
    err, err_p = O.rel_l2(got, ref), O.rel_l2(got_p, ref)
    print(f"benchmark geometry rel_l2 lattice {err:.3e} table {err_p:.3e} status {st}")
    assert st == 0
    assert err < max(2.0 * err_p, 1e-6)
