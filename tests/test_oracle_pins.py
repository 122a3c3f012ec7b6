"""Pins for the FP64 oracle: each test checks it against something other than
itself (direct sums, an independent solver, spatial-domain circular shifts,
closed forms, integrals, finite differences)."""
import cmath
import math

import numpy as np
import pytest

from oracle import brute
from oracle import fdl_oracle as O


# ---------------------------------------------------------------- DFT ------

@pytest.mark.parametrize("H,W", [(8, 8), (6, 10), (12, 9), (9, 6)])
def test_rfft2_matches_direct_sum(H, W):
    rng = np.random.default_rng(1)
    img = rng.standard_normal((H, W))
    full = brute.naive_dft2(img)
    np.testing.assert_allclose(O.rfft2(img), full[:, : W // 2 + 1], rtol=0, atol=1e-11)


@pytest.mark.parametrize("H,W", [(8, 8), (6, 10), (10, 4)])
def test_irfft2_drops_imag_of_self_conjugate_bins(H, W):
    rng = np.random.default_rng(2)
    half = rng.standard_normal((H, W // 2 + 1)) + 1j * rng.standard_normal((H, W // 2 + 1))
    ref = brute.naive_idft2_real(brute.hermitian_extend(half, W))
    np.testing.assert_allclose(O.irfft2(half, H, W), ref, rtol=0, atol=1e-12)
    img = rng.standard_normal((H, W))
    np.testing.assert_allclose(O.irfft2(O.rfft2(img), H, W), img, atol=1e-12)


def test_frequency_grid_conventions():
    wx, wy = O.freq_grid(8, 8)
    assert wx[0, 4] == 0.5            # Nyquist column is +1/2
    assert wy[4, 0] == -0.5           # Nyquist row is -1/2
    assert wy[1, 0] == 0.125 and wy[7, 0] == -0.125


# ------------------------------------------------------- A and M ----------

def _explicit_A(u, d, wx, wy):
    m, n = len(u), len(d)
    A = np.zeros((m, n), dtype=np.complex128)
    for j in range(m):
        for k in range(n):
            A[j, k] = cmath.exp(2j * math.pi * d[k] * (u[j][0] * wx + u[j][1] * wy))
    return A


def test_gram_dirichlet_closed_form_integer_grid():
    """Integer grid {-R..R}^2: (A^H A)_{k1 k2} = D(th_x) D(th_y),
    th = 2 pi (d_k2 - d_k1) w, D(t) = sin((2R+1) t / 2) / sin(t / 2)."""
    R = 2
    g = np.arange(-R, R + 1)
    vv, uu = np.meshgrid(g, g, indexing="ij")
    u = np.stack([uu.ravel(), vv.ravel()], 1).astype(float)
    d = np.array([-1.3, -0.2, 0.7, 1.9])
    wx = np.array([0.0, 0.11, 0.31, 0.5, 0.05])
    wy = np.array([0.0, -0.23, 0.17, -0.5, 0.41])
    A = O.a_matrix(u, d, wx, wy)
    G = np.conj(np.swapaxes(A, 1, 2)) @ A

    def dirichlet(t):
        if abs(math.sin(t / 2)) < 1e-12:
            return 2 * R + 1.0
        return math.sin((2 * R + 1) * t / 2) / math.sin(t / 2)

    for f in range(len(wx)):
        for a in range(len(d)):
            for b in range(len(d)):
                dd = d[b] - d[a]
                ref = dirichlet(2 * math.pi * dd * wx[f]) * dirichlet(2 * math.pi * dd * wy[f])
                assert abs(G[f, a, b] - ref) < 1e-10
        assert np.allclose(np.diag(G[f]).real, len(u), atol=1e-12)


def test_a_matrix_against_explicit_loops():
    rng = np.random.default_rng(3)
    u = rng.uniform(-3, 3, (7, 2))
    d = rng.uniform(-2, 2, 5)
    wx = rng.uniform(0, 0.5, 4)
    wy = rng.uniform(-0.5, 0.5, 4)
    A = O.a_matrix(u, d, wx, wy)
    for f in range(4):
        np.testing.assert_allclose(A[f], _explicit_A(u, d, wx[f], wy[f]), atol=1e-13)


# --------------------------------------------------------- construct ------

def _tiny_problem(seed, m=6, n=4, C=2, H=8, W=8):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-2, 2, (m, 2))
    d = np.sort(rng.uniform(-2, 2, n))
    imgs = rng.standard_normal((m, C, H, W))
    return u, d, O.rfft2(imgs)


@pytest.mark.parametrize("reg", [O.REG_VIEW2, O.REG_LAYER2, O.REG_L2])
def test_construct_matches_stacked_least_squares(reg):
    H, W = 8, 8
    u, d, spec = _tiny_problem(4, H=H, W=W)
    lam, eps = 0.3, 1e-2
    x = O.construct(spec, u, d, H, W, lam, eps, reg)
    wx, wy = O.freq_grid(H, W)
    m, C = spec.shape[:2]
    n = len(d)
    for ky in range(H):
        for kx in range(W // 2 + 1):
            A = _explicit_A(u, d, wx[ky, kx], wy[ky, kx])
            if reg == O.REG_VIEW2:
                w2 = wx[ky, kx] ** 2 + wy[ky, kx] ** 2
                Gam = np.diag(w2 * d ** 2)
            elif reg == O.REG_LAYER2:
                Gam = -2 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
            else:
                Gam = np.eye(n)
            ref = brute.stacked_lstsq(A, spec[:, :, ky, kx], Gam, lam, eps)
            np.testing.assert_allclose(x[:, :, ky, kx], ref, rtol=1e-9, atol=1e-9)


def test_construct_dc_closed_form():
    """At w = 0 every A_jk = 1 and the view regulariser vanishes, so
    x_k(0) = sum_j b_j / (m n + eps) for every layer."""
    H, W = 8, 8
    u, d, spec = _tiny_problem(5, m=9, n=5, H=H, W=W)
    eps = 1e-3
    x = O.construct(spec, u, d, H, W, 0.7, eps, O.REG_VIEW2)
    m, n = 9, 5
    ref = spec[:, :, 0, 0].sum(axis=0) / (m * n + eps)
    for k in range(n):
        np.testing.assert_allclose(x[k, :, 0, 0], ref, rtol=1e-9)  # cond(M) ~ mn/eps


def _roll_views(layers, u_int, d_int):
    """Views from spatial layers by circular shifts: view_j(y, x) =
    sum_k layer_k(y + v_j d_k, x + u_j d_k) (Eq. Prior1 with integer shifts),
    no Fourier arithmetic."""
    n, C, H, W = layers.shape
    out = np.zeros((len(u_int), C, H, W))
    for j, (uj, vj) in enumerate(u_int):
        for k in range(n):
            out[j] += np.roll(layers[k], (-vj * d_int[k], -uj * d_int[k]), axis=(-2, -1))
    return out


def test_construct_exact_recovery_of_band_limited_layers():
    """Noise-free views of layers whose spectra live only where A is well
    conditioned are inverted exactly when lambda, eps -> 0."""
    H, W = 16, 16
    u_int = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    d_int = [-1, 0, 2]
    rng = np.random.default_rng(6)
    layers = rng.standard_normal((3, 1, H, W))
    spec = O.rfft2(layers)
    wx, wy = O.flat_freqs(H, W)
    A = O.a_matrix(np.array(u_int, float), np.array(d_int, float), wx, wy)
    cond = np.linalg.cond(A).reshape(H, W // 2 + 1)
    spec[:, :, cond >= 1e3] = 0.0
    layers = O.irfft2(spec, H, W)
    spec = O.rfft2(layers)
    assert (cond < 1e3).mean() > 0.5
    views = _roll_views(layers, u_int, d_int)
    x = O.construct(O.rfft2(views), np.array(u_int, float), np.array(d_int, float), H, W,
                    1e-12, 1e-12, O.REG_VIEW2)
    assert O.rel_l2(x, spec) < 1e-7


def test_construct_reproduces_input_views():
    """All-band layers are not identifiable, but with lambda, eps -> 0 the
    layers rendered back at the input positions reproduce the views."""
    H, W = 16, 16
    u_int = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    d_int = [-2, -1, 0, 1, 2]
    rng = np.random.default_rng(7)
    layers = rng.standard_normal((5, 2, H, W))
    views = _roll_views(layers, u_int, d_int)
    u = np.array(u_int, float)
    d = np.array(d_int, float)
    x = O.construct(O.rfft2(views), u, d, H, W, 1e-12, 1e-12, O.REG_VIEW2)
    rv = np.zeros((9, 5))
    rv[:, :2] = u
    back = O.render_images(x, d, rv, H, W)
    assert O.rel_l2(back, views) < 1e-6


def test_construct_sampled_bins_match_full():
    H, W = 8, 12
    u, d, spec = _tiny_problem(8, H=H, W=W)
    full = O.construct(spec, u, d, H, W, 0.1, 1e-3)
    idx = np.array([0, 5, 17, 30, 55])
    part = O.construct(spec, u, d, H, W, 0.1, 1e-3, freq_index=idx)
    np.testing.assert_allclose(part, full.reshape(len(d), spec.shape[1], -1)[:, :, idx], atol=1e-13)


# ------------------------------------------------------------ render ------

def test_render_integer_shift_is_circular_roll():
    H, W = 12, 16
    rng = np.random.default_rng(9)
    layer = rng.standard_normal((1, 1, H, W))
    spec = O.rfft2(layer)
    for (u0, v0, dk) in [(1, 0, 2), (-2, 1, 1), (1, -1, -3)]:
        img = O.render_images(spec, np.array([float(dk)]), np.array([[u0, v0, 0, 0, 0]], float), H, W)
        ref = np.roll(layer[0], (-v0 * dk, -u0 * dk), axis=(-2, -1))
        np.testing.assert_allclose(img[0], ref, atol=1e-12)


def test_render_zero_radius_is_pinhole_and_in_focus_layer_is_sharp():
    H, W = 8, 8
    rng = np.random.default_rng(10)
    x = O.rfft2(rng.standard_normal((3, 1, H, W)))
    d = np.array([-1.0, 0.5, 2.0])
    pin = O.render(x, d, np.array([[0.3, -0.7, 0.0, 0.0, 0]]), H, W)
    for shape in (1, 2):
        r0 = O.render(x, d, np.array([[0.3, -0.7, 1.1, 0.0, shape]]), H, W)
        np.testing.assert_allclose(r0, pin, atol=1e-12)
        # only layer 1 present and focused on it: the aperture has no effect
        x1 = np.zeros_like(x)
        x1[1] = x[1]
        a = O.render(x1, d, np.array([[0.3, -0.7, 0.5, 1.7, shape]]), H, W)
        b = O.render(x1, d, np.array([[0.3, -0.7, 0.0, 0.0, 0]]), H, W)
        np.testing.assert_allclose(a, b, atol=1e-12)


@pytest.mark.parametrize("shape,rho", [(1, 0.8), (1, 1.7), (2, 0.6), (2, 1.3)])
def test_aperture_spectrum_against_quadrature(shape, rho):
    for xi in [(0.0, 0.0), (0.13, -0.21), (0.41, 0.07), (-0.3, 0.33)]:
        q = brute.aperture_quadrature(shape, rho, xi[0], xi[1], N=1201)
        a = float(O.psi_hat(shape, rho, np.array([xi[0]]), np.array([xi[1]]))[0])
        assert abs(a - q) < 2e-3, (shape, rho, xi, a, q)


def test_render_matches_refocus_integral():
    """Eq. BsFourier against its defining integral Eq. BsIntermediate."""
    rng = np.random.default_rng(11)
    n = 3
    d = np.array([-1.2, 0.1, 0.9])
    Lb = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    wx, wy = 0.19, -0.27
    for (u0, v0, s, shape, rho) in [(0.4, -0.3, 0.5, 1, 0.9), (-1.0, 0.6, -0.7, 2, 0.7)]:
        # evaluate closed form at a single bin through psi_hat
        acc = 0j
        for k in range(n):
            acc += (cmath.exp(2j * math.pi * d[k] * (u0 * wx + v0 * wy))
                    * O.psi_hat(shape, rho, np.array([(s - d[k]) * wx]), np.array([(s - d[k]) * wy]))[0]
                    * Lb[k])
        q = brute.refocus_quadrature(Lb, d, u0, v0, s, shape, rho, wx, wy, N=801)
        assert abs(acc - q) < 3e-3 * (1 + abs(q)), (acc, q)


# ------------------------------------------------------- calibration ------

def _calib_case(seed=12, m=5, n=3, H=8, W=8, C=1):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.5, 1.5, (m, 2))
    d = np.sort(rng.uniform(-1.5, 1.5, n))
    spec = O.rfft2(rng.standard_normal((m, C, H, W)))
    F = H * (W // 2 + 1)
    return u, d, spec, np.arange(1, F)


@pytest.mark.parametrize("reg", [O.REG_LAYER2, O.REG_VIEW2])
def test_fit_gradient_matches_finite_differences(reg):
    """Eq. gradP / gradD (envelope theorem) against central differences.
    With the view regulariser the regulariser depends on d, so only the
    u-gradient is exact there (the paper's reason for the layer regulariser)."""
    H, W = 8, 8
    u, d, spec, S = _calib_case()
    lam, eps = 1e-2, 1e-3
    _, gu, gd = O.calib_fit_loss_grad(spec, u, d, H, W, lam, eps, reg, S)
    fu = brute.central_fd(lambda uu: O.calib_fit_loss_grad(spec, uu, d, H, W, lam, eps, reg, S)[0], u)
    np.testing.assert_allclose(gu, fu, rtol=1e-6, atol=1e-9 * np.abs(fu).max())
    if reg == O.REG_LAYER2:
        fd = brute.central_fd(lambda dd: O.calib_fit_loss_grad(spec, u, dd, H, W, lam, eps, reg, S)[0], d)
        np.testing.assert_allclose(gd, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


def test_loo_loss_matches_press_identity():
    H, W = 8, 8
    u, d, spec, S = _calib_case(seed=13, C=2)
    lam, eps = 1e-2, 1e-3
    loss = O.calib_loo_loss(spec, u, d, H, W, lam, eps, O.REG_LAYER2, S)
    wx, wy = O.flat_freqs(H, W)
    RtR = O.second_difference(len(d))
    RtR = RtR.T @ RtR
    m, C = spec.shape[:2]
    tot = 0.0
    for f in S:
        A = _explicit_A(u, d, wx[f], wy[f])
        b = spec.reshape(m, C, -1)[:, :, f] / math.sqrt(H * W)
        tot += np.sum(np.abs(brute.press_residuals(A, b, RtR, lam, eps)) ** 2)
    assert abs(loss - tot) < 1e-10 * abs(loss)


def test_loo_gradient_matches_finite_differences():
    H, W = 8, 8
    u, d, spec, S = _calib_case(seed=14)
    S = S[::3]
    lam, eps = 1e-2, 1e-3
    _, gu, gd = O.calib_loo_loss_grad(spec, u, d, H, W, lam, eps, O.REG_LAYER2, S)
    f = lambda uu, dd: O.calib_loo_loss(spec, uu, dd, H, W, lam, eps, O.REG_LAYER2, S)
    fu = brute.central_fd(lambda uu: f(uu, d), u)
    fd = brute.central_fd(lambda dd: f(u, dd), d)
    np.testing.assert_allclose(gu, fu, rtol=1e-6, atol=1e-9 * np.abs(fu).max())
    np.testing.assert_allclose(gd, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


@pytest.mark.parametrize("mode", [O.LOSS_FIT, O.LOSS_LOO])
def test_gradient_gauge_identity(mode):
    """Any loss of P = u d^T satisfies sum_j <u_j, grad u_j> = sum_k d_k grad d_k
    (scaling u by a and d by 1/a leaves P unchanged)."""
    H, W = 8, 8
    u, d, spec, S = _calib_case(seed=15)
    _, gu, gd = O.calib_loss_grad(spec, u, d, H, W, 1e-2, 1e-3, O.REG_LAYER2, mode, S)
    lhs = np.sum(u * gu)
    rhs = np.sum(d * gd)
    assert abs(lhs - rhs) < 1e-9 * (abs(lhs) + abs(rhs))


def test_gd_step_hand_values():
    u2, d2 = O.gd_step(np.array([[1.0, 0.0]]), np.array([2.0]), np.array([[2.0, 0.0]]), np.array([0.5]),
                       alpha=0.2, eps_g=0.0)
    np.testing.assert_allclose(u2, [[0.9, 0.0]])
    np.testing.assert_allclose(d2, [1.6])


# ------------------------------------------------ aperture-view construction ------

def _aperture_views(rng, m, spread=1.5):
    """Input views with their own apertures: positions, focus, radius, shape."""
    v = np.zeros((m, 5))
    v[:, 0:2] = rng.uniform(-spread, spread, (m, 2))
    v[:, 2] = rng.uniform(-1.5, 1.5, m)
    v[:, 3] = rng.uniform(0.2, 1.2, m)
    v[:, 4] = rng.integers(0, 3, m)
    return v


def test_construct_views_with_pinholes_equals_construct():
    """psi_hat = 1 for every view reduces Eq. AMatGeneral to the sub-aperture case."""
    H, W = 8, 10
    u, d, spec = _tiny_problem(6, H=H, W=W)
    views = np.zeros((u.shape[0], 5))
    views[:, 0:2] = u
    views[:, 3] = np.linspace(0.0, 2.0, u.shape[0])      # radius ignored by a pinhole
    a = O.construct(spec, u, d, H, W, 0.1, 1e-3, O.REG_LAYER2)
    b = O.construct_views(spec, views, d, H, W, 0.1, 1e-3, O.REG_LAYER2)
    np.testing.assert_array_equal(a, b)


def test_construct_views_matches_stacked_least_squares_with_quadrature_apertures():
    """A_jk = exp(2 pi i d_k <u_j, w>) x (aperture transform by midpoint
    quadrature of the unit-integral disk / square), solved as a stacked least
    squares problem, bin by bin (quadrature error ~1e-4 bounds the agreement)."""
    H, W = 6, 6
    rng = np.random.default_rng(21)
    m, n = 5, 3
    views = _aperture_views(rng, m)
    views[:, 4] = [1, 2, 0, 1, 2]
    d = np.array([-1.0, 0.3, 1.1])
    spec = O.rfft2(rng.standard_normal((m, 1, H, W)))
    lam, eps = 0.3, 1e-2
    x = O.construct_views(spec, views, d, H, W, lam, eps, O.REG_L2)
    wx, wy = O.freq_grid(H, W)
    for ky in range(H):
        for kx in range(W // 2 + 1):
            A = np.zeros((m, n), dtype=np.complex128)
            for j in range(m):
                u0, v0, s, rho, shape = views[j]
                for k in range(n):
                    ph = np.exp(2j * math.pi * d[k] * (u0 * wx[ky, kx] + v0 * wy[ky, kx]))
                    ap = 1.0 if shape == 0 else brute.aperture_quadrature(
                        int(shape), rho, (s - d[k]) * wx[ky, kx], (s - d[k]) * wy[ky, kx], N=401)
                    A[j, k] = ph * ap
            ref = brute.stacked_lstsq(A, spec[:, :, ky, kx], np.eye(n), lam, eps)
            np.testing.assert_allclose(x[:, :, ky, kx], ref, rtol=2e-3, atol=2e-3)


def test_construct_views_recovers_layers_from_a_focal_stack():
    """Noise-free wide-aperture view spectra (a focal stack at the centre plus
    four pinholes) rendered from layers whose spectra live where A is well
    conditioned are inverted exactly when lambda, eps -> 0 (rendering is
    pinned separately against the refocus integral; the spectra are used as
    rendered, without the image round trip that would symmetrise the
    self-conjugate bins)."""
    H, W = 16, 16
    d = np.array([-1.0, 0.0, 1.5])
    views = np.array([[0, 0, s, 1.0, 1] for s in (-1.0, 0.0, 1.5)]
                     + [[a, b, 0, 0, 0] for a, b in ((-1, -1), (1, -1), (-1, 1), (1, 1))], dtype=float)
    rng = np.random.default_rng(9)
    wx, wy = O.flat_freqs(H, W)
    A = O.a_matrix_views(views, d, wx, wy)
    cond = np.linalg.cond(A).reshape(H, W // 2 + 1)
    spec = O.rfft2(rng.standard_normal((3, 1, H, W)))
    spec[:, :, cond >= 1e3] = 0.0
    spec = O.rfft2(O.irfft2(spec, H, W))
    assert (cond < 1e3).mean() > 0.5
    inputs = O.render(spec, d, views, H, W)
    x = O.construct_views(inputs, views, d, H, W, 1e-12, 1e-12, O.REG_L2)
    assert O.rel_l2(x, spec) < 1e-7


# ------------------------------------------------ relaxed model (Sec. VIII-B) ------

def _relaxed_case(seed=21, m=5, n=3, H=8, W=8, C=1):
    """A shift matrix that is far from rank 1, plus random input spectra."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(-2.0, 2.0, (m, n, 2))
    spec = O.rfft2(rng.standard_normal((m, C, H, W)))
    F = H * (W // 2 + 1)
    return P, spec, np.arange(1, F)


@pytest.mark.parametrize("reg", [O.REG_LAYER2, O.REG_L2])
def test_relaxed_construct_matches_stacked_least_squares(reg):
    H, W = 8, 8
    P, spec, _ = _relaxed_case(C=2)
    m, n = P.shape[:2]
    lam, eps = 0.2, 1e-2
    x = O.construct_relaxed(spec, P, H, W, lam, eps, reg)
    wx, wy = O.freq_grid(H, W)
    Gam = O.second_difference(n) if reg == O.REG_LAYER2 else np.eye(n)
    for ky in range(H):
        for kx in range(W // 2 + 1):
            A = np.zeros((m, n), dtype=np.complex128)
            for j in range(m):
                for k in range(n):
                    A[j, k] = cmath.exp(2j * math.pi * (P[j, k, 0] * wx[ky, kx] + P[j, k, 1] * wy[ky, kx]))
            ref = brute.stacked_lstsq(A, spec[:, :, ky, kx], Gam, lam, eps)
            np.testing.assert_allclose(x[:, :, ky, kx], ref, rtol=1e-9, atol=1e-9)


def test_relaxed_construct_rejects_the_view_regulariser():
    P, spec, _ = _relaxed_case()
    with pytest.raises(ValueError):
        O.construct_relaxed(spec, P, 8, 8, 0.1, 1e-3, O.REG_VIEW2)


def test_relaxed_render_integer_shifts_is_sum_of_rolls():
    """B_j = sum_k L_k shifted by the integer pair P_jk, done as circular
    shifts of the spatial layers (no Fourier arithmetic)."""
    H, W = 12, 16
    rng = np.random.default_rng(22)
    layers = rng.standard_normal((3, 2, H, W))
    P = rng.integers(-3, 4, (4, 3, 2)).astype(float)
    img = O.irfft2(O.render_relaxed(O.rfft2(layers), P, H, W), H, W)
    ref = np.zeros((4, 2, H, W))
    for j in range(4):
        for k in range(3):
            ref[j] += np.roll(layers[k], (-int(P[j, k, 1]), -int(P[j, k, 0])), axis=(-2, -1))
    np.testing.assert_allclose(img, ref, atol=1e-12)


def test_relaxed_model_data_is_reproduced():
    """Views made by the relaxed model itself (integer shifts, not rank 1):
    the layers built with those shifts and lambda, eps -> 0 render the inputs
    back, while the best rank-1 model of the same size cannot."""
    H, W = 16, 16
    rng = np.random.default_rng(23)
    n = 4
    layers = rng.standard_normal((n, 1, H, W))
    u_int = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    d_int = [-2, -1, 1, 2]
    P = O.shifts_rank1(np.array(u_int, float), np.array(d_int, float))
    P[0, 0] += (1, 0)      # two occlusion-like deviations from P = u d^T
    P[8, 3] += (0, -1)
    views = np.zeros((9, 1, H, W))
    for j in range(9):
        for k in range(n):
            views[j] += np.roll(layers[k], (-int(P[j, k, 1]), -int(P[j, k, 0])), axis=(-2, -1))
    x = O.construct_relaxed(O.rfft2(views), P, H, W, 1e-12, 1e-12, O.REG_L2)
    back = O.irfft2(O.render_relaxed(x, P, H, W), H, W)
    assert O.rel_l2(back, views) < 1e-6
    u = np.array(u_int, float)
    d = np.array(d_int, float)
    x1 = O.construct(O.rfft2(views), u, d, H, W, 1e-12, 1e-12, O.REG_L2)
    rv = np.zeros((9, 5))
    rv[:, :2] = u
    assert O.rel_l2(O.render_images(x1, d, rv, H, W), views) > 1e-2


@pytest.mark.parametrize("mode", [O.LOSS_FIT, O.LOSS_LOO])
def test_relaxed_gradient_of_rank1_shifts_gives_the_calibration_gradient(mode):
    """With P = u d^T the chain rule through P_jk = d_k u_j turns grad P into
    grad u_j = sum_k d_k grad P_jk and grad d_k = sum_j <u_j, grad P_jk>
    (Eqs. gradD, gradP), which must equal the finite-difference-pinned
    calibration gradients."""
    H, W = 8, 8
    rng = np.random.default_rng(24)
    u = rng.uniform(-1.5, 1.5, (5, 2))
    d = np.sort(rng.uniform(-1.5, 1.5, 3))
    spec = O.rfft2(rng.standard_normal((5, 1, H, W)))
    S = np.arange(1, H * (W // 2 + 1), 2)
    lam, eps = 1e-2, 1e-3
    loss, gu, gd = O.calib_loss_grad(spec, u, d, H, W, lam, eps, O.REG_LAYER2, mode, S)
    lossP, gP = O.calib_relaxed_loss_grad(spec, O.shifts_rank1(u, d), H, W, lam, eps, O.REG_LAYER2, mode, S)
    assert abs(loss - lossP) < 1e-12 * abs(loss)
    np.testing.assert_allclose(np.einsum("jkc,k->jc", gP, d), gu, rtol=1e-9, atol=1e-12 * np.abs(gu).max())
    np.testing.assert_allclose(np.einsum("jkc,jc->k", gP, u), gd, rtol=1e-9, atol=1e-12 * np.abs(gd).max())


def test_relaxed_fit_gradient_matches_finite_differences():
    H, W = 8, 8
    P, spec, S = _relaxed_case(seed=25, m=4, n=3)
    lam, eps = 1e-2, 1e-3
    _, g = O.calib_relaxed_fit_loss_grad(spec, P, H, W, lam, eps, O.REG_LAYER2, S)
    fd = brute.central_fd(lambda PP: O.calib_relaxed_fit_loss_grad(spec, PP, H, W, lam, eps, O.REG_LAYER2, S)[0], P)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


def test_relaxed_loo_gradient_matches_finite_differences():
    H, W = 8, 8
    P, spec, S = _relaxed_case(seed=26, m=4, n=2)
    S = S[::3]
    lam, eps = 1e-2, 1e-3
    _, g = O.calib_relaxed_loo_loss_grad(spec, P, H, W, lam, eps, O.REG_L2, S)

    def loo(PP):
        # the leave-one-out loss straight from its definition: one refit per left-out view
        wx, wy = O.flat_freqs(H, W)
        m, C = spec.shape[:2]
        tot = 0.0
        for f in S:
            A = O.a_matrix_shifts(PP, wx[f:f + 1], wy[f:f + 1])[0]
            b = spec.reshape(m, C, -1)[:, :, f] / math.sqrt(H * W)
            tot += np.sum(np.abs(brute.press_residuals(A, b, np.eye(PP.shape[1]), lam, eps)) ** 2)
        return tot

    fd = brute.central_fd(loo, P)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


def test_relaxed_gd_step_hand_values():
    P2 = O.gd_step_relaxed(np.array([[[1.0, 0.0]], [[0.0, 1.0]]]), np.array([[[2.0, 0.0]], [[0.0, 0.0]]]),
                           alpha=0.2, eps_g=0.0)
    np.testing.assert_allclose(P2, [[[0.9, 0.0]], [[0.0, 1.0]]])


# ------------------------------------------------ drawn apertures (Sec. VI) ------

def _drawn_disk(S):
    c = (np.arange(S) - (S - 1) / 2) * (2.0 / S)
    return ((c[None, :] ** 2 + c[:, None] ** 2) <= 1.0).astype(float)


def test_aperture_table_matches_direct_sum():
    """Every table entry is the Fourier sum of the unit-sum image over its
    pixel centres (p - (S-1)/2) 2/S at xi = k S/(2N); the entry at k also
    stands for k - N (periodic samples)."""
    rng = np.random.default_rng(31)
    S, pad = 5, 3
    img = rng.uniform(0, 1, (S, S))
    T = O.aperture_table(img, pad)
    N = S * pad
    w = img / img.sum()
    c = (np.arange(S) - (S - 1) / 2) * (2.0 / S)
    for ky in range(N):
        for kx in range(N):
            for sx, sy in ((0, 0), (-N, 0), (0, -N), (-N, -N)):
                xx = (kx + sx) * S / (2 * N)
                xy = (ky + sy) * S / (2 * N)
                ref = sum(w[py, px] * cmath.exp(-2j * math.pi * (c[px] * xx + c[py] * xy))
                          for py in range(S) for px in range(S))
                assert abs(T[ky, kx] - ref) < 1e-12


def test_table_interpolation_nodes_zero_radius_and_midpoints():
    rng = np.random.default_rng(32)
    S, pad = 7, 2
    T = O.aperture_table(rng.uniform(0, 1, (S, S)), pad)
    N = S * pad
    step = S / (2 * N)                                   # xi between samples (rho = 1)
    k = np.array([0, 3, 9, N - 1, -2])
    got = O.psi_hat_table(T, S, 1.0, k * step, 2 * k * step)
    np.testing.assert_allclose(got, T[(2 * k) % N, k % N], atol=1e-13)
    assert np.all(O.psi_hat_table(T, S, 0.0, np.array([0.3, -2.0]), np.array([1.0, 0.5])) == T[0, 0])
    assert abs(T[0, 0] - 1.0) < 1e-15
    mid = O.psi_hat_table(T, S, 1.0, np.array([2.5 * step]), np.array([4.5 * step]))[0]
    assert abs(mid - 0.25 * (T[4, 2] + T[4, 3] + T[5, 2] + T[5, 3])) < 1e-14


def test_drawn_full_square_samples_are_the_dirichlet_kernel_near_the_sinc():
    """A full image is a sampled square of half-side 1: its spectrum samples
    are products of Dirichlet kernels sin(2 pi xi) / (S sin(2 pi xi / S))
    (closed form of the geometric series), within (2 pi xi / S)^2 / 6 of the
    analytic sinc(2 xi) of the square aperture."""
    S, pad = 31, 4
    T = O.aperture_table(np.ones((S, S)), pad)
    N = S * pad
    k = np.arange(-N // 2, N // 2)
    xi = k * S / (2 * N)
    with np.errstate(invalid="ignore", divide="ignore"):
        dk = np.where(k == 0, 1.0, np.sin(2 * math.pi * xi) / (S * np.sin(2 * math.pi * xi / S)))
    np.testing.assert_allclose(T[0, k % N], dk, atol=1e-12)
    np.testing.assert_allclose(T[k % N, 0], dk, atol=1e-12)
    np.testing.assert_allclose(T[np.ix_(k % N, k % N)], np.outer(dk, dk), atol=1e-12)
    small = np.abs(xi) <= 2.0
    bound = (2 * math.pi * xi[small] / S) ** 2 / 6 + 1e-12
    assert np.all(np.abs(dk[small] - np.sinc(2 * xi[small])) <= bound)


def test_drawn_disk_render_approaches_the_analytic_disk():
    """Rendering with an inscribed drawn disk converges to the analytic disk
    aperture as the drawing gets finer and the padding larger."""
    H, W = 16, 16
    rng = np.random.default_rng(33)
    layers = O.rfft2(rng.standard_normal((3, 1, H, W)))
    d = np.array([-1.0, 0.0, 1.5])
    views = np.array([[0.5, -0.5, 0.3, 1.2, O.AP_DISK], [0.0, 1.0, -0.8, 2.0, O.AP_DISK]])
    ref = O.render(layers, d, views, H, W)
    errs = []
    for S, pad in ((15, 2), (63, 4), (127, 16)):
        T = O.aperture_table(_drawn_disk(S), pad)
        v = views.copy()
        v[:, 4] = O.AP_IMAGE
        errs.append(O.rel_l2(O.render_tabulated(layers, d, v, H, W, T, S), ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 3e-3


def test_render_tabulated_without_image_views_is_render():
    H, W = 12, 12
    rng = np.random.default_rng(34)
    layers = O.rfft2(rng.standard_normal((2, 2, H, W)))
    d = np.array([-0.5, 1.0])
    views = np.array([[0.5, 0.0, 0.3, 1.0, O.AP_DISK], [1.0, -1.0, 0.0, 0.7, O.AP_SQUARE], [0, 0, 0, 0, 0]])
    T = O.aperture_table(np.ones((5, 5)), 2)
    np.testing.assert_allclose(O.render_tabulated(layers, d, views, H, W, T, 5), O.render(layers, d, views, H, W),
                               atol=1e-12)


# ------------------------------------- finite-region view regulariser (Eq. GTG) ------

def test_region_regulariser_matches_quadrature_of_its_integral():
    """Eq. GTG written as an integral over the square [-r/2, r/2]^2 of
    Gamma_k1(u) conj(Gamma_k2(u)), Gamma_k(u) = |w|^2 d_k^2 exp(2 pi i d_k <u, w>),
    divided by r^2, by the midpoint rule on a fine grid."""
    d = np.array([-1.3, -0.2, 0.4, 1.7])
    wx = np.array([0.11, -0.31, 0.05])
    wy = np.array([-0.07, 0.22, 0.0])
    r = 3.0
    R = O.reg_matrix(O.REG_VIEW2_REGION, d, wx, wy, r)
    N = 400
    t = (np.arange(N) + 0.5) / N * r - r / 2
    uu, vv = np.meshgrid(t, t, indexing="xy")
    for f in range(3):
        w2 = wx[f] ** 2 + wy[f] ** 2
        G = np.stack([w2 * dk ** 2 * np.exp(2j * math.pi * dk * (uu * wx[f] + vv * wy[f])) for dk in d])
        Q = np.einsum("kab,lab->kl", G, np.conj(G)) * (r / N) ** 2 / r ** 2
        np.testing.assert_allclose(R[f], Q, rtol=0, atol=1e-5 * np.abs(Q).max())


def test_region_regulariser_tends_to_the_view_regulariser():
    """r -> infinity: the off-diagonal sinc products vanish (as 1/(pi r dd w)^2
    at most) and the diagonal is diag(|w|^4 d^4) for every r."""
    rng = np.random.default_rng(35)
    d = np.sort(rng.uniform(-2, 2, 6))
    wx = rng.uniform(-0.5, 0.5, 10)
    wy = rng.uniform(-0.5, 0.5, 10)
    V = O.reg_matrix(O.REG_VIEW2, d, wx, wy)
    for r in (10.0, 1e3, 1e5):
        R = O.reg_matrix(O.REG_VIEW2_REGION, d, wx, wy, r)
        idx = np.arange(6)
        np.testing.assert_allclose(R[:, idx, idx], V[:, idx, idx], rtol=1e-14)
        dd = np.abs(d[:, None] - d[None, :]) + np.eye(6)
        bound = 1.0 / (math.pi * r * dd[None] * np.abs(wx)[:, None, None]) / (math.pi * r * dd[None] *
                                                                              np.abs(wy)[:, None, None])
        off = np.abs(R - V)
        assert np.all(off <= bound * np.abs(V).max() + 1e-300)


def test_region_regulariser_is_positive_semidefinite_and_construct_uses_it():
    rng = np.random.default_rng(36)
    d = np.sort(rng.uniform(-2, 2, 7))
    wx = rng.uniform(-0.5, 0.5, 20)
    wy = rng.uniform(-0.5, 0.5, 20)
    R = O.reg_matrix(O.REG_VIEW2_REGION, d, wx, wy, 2.5)
    ev = np.linalg.eigvalsh(R)
    assert ev.min() >= -1e-12 * ev.max()
    H, W = 8, 8
    u, d2, spec = _tiny_problem(5, H=H, W=W)
    lam, eps = 0.4, 1e-2
    x = O.construct(spec, u, d2, H, W, lam, eps, O.REG_VIEW2_REGION, region=2.0)
    wgx, wgy = O.freq_grid(H, W)
    for ky in range(H):
        for kx in range(W // 2 + 1):
            A = _explicit_A(u, d2, wgx[ky, kx], wgy[ky, kx])
            Rk = O.reg_matrix(O.REG_VIEW2_REGION, d2, np.array([wgx[ky, kx]]), np.array([wgy[ky, kx]]), 2.0)[0]
            # a square root of the (semi-definite) regulariser as the stacked rows
            lam_k, U = np.linalg.eigh(Rk)
            Gam = (U * np.sqrt(np.clip(lam_k, 0, None))).T
            ref = brute.stacked_lstsq(A, spec[:, :, ky, kx], Gam, lam, eps)
            np.testing.assert_allclose(x[:, :, ky, kx], ref, rtol=1e-8, atol=1e-9)
