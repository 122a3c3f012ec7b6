"""Plain FP64 CPU oracle for the Fourier Disparity Layer (FDL) hot path.

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU library.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path never does.  It shares no code
with the HIP library or its Python binding.

Everything is numpy float64 / complex128, written for clarity, not speed:
each step follows the paper's definitions (Le Pendu, Guillemot, Smolic,
"A Fourier Disparity Layer representation for Light Fields").  Library
primitives used as steps: numpy.fft (2D DFT), numpy.linalg.solve (dense
solve), scipy.special.j1 (Bessel J1) and torch autograd (derivative of the
leave-one-out loss).

Array conventions
-----------------
* images ``[..., H, W]`` real; spectra ``[..., H, W//2+1]`` complex, the
  unnormalised forward DFT ``sum_x img(x) exp(-2 pi i <x, w>)`` restricted to
  the Hermitian half (Sec. VII, Complexity).
* frequencies in cycles/pixel: w_x = rfftfreq(W) (columns, Nyquist +0.5),
  w_y = fftfreq(H) (rows, Nyquist -0.5).
* view position ``u[j] = (u, v)`` (horizontal, vertical), disparities ``d[k]``
  in pixels per unit of position, p_j(w) = u_j,x w_x + u_j,y w_y.
* A_jk(w) = exp(+2 pi i d_k p_j(w))   (Eq. AMatGeneral with psi_j = delta;
  the 2D form replaces u w by the inner product <u, w>, Sec. III).

Readings of the paper used here (each stated where it is used):
* R1  eps is added to the normal matrix as eps*I outside lambda (Sec. V-C-1,
      the remark after Eq. 2ndOrderView: "equivalent to an l2 term").
* R2  2D second-order view regulariser: diag(|w|^4 d_k^4) (Eq. 2ndOrderView).
* R3  apertures have unit integral, so psi_hat(0) = 1; disk of radius rho,
      square of half-side rho, rho = 0 is a pinhole (Sec. VI, scale factor f).
* R4  calibration loss uses orthonormal spectra (DFT / sqrt(HW)) and, as in
      Eq. CalibrationProb, the SUM over the sampled frequencies (the
      stochastic subset replaces the full sum); the update uses ||grad||^2
      as printed.
* R5  relaxed model (Sec. VIII-B): in 2D the shift of layer k in view j is a
      pair P_jk = (P^x_jk, P^y_jk), rank-1 case P_jk = d_k u_j; the phase is
      <P_jk, w>; grad P^x = sum_q G_jk w_x, grad P^y = sum_q G_jk w_y (Eq. gradP
      with both components); the update normalises by the squared norm over all
      2mn entries; the regulariser must not depend on d (LAYER2 or L2).
* R7  second-order view regulariser over a finite camera-plane region
      (Eq. GTG): in 2D the region is the square [-r/2, r/2]^2 and the
      derivative functional is |w|^2 d_k^2 exp(2 pi i d_k <u, w>) (reading R2),
      so after division by the area r^2 the matrix is
      |w|^4 d_k1^2 d_k2^2 sinc(r (d_k1 - d_k2) w_x) sinc(r (d_k1 - d_k2) w_y),
      whose r -> infinity limit is the diagonal of REG_VIEW2.
* R6  drawn apertures (Sec. VI): an S x S image (S odd) tiles the box
      [-1, 1]^2 of the aperture's own coordinates with cells of side 2/S,
      pixel p centred at (p - (S-1)/2) 2/S (a symmetric grid), normalised to
      unit sum; its spectrum is taken from the DFT of the image zero-padded
      to N = pad S, i.e. at xi = k S / (2N) = k / (2 pad), k in [0, N) (the
      samples are N-periodic because S - 1 is even), and read between samples
      by bilinear interpolation with periodic wrap; a view's radius rho
      scales the box, psi_hat_rho(xi) = psi_hat_1(rho xi), as the paper's
      factor f does (a full image is the square of half-side rho, an
      inscribed disk the disk of radius rho).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
from scipy.special import j1 as _bessel_j1

REG_VIEW2 = 0
REG_LAYER2 = 1
REG_L2 = 2
REG_VIEW2_REGION = 3

AP_PINHOLE = 0
AP_DISK = 1
AP_SQUARE = 2
AP_IMAGE = 3

LOSS_FIT = 0
LOSS_LOO = 1


# ---------------------------------------------------------------------------
# Spectra and frequency grid (Sec. V-A: DFT of each image; Sec. VII: half
# spectrum by Hermitian symmetry)
# ---------------------------------------------------------------------------

def rfft2(img: np.ndarray) -> np.ndarray:
    """Unnormalised forward 2D DFT of real images over the last two axes,
    half spectrum [..., H, W//2+1], complex128."""
    return np.fft.rfft2(np.asarray(img, dtype=np.float64), axes=(-2, -1))


def irfft2(spec: np.ndarray, H: int, W: int) -> np.ndarray:
    """Inverse of :func:`rfft2` with 1/(HW) normalisation.  The half spectrum
    is extended by Hermitian symmetry; imaginary parts of self-conjugate bins
    (DC and Nyquist rows/columns) do not contribute."""
    return np.fft.irfft2(np.asarray(spec, dtype=np.complex128), s=(H, W), axes=(-2, -1))


def freq_grid(H: int, W: int):
    """(w_x, w_y) broadcast to [H, W//2+1], cycles/pixel."""
    wx = np.fft.rfftfreq(W)[None, :]
    wy = np.fft.fftfreq(H)[:, None]
    Wh = W // 2 + 1
    return np.broadcast_to(wx, (H, Wh)).astype(np.float64), np.broadcast_to(wy, (H, Wh)).astype(np.float64)


def flat_freqs(H: int, W: int):
    """Flattened (w_x, w_y), bin f = ky*(W//2+1) + kx."""
    wx, wy = freq_grid(H, W)
    return wx.ravel().copy(), wy.ravel().copy()


# ---------------------------------------------------------------------------
# The matrix A and the regularisers (Sec. V-A, V-C)
# ---------------------------------------------------------------------------

def a_matrix(u: np.ndarray, d: np.ndarray, wx: np.ndarray, wy: np.ndarray) -> np.ndarray:
    """A[f, j, k] = exp(+2 pi i d_k <u_j, w_f>)  (Eq. AMatGeneral, sub-aperture
    inputs, generalised to 2D).  u: [m,2], d: [n], wx, wy: [F]."""
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    p = wx[:, None] * u[None, :, 0] + wy[:, None] * u[None, :, 1]          # [F, m]
    return np.exp(2j * math.pi * p[:, :, None] * d[None, None, :])          # [F, m, n]


def second_difference(n: int) -> np.ndarray:
    """Gamma = tridiag(1, -2, 1), n x n (Eq. 2ndOrderLayer)."""
    G = -2.0 * np.eye(n)
    if n > 1:
        G += np.eye(n, k=1) + np.eye(n, k=-1)
    return G


def reg_matrix(reg: int, d: np.ndarray, wx: np.ndarray, wy: np.ndarray, r: Optional[float] = None) -> np.ndarray:
    """Gamma^H Gamma per frequency, [F, n, n] (real).

    REG_VIEW2:  diag(|w|^4 d_k^4)  -- Eq. 2ndOrderView, the r -> infinity limit
                of Eq. GTG, with w^4 read as (w_x^2 + w_y^2)^2 in 2D (R2).
    REG_LAYER2: Gamma^T Gamma with Gamma = tridiag(1,-2,1) (Eq. 2ndOrderLayer).
    REG_L2:     identity (Sec. V-C, classical l2).
    REG_VIEW2_REGION: Eq. GTG over the camera-plane square of side r, divided
                by its area (R7); dense, real, positive semi-definite.
    """
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    F = wx.shape[0]
    if reg == REG_VIEW2:
        w4 = (wx * wx + wy * wy) ** 2                                       # [F]
        R = np.zeros((F, n, n))
        idx = np.arange(n)
        R[:, idx, idx] = w4[:, None] * (d ** 4)[None, :]
        return R
    if reg == REG_LAYER2:
        G = second_difference(n)
        return np.broadcast_to(G.T @ G, (F, n, n)).copy()
    if reg == REG_L2:
        return np.broadcast_to(np.eye(n), (F, n, n)).copy()
    if reg == REG_VIEW2_REGION:
        # Eq. GTG divided by the region's area (R7); r is the side of the region
        if r is None or not r > 0:
            raise ValueError("REG_VIEW2_REGION needs the region side r > 0")
        w4 = (wx * wx + wy * wy) ** 2
        dd = d[:, None] - d[None, :]                                       # [n, n]
        sx = np.sinc(r * dd[None] * wx[:, None, None])
        sy = np.sinc(r * dd[None] * wy[:, None, None])
        return w4[:, None, None] * (d * d)[None, :, None] * (d * d)[None, None, :] * sx * sy
    raise ValueError(f"unknown regulariser {reg}")


def normal_matrix(A: np.ndarray, R: np.ndarray, lam: float, eps: float) -> np.ndarray:
    """M = A^H A + lam Gamma^H Gamma + eps I  (Eq. LayerConstructionClosedForm
    plus the eps term of reading R1)."""
    n = A.shape[-1]
    AhA = np.conj(np.swapaxes(A, -1, -2)) @ A
    return AhA + lam * R + eps * np.eye(n)[None, :, :]


# ---------------------------------------------------------------------------
# Layer construction (Sec. V-A, Eq. LayerConstructionClosedForm)
# ---------------------------------------------------------------------------

def construct(view_spec: np.ndarray, u: np.ndarray, d: np.ndarray, H: int, W: int,
              lam: float, eps: float, reg: int = REG_VIEW2,
              freq_index: Optional[np.ndarray] = None, chunk: int = 2048,
              region: Optional[float] = None) -> np.ndarray:
    """Closed-form Tikhonov solution x(w) = (A^H A + lam G + eps I)^-1 A^H b(w)
    at every half-spectrum bin, independently per bin and shared across colour
    channels.

    view_spec: [m, C, H, W//2+1] complex spectra of the input views.
    Returns layer spectra [n, C, H, W//2+1] complex128, or, when
    ``freq_index`` (flat bin indices) is given, [n, C, len(freq_index)].
    ``region`` is the side r of the camera-plane square of REG_VIEW2_REGION.
    """
    view_spec = np.asarray(view_spec)
    m, C = view_spec.shape[:2]
    n = len(d)
    wx_all, wy_all = flat_freqs(H, W)
    b_all = view_spec.reshape(m, C, -1)
    if freq_index is None:
        freq_index = np.arange(wx_all.shape[0])
    freq_index = np.asarray(freq_index, dtype=np.int64)
    out = np.zeros((n, C, freq_index.shape[0]), dtype=np.complex128)
    for s in range(0, freq_index.shape[0], chunk):
        fi = freq_index[s:s + chunk]
        wx, wy = wx_all[fi], wy_all[fi]
        A = a_matrix(u, d, wx, wy)                                         # [F, m, n]
        M = normal_matrix(A, reg_matrix(reg, d, wx, wy, region), lam, eps)  # [F, n, n]
        b = np.transpose(b_all[:, :, fi], (2, 0, 1)).astype(np.complex128)  # [F, m, C]
        c = np.conj(np.swapaxes(A, -1, -2)) @ b                           # [F, n, C]
        x = np.linalg.solve(M, c)                                          # [F, n, C]
        out[:, :, s:s + chunk] = np.transpose(x, (1, 2, 0))
    if freq_index.shape[0] == wx_all.shape[0] and np.array_equal(freq_index, np.arange(wx_all.shape[0])):
        return out.reshape(n, C, H, W // 2 + 1)
    return out


# ---------------------------------------------------------------------------
# Aperture spectra and rendering (Sec. IV-B Eq. BsFourier, Sec. VI)
# ---------------------------------------------------------------------------

def psi_hat(shape: int, rho: float, xi_x: np.ndarray, xi_y: np.ndarray) -> np.ndarray:
    """Fourier transform of a unit-integral aperture at frequency xi (R3).

    pinhole: 1 (psi = delta).
    disk of radius rho: 2 J1(z)/z, z = 2 pi rho |xi|.
    square of half-side rho: sinc(2 rho xi_x) sinc(2 rho xi_y), sinc(t) = sin(pi t)/(pi t).
    """
    xi_x = np.asarray(xi_x, dtype=np.float64)
    xi_y = np.asarray(xi_y, dtype=np.float64)
    if shape == AP_PINHOLE or rho == 0.0:
        return np.ones(np.broadcast(xi_x, xi_y).shape)
    if shape == AP_DISK:
        z = 2.0 * math.pi * rho * np.sqrt(xi_x * xi_x + xi_y * xi_y)
        out = np.ones_like(z)
        nz = z != 0.0
        out[nz] = 2.0 * _bessel_j1(z[nz]) / z[nz]
        return out
    if shape == AP_SQUARE:
        return np.sinc(2.0 * rho * xi_x) * np.sinc(2.0 * rho * xi_y)
    raise ValueError(f"unknown aperture shape {shape}")


def render(layer_spec: np.ndarray, d: np.ndarray, views: np.ndarray, H: int, W: int) -> np.ndarray:
    """B_v(w) = sum_k exp(+2 pi i d_k <u0_v, w>) psi_hat_v((s_v - d_k) w) L_k(w)
    (Eq. BsFourier, 2D).  views: [V, 5] rows (u, v, focus s, radius rho, shape).
    layer_spec: [n, C, H, W//2+1].  Returns [V, C, H, W//2+1] complex128."""
    layer_spec = np.asarray(layer_spec)
    n, C = layer_spec.shape[:2]
    d = np.asarray(d, dtype=np.float64)
    views = np.asarray(views, dtype=np.float64).reshape(-1, 5)
    wx, wy = freq_grid(H, W)
    out = np.zeros((views.shape[0], C) + wx.shape, dtype=np.complex128)
    for v, (u0, v0, s, rho, shape) in enumerate(views):
        acc = np.zeros((C,) + wx.shape, dtype=np.complex128)
        for k in range(n):
            phase = np.exp(2j * math.pi * d[k] * (u0 * wx + v0 * wy))
            filt = psi_hat(int(round(shape)), rho, (s - d[k]) * wx, (s - d[k]) * wy)
            acc += (phase * filt)[None, :, :] * layer_spec[k]
        out[v] = acc
    return out


def render_images(layer_spec: np.ndarray, d: np.ndarray, views: np.ndarray, H: int, W: int) -> np.ndarray:
    """Rendered images [V, C, H, W]: :func:`render` followed by the inverse DFT."""
    return irfft2(render(layer_spec, d, views, H, W), H, W)


def a_matrix_views(views: np.ndarray, d: np.ndarray, wx: np.ndarray, wy: np.ndarray) -> np.ndarray:
    """Eq. AMatGeneral with an aperture per input view:
    A_jk(w) = exp(+2 pi i d_k <u_j, w>) psi_hat_j((s_j - d_k) w), views [m, 5]
    rows (u, v, focus s, radius rho, shape) as for :func:`render` (the input
    view j is the rendering of the layers with its own aperture and focus).
    wx, wy are the bins' frequencies ([F]); returns [F, m, n] complex128."""
    views = np.asarray(views, dtype=np.float64).reshape(-1, 5)
    d = np.asarray(d, dtype=np.float64)
    A = a_matrix(views[:, 0:2], d, wx, wy)
    for j, (_, _, s, rho, shape) in enumerate(views):
        for k in range(d.shape[0]):
            A[:, j, k] *= psi_hat(int(round(shape)), rho, (s - d[k]) * wx, (s - d[k]) * wy)
    return A


def construct_views(view_spec: np.ndarray, views: np.ndarray, d: np.ndarray, H: int, W: int,
                    lam: float, eps: float, reg: int = REG_VIEW2,
                    freq_index: Optional[np.ndarray] = None, chunk: int = 2048) -> np.ndarray:
    """Layer construction from input views taken with their own apertures
    (focal stacks, wide-aperture or mixed inputs; Eq. AMatGeneral, Sec. V-A):
    the closed form of :func:`construct` with A from :func:`a_matrix_views`.
    Returns layer spectra [n, C, H, W//2+1] complex128, or [n, C, len(freq_index)]."""
    view_spec = np.asarray(view_spec)
    m, C = view_spec.shape[:2]
    n = len(d)
    wx_all, wy_all = flat_freqs(H, W)
    b_all = view_spec.reshape(m, C, -1)
    if freq_index is None:
        freq_index = np.arange(wx_all.shape[0])
    freq_index = np.asarray(freq_index, dtype=np.int64)
    out = np.zeros((n, C, freq_index.shape[0]), dtype=np.complex128)
    for s in range(0, freq_index.shape[0], chunk):
        fi = freq_index[s:s + chunk]
        wx, wy = wx_all[fi], wy_all[fi]
        A = a_matrix_views(views, d, wx, wy)
        M = normal_matrix(A, reg_matrix(reg, d, wx, wy), lam, eps)
        b = np.transpose(b_all[:, :, fi], (2, 0, 1)).astype(np.complex128)
        c = np.conj(np.swapaxes(A, -1, -2)) @ b
        x = np.linalg.solve(M, c)
        out[:, :, s:s + chunk] = np.transpose(x, (1, 2, 0))
    if freq_index.shape[0] == wx_all.shape[0] and np.array_equal(freq_index, np.arange(wx_all.shape[0])):
        return out.reshape(n, C, H, W // 2 + 1)
    return out


def forward_views(layers: np.ndarray, u: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Sub-aperture views of a layer stack (Eq. FourierView): the spectra of
    the spatial layers [n, C, H, W] phase-shifted to each position u_j and
    summed.  Returns views [m, C, H, W] float64."""
    n, C, H, W = layers.shape
    views = np.zeros((u.shape[0], 5))
    views[:, 0:2] = u
    return render_images(rfft2(layers), d, views, H, W)


# ---------------------------------------------------------------------------
# Calibration (Sec. V-B, Eqs. CalibrationProb, gradD, gradP and the update)
# ---------------------------------------------------------------------------

def _calib_system(view_spec, u, d, H, W, lam, eps, reg, freq_index):
    m, C = view_spec.shape[:2]
    wx_all, wy_all = flat_freqs(H, W)
    fi = np.asarray(freq_index, dtype=np.int64)
    wx, wy = wx_all[fi], wy_all[fi]
    b = np.transpose(view_spec.reshape(m, C, -1)[:, :, fi], (2, 0, 1)).astype(np.complex128)
    b = b / math.sqrt(H * W)                       # orthonormal spectra (R4)
    R = reg_matrix(reg, d, wx, wy)
    return wx, wy, b, R


def calib_fit_loss_grad(view_spec: np.ndarray, u: np.ndarray, d: np.ndarray, H: int, W: int,
                        lam: float, eps: float, reg: int, freq_index: np.ndarray):
    """Paper-mode calibration objective and its gradient.

    E(u, d) = sum_{q in S} min_x ||A_q x - b_q||^2 + lam ||Gamma x||^2 + eps ||x||^2
    (Eq. CalibrationProb with R1, R4).  With x_q at the minimum, the gradient
    is that of the data term alone (the regulariser does not depend on u, d):
    G_jk(q) = 4 pi Im( conj(x_k) conj(A_jk) r_j ),  r = A x - b   (Eq. gradP),
    grad u_j = sum_q sum_k d_k G_jk(q) w_q          (2-vector, Eq. gradD generalised),
    grad d_k = sum_q sum_j G_jk(q) <u_j, w_q>.
    Returns (loss, grad_u [m,2], grad_d [n]) as float64.
    """
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    wx, wy, b, R = _calib_system(view_spec, u, d, H, W, lam, eps, reg, freq_index)
    Q = wx.shape[0]
    A = a_matrix(u, d, wx, wy)                                             # [Q, m, n]
    M = normal_matrix(A, R, lam, eps)
    Ah = np.conj(np.swapaxes(A, -1, -2))
    x = np.linalg.solve(M, Ah @ b)                                         # [Q, n, C]
    r = A @ x - b                                                          # [Q, m, C]
    n = d.shape[0]
    Rfull = lam * R + eps * np.eye(n)[None]
    loss = (np.sum(np.abs(r) ** 2)
            + np.real(np.einsum("qkc,qkl,qlc->", np.conj(x), Rfull, x)))
    # G[q, j, k] = 4 pi Im( sum_c conj(x_kc) conj(A_jk) r_jc )
    G = 4.0 * math.pi * np.imag(np.conj(A) * np.einsum("qkc,qjc->qjk", np.conj(x), r))
    grad_u = np.zeros((u.shape[0], 2))
    grad_u[:, 0] = np.einsum("qjk,k,q->j", G, d, wx)
    grad_u[:, 1] = np.einsum("qjk,k,q->j", G, d, wy)
    p = wx[:, None] * u[None, :, 0] + wy[:, None] * u[None, :, 1]          # [Q, m]
    grad_d = np.einsum("qjk,qj->k", G, p)
    return float(loss), grad_u, grad_d


def calib_loo_loss(view_spec: np.ndarray, u: np.ndarray, d: np.ndarray, H: int, W: int,
                   lam: float, eps: float, reg: int, freq_index: np.ndarray) -> float:
    """Leave-one-out view-prediction loss, straight from its definition:
    E = sum_{q in S} sum_j sum_c | b_jc - a_j x^(-j)_c |^2, where x^(-j)
    solves the same regularised problem (Eq. LayerConstructProb) with view j
    removed.  One explicit refit per view and frequency."""
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    wx, wy, b, R = _calib_system(view_spec, u, d, H, W, lam, eps, reg, freq_index)
    Q = wx.shape[0]
    A = a_matrix(u, d, wx, wy)
    m, n = A.shape[1], A.shape[2]
    total = 0.0
    for j in range(m):
        keep = np.arange(m) != j
        Aj = A[:, keep, :]
        M = normal_matrix(Aj, R, lam, eps)
        x = np.linalg.solve(M, np.conj(np.swapaxes(Aj, -1, -2)) @ b[:, keep, :])
        pred = np.einsum("qk,qkc->qc", A[:, j, :], x)
        total += np.sum(np.abs(b[:, j, :] - pred) ** 2)
    return float(total)


def calib_loo_loss_grad(view_spec: np.ndarray, u: np.ndarray, d: np.ndarray, H: int, W: int,
                        lam: float, eps: float, reg: int, freq_index: np.ndarray):
    """LOO loss and its exact gradient with respect to u and d.

    The loss is :func:`calib_loo_loss` (explicit refits); the derivative is
    taken by reverse-mode automatic differentiation of that same computation
    in complex128 (torch autograd, CPU) -- no hand-derived adjoint here.
    Returns (loss, grad_u [m,2], grad_d [n]) as float64."""
    import torch

    wx_np, wy_np, b_np, R_np = _calib_system(view_spec, u, d, H, W, lam, eps, reg, freq_index)
    Q = wx_np.shape[0]
    tu = torch.tensor(np.asarray(u, dtype=np.float64), requires_grad=True)
    td = torch.tensor(np.asarray(d, dtype=np.float64), requires_grad=True)
    wx = torch.tensor(wx_np)
    wy = torch.tensor(wy_np)
    b = torch.tensor(b_np)
    R = torch.tensor(R_np, dtype=torch.complex128)
    m = tu.shape[0]
    n = td.shape[0]
    p = wx[:, None] * tu[None, :, 0] + wy[:, None] * tu[None, :, 1]
    A = torch.exp(2j * math.pi * (p[:, :, None] * td[None, None, :]).to(torch.complex128))
    eye = torch.eye(n, dtype=torch.complex128)
    total = torch.zeros((), dtype=torch.float64)
    for j in range(m):
        keep = [i for i in range(m) if i != j]
        Aj = A[:, keep, :]
        Ajh = Aj.conj().transpose(-1, -2)
        M = Ajh @ Aj + lam * R + eps * eye
        x = torch.linalg.solve(M, Ajh @ b[:, keep, :])
        pred = torch.einsum("qk,qkc->qc", A[:, j, :], x)
        total = total + torch.sum(torch.abs(b[:, j, :] - pred) ** 2)
    loss = total
    loss.backward()
    return float(loss.detach()), tu.grad.numpy().copy(), td.grad.numpy().copy()


def calib_loss_grad(view_spec, u, d, H, W, lam, eps, reg, mode, freq_index):
    """Dispatch on the loss mode (LOSS_FIT: Eq. CalibrationProb; LOSS_LOO)."""
    if mode == LOSS_FIT:
        return calib_fit_loss_grad(view_spec, u, d, H, W, lam, eps, reg, freq_index)
    if mode == LOSS_LOO:
        return calib_loo_loss_grad(view_spec, u, d, H, W, lam, eps, reg, freq_index)
    raise ValueError(f"unknown loss mode {mode}")


def gd_step(u: np.ndarray, d: np.ndarray, grad_u: np.ndarray, grad_d: np.ndarray,
            alpha: float = 0.2, eps_g: float = 1e-6):
    """u' = u - alpha grad_u / (eps + ||grad_u||_2^2), same for d (the update
    of Sec. V-B, squared norm as printed, alpha = 0.2)."""
    gu = np.asarray(grad_u, dtype=np.float64)
    gd = np.asarray(grad_d, dtype=np.float64)
    u2 = np.asarray(u, dtype=np.float64) - alpha * gu / (eps_g + np.sum(gu * gu))
    d2 = np.asarray(d, dtype=np.float64) - alpha * gd / (eps_g + np.sum(gd * gd))
    return u2, d2


# ---------------------------------------------------------------------------
# Relaxed FDL model (Sec. VIII-B, denoising): a free shift for every pair of
# input view and layer instead of the rank-1 product d_k u_j (reading R5)
# ---------------------------------------------------------------------------

def shifts_rank1(u: np.ndarray, d: np.ndarray) -> np.ndarray:
    """P[j, k] = d_k u_j, the rank-1 shift matrix of the unrelaxed model,
    [m, n, 2] float64 (last axis: horizontal, vertical)."""
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    return d[None, :, None] * u[:, None, :]


def a_matrix_shifts(shifts: np.ndarray, wx: np.ndarray, wy: np.ndarray) -> np.ndarray:
    """A[f, j, k] = exp(+2 pi i <P_jk, w_f>) for a free shift matrix
    P [m, n, 2]; with P = :func:`shifts_rank1` this is :func:`a_matrix`."""
    P = np.asarray(shifts, dtype=np.float64)
    t = wx[:, None, None] * P[None, :, :, 0] + wy[:, None, None] * P[None, :, :, 1]
    return np.exp(2j * math.pi * t)


def _check_relaxed_reg(reg: int) -> None:
    if reg not in (REG_LAYER2, REG_L2):
        raise ValueError("the relaxed model has no layer disparities: use REG_LAYER2 or REG_L2")


def construct_relaxed(view_spec: np.ndarray, shifts: np.ndarray, H: int, W: int,
                      lam: float, eps: float, reg: int = REG_LAYER2,
                      freq_index: Optional[np.ndarray] = None, chunk: int = 2048) -> np.ndarray:
    """Layers of the relaxed model: the closed form of :func:`construct` with
    A from :func:`a_matrix_shifts` (the layers are built "using the shifts
    P_jk instead of u_j d_k", Sec. VIII-B).  Returns [n, C, H, W//2+1]
    complex128, or [n, C, len(freq_index)]."""
    _check_relaxed_reg(reg)
    view_spec = np.asarray(view_spec)
    m, C = view_spec.shape[:2]
    n = np.asarray(shifts).shape[1]
    wx_all, wy_all = flat_freqs(H, W)
    b_all = view_spec.reshape(m, C, -1)
    if freq_index is None:
        freq_index = np.arange(wx_all.shape[0])
    freq_index = np.asarray(freq_index, dtype=np.int64)
    out = np.zeros((n, C, freq_index.shape[0]), dtype=np.complex128)
    for s in range(0, freq_index.shape[0], chunk):
        fi = freq_index[s:s + chunk]
        wx, wy = wx_all[fi], wy_all[fi]
        A = a_matrix_shifts(shifts, wx, wy)
        M = normal_matrix(A, reg_matrix(reg, np.zeros(n), wx, wy), lam, eps)
        b = np.transpose(b_all[:, :, fi], (2, 0, 1)).astype(np.complex128)
        x = np.linalg.solve(M, np.conj(np.swapaxes(A, -1, -2)) @ b)
        out[:, :, s:s + chunk] = np.transpose(x, (1, 2, 0))
    if freq_index.shape[0] == wx_all.shape[0] and np.array_equal(freq_index, np.arange(wx_all.shape[0])):
        return out.reshape(n, C, H, W // 2 + 1)
    return out


def render_relaxed(layer_spec: np.ndarray, shifts: np.ndarray, H: int, W: int) -> np.ndarray:
    """The input views as the relaxed model predicts them (the denoised
    result, Sec. VIII-B): B_j(w) = sum_k exp(+2 pi i <P_jk, w>) L_k(w) for
    every row j of P [V, n, 2].  Returns [V, C, H, W//2+1] complex128."""
    layer_spec = np.asarray(layer_spec)
    n, C = layer_spec.shape[:2]
    P = np.asarray(shifts, dtype=np.float64)
    wx, wy = freq_grid(H, W)
    out = np.zeros((P.shape[0], C) + wx.shape, dtype=np.complex128)
    for j in range(P.shape[0]):
        for k in range(n):
            out[j] += np.exp(2j * math.pi * (P[j, k, 0] * wx + P[j, k, 1] * wy))[None] * layer_spec[k]
    return out


def calib_relaxed_fit_loss_grad(view_spec: np.ndarray, shifts: np.ndarray, H: int, W: int,
                                lam: float, eps: float, reg: int, freq_index: np.ndarray):
    """Objective of Eq. CalibrationProb as a function of a free shift matrix
    and its gradient, Eq. gradP with both components (R5):
    G_jk(q) = 4 pi Im(conj(x_k) conj(A_jk) r_j), r = A x - b,
    grad P^x_jk = sum_q G_jk(q) w_x(q), grad P^y_jk = sum_q G_jk(q) w_y(q).
    Returns (loss, grad_P [m, n, 2]) as float64."""
    _check_relaxed_reg(reg)
    P = np.asarray(shifts, dtype=np.float64)
    n = P.shape[1]
    wx, wy, b, R = _calib_system(view_spec, None, np.zeros(n), H, W, lam, eps, reg, freq_index)
    A = a_matrix_shifts(P, wx, wy)
    M = normal_matrix(A, R, lam, eps)
    x = np.linalg.solve(M, np.conj(np.swapaxes(A, -1, -2)) @ b)
    r = A @ x - b
    Rfull = lam * R + eps * np.eye(n)[None]
    loss = (np.sum(np.abs(r) ** 2)
            + np.real(np.einsum("qkc,qkl,qlc->", np.conj(x), Rfull, x)))
    G = 4.0 * math.pi * np.imag(np.conj(A) * np.einsum("qkc,qjc->qjk", np.conj(x), r))
    grad = np.stack([np.einsum("qjk,q->jk", G, wx), np.einsum("qjk,q->jk", G, wy)], axis=-1)
    return float(loss), grad


def calib_relaxed_loo_loss_grad(view_spec: np.ndarray, shifts: np.ndarray, H: int, W: int,
                                lam: float, eps: float, reg: int, freq_index: np.ndarray):
    """Leave-one-out loss of the relaxed model (explicit refit without each
    view, as :func:`calib_loo_loss`) and its gradient with respect to P by
    reverse-mode automatic differentiation (torch autograd, complex128, CPU).
    Returns (loss, grad_P [m, n, 2])."""
    import torch

    _check_relaxed_reg(reg)
    P0 = np.asarray(shifts, dtype=np.float64)
    n = P0.shape[1]
    wx_np, wy_np, b_np, R_np = _calib_system(view_spec, None, np.zeros(n), H, W, lam, eps, reg, freq_index)
    tP = torch.tensor(P0, requires_grad=True)
    wx = torch.tensor(wx_np)
    wy = torch.tensor(wy_np)
    b = torch.tensor(b_np)
    R = torch.tensor(R_np, dtype=torch.complex128)
    m = tP.shape[0]
    t = wx[:, None, None] * tP[None, :, :, 0] + wy[:, None, None] * tP[None, :, :, 1]
    A = torch.exp(2j * math.pi * t.to(torch.complex128))
    eye = torch.eye(n, dtype=torch.complex128)
    total = torch.zeros((), dtype=torch.float64)
    for j in range(m):
        keep = [i for i in range(m) if i != j]
        Aj = A[:, keep, :]
        Ajh = Aj.conj().transpose(-1, -2)
        x = torch.linalg.solve(Ajh @ Aj + lam * R + eps * eye, Ajh @ b[:, keep, :])
        pred = torch.einsum("qk,qkc->qc", A[:, j, :], x)
        total = total + torch.sum(torch.abs(b[:, j, :] - pred) ** 2)
    total.backward()
    return float(total.detach()), tP.grad.numpy().copy()


def calib_relaxed_loss_grad(view_spec, shifts, H, W, lam, eps, reg, mode, freq_index):
    """Dispatch on the loss mode for the relaxed model."""
    if mode == LOSS_FIT:
        return calib_relaxed_fit_loss_grad(view_spec, shifts, H, W, lam, eps, reg, freq_index)
    if mode == LOSS_LOO:
        return calib_relaxed_loo_loss_grad(view_spec, shifts, H, W, lam, eps, reg, freq_index)
    raise ValueError(f"unknown loss mode {mode}")


def gd_step_relaxed(shifts: np.ndarray, grad: np.ndarray, alpha: float = 0.2, eps_g: float = 1e-6) -> np.ndarray:
    """P' = P - alpha grad_P / (eps + ||grad_P||^2), the update of Sec. V-B
    applied to the whole shift matrix (R5)."""
    g = np.asarray(grad, dtype=np.float64)
    return np.asarray(shifts, dtype=np.float64) - alpha * g / (eps_g + np.sum(g * g))


# ---------------------------------------------------------------------------
# Drawn apertures: the discrete aperture spectrum of Sec. VI (reading R6)
# ---------------------------------------------------------------------------

def aperture_table(img: np.ndarray, pad: int) -> np.ndarray:
    """Spectrum samples of a drawn aperture, [N, N] complex128 (rows: k_y,
    columns: k_x), N = pad S: the DFT of the unit-sum image zero-padded to
    N x N (numpy.fft.fft2), times exp(+i pi (S-1)(k_x + k_y) / N), which moves
    the origin from pixel 0 to the centre pixel (S-1)/2; entry k is psi_hat
    at xi = k S / (2N)."""
    a = np.asarray(img, dtype=np.float64)
    S = a.shape[0]
    if a.shape != (S, S) or S % 2 == 0:
        raise ValueError("the aperture image must be S x S with S odd")
    N = pad * S
    w = np.zeros((N, N))
    w[:S, :S] = a / a.sum()
    X = np.fft.fft2(w)
    k = np.arange(N)
    ph = np.exp(1j * math.pi * (S - 1) * k / N)
    return X * ph[:, None] * ph[None, :]


def psi_hat_table(table: np.ndarray, S: int, rho: float, xi_x: np.ndarray, xi_y: np.ndarray) -> np.ndarray:
    """psi_hat_rho(xi) = psi_hat_1(rho xi) read from :func:`aperture_table` by
    bilinear interpolation in the continuous sample index t = rho xi 2N/S,
    with periodic wrap of the sample grid (rho = 0 gives exactly 1)."""
    N = table.shape[0]
    tx = np.asarray(rho * np.asarray(xi_x, dtype=np.float64) * (2.0 * N / S))
    ty = np.asarray(rho * np.asarray(xi_y, dtype=np.float64) * (2.0 * N / S))
    x0 = np.floor(tx)
    y0 = np.floor(ty)
    fx = tx - x0
    fy = ty - y0
    ix = x0.astype(np.int64) % N
    iy = y0.astype(np.int64) % N
    ix1 = (ix + 1) % N
    iy1 = (iy + 1) % N
    return ((1 - fy) * ((1 - fx) * table[iy, ix] + fx * table[iy, ix1])
            + fy * ((1 - fx) * table[iy1, ix] + fx * table[iy1, ix1]))


def render_tabulated(layer_spec: np.ndarray, d: np.ndarray, views: np.ndarray, H: int, W: int,
                     table: np.ndarray, S: int) -> np.ndarray:
    """:func:`render` in which views of shape AP_IMAGE use the drawn aperture
    whose spectrum is ``table`` (image size S), scaled by their radius."""
    layer_spec = np.asarray(layer_spec)
    n, C = layer_spec.shape[:2]
    d = np.asarray(d, dtype=np.float64)
    views = np.asarray(views, dtype=np.float64).reshape(-1, 5)
    wx, wy = freq_grid(H, W)
    out = np.zeros((views.shape[0], C) + wx.shape, dtype=np.complex128)
    for v, (u0, v0, s, rho, shape) in enumerate(views):
        acc = np.zeros((C,) + wx.shape, dtype=np.complex128)
        for k in range(n):
            phase = np.exp(2j * math.pi * d[k] * (u0 * wx + v0 * wy))
            if int(round(shape)) == AP_IMAGE:
                filt = psi_hat_table(table, S, rho, (s - d[k]) * wx, (s - d[k]) * wy)
            else:
                filt = psi_hat(int(round(shape)), rho, (s - d[k]) * wx, (s - d[k]) * wy)
            acc += (phase * filt)[None, :, :] * layer_spec[k]
        out[v] = acc
    return out


def rel_l2(y: np.ndarray, ref: np.ndarray) -> float:
    """||y - ref||_2 / ||ref||_2 over the whole array, in float64."""
    y = np.asarray(y).astype(np.complex128)
    ref = np.asarray(ref).astype(np.complex128)
    den = np.sqrt(np.sum(np.abs(ref) ** 2))
    return float(np.sqrt(np.sum(np.abs(y - ref) ** 2)) / max(den, 1e-300))
