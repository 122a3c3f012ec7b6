"""Brute-force checkers used to pin the FP64 oracle on tiny inputs.

TEST INFRASTRUCTURE ONLY (same rule as ``fdl_oracle``).  Every function here
reaches the oracle's result by a different route: direct sums instead of
FFTs, an augmented least-squares solve instead of the normal equations, the
spatial-domain integral instead of its closed form, finite differences
instead of analytic gradients, or the closed-form leave-one-out identity
instead of explicit refits.
"""
from __future__ import annotations

import math

import numpy as np


def naive_dft2(img: np.ndarray) -> np.ndarray:
    """sum_{y,x} img[y,x] exp(-2 pi i (ky y / H + kx x / W)), full spectrum [H, W],
    by direct summation (O(H^2 W^2))."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    ys = np.arange(H)
    xs = np.arange(W)
    out = np.zeros((H, W), dtype=np.complex128)
    for ky in range(H):
        for kx in range(W):
            ph = np.exp(-2j * math.pi * (ky * ys[:, None] / H + kx * xs[None, :] / W))
            out[ky, kx] = np.sum(img * ph)
    return out


def naive_idft2_real(full_spec: np.ndarray) -> np.ndarray:
    """Real part of (1/HW) sum_k X[k] exp(+2 pi i <k, x>) by direct summation."""
    H, W = full_spec.shape
    ys = np.arange(H)
    xs = np.arange(W)
    out = np.zeros((H, W), dtype=np.complex128)
    for y in range(H):
        for x in range(W):
            ph = np.exp(2j * math.pi * (ys[:, None] * y / H + xs[None, :] * x / W))
            out[y, x] = np.sum(full_spec * ph)
    return (out / (H * W)).real


def hermitian_extend(half: np.ndarray, W: int) -> np.ndarray:
    """Rebuild the full [H, W] spectrum from a half spectrum [H, W//2+1] using
    X[-k] = conj(X[k]) for the missing columns, keeping the given columns."""
    H, Wh = half.shape
    full = np.zeros((H, W), dtype=np.complex128)
    full[:, :Wh] = half
    for kx in range(Wh, W):
        for ky in range(H):
            full[ky, kx] = np.conj(half[(-ky) % H, (-kx) % W])
    return full


def stacked_lstsq(A: np.ndarray, b: np.ndarray, Gamma: np.ndarray, lam: float, eps: float) -> np.ndarray:
    """argmin_x ||A x - b||^2 + lam ||Gamma x||^2 + eps ||x||^2 as one ordinary
    least-squares problem on the stacked system [A; sqrt(lam) Gamma; sqrt(eps) I],
    solved by numpy.linalg.lstsq (SVD based, never forms A^H A)."""
    n = A.shape[1]
    big = np.vstack([A, math.sqrt(lam) * Gamma, math.sqrt(eps) * np.eye(n)])
    rhs = np.concatenate([b, np.zeros((Gamma.shape[0] + n,) + b.shape[1:], dtype=b.dtype)], axis=0)
    x, *_ = np.linalg.lstsq(big, rhs, rcond=None)
    return x


def press_residuals(A: np.ndarray, b: np.ndarray, RtR: np.ndarray, lam: float, eps: float) -> np.ndarray:
    """Leave-one-out residuals by the PRESS identity
    b_j - a_j x^(-j) = r_j / (1 - h_jj), r = b - A x, h_jj = a_j M^-1 a_j^H,
    for one frequency.  A: [m, n], b: [m, C].  Returns [m, C]."""
    n = A.shape[1]
    M = A.conj().T @ A + lam * RtR + eps * np.eye(n)
    Minv = np.linalg.inv(M)
    x = Minv @ (A.conj().T @ b)
    r = b - A @ x
    h = np.real(np.einsum("jk,kl,jl->j", A, Minv, A.conj()))
    return r / (1.0 - h)[:, None]


def central_fd(fun, x0: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of a scalar function of a float64 array."""
    x0 = np.asarray(x0, dtype=np.float64)
    g = np.zeros_like(x0)
    flat = x0.ravel()
    gf = g.ravel()
    for i in range(flat.size):
        xp = flat.copy()
        xm = flat.copy()
        xp[i] += h
        xm[i] -= h
        gf[i] = (fun(xp.reshape(x0.shape)) - fun(xm.reshape(x0.shape))) / (2.0 * h)
    return g


def aperture_quadrature(shape: int, rho: float, xi_x: float, xi_y: float, N: int = 801) -> float:
    """int psi(u) exp(-2 pi i <u, xi>) du for a unit-integral disk (radius rho)
    or square (half-side rho), by the midpoint rule on an N x N grid over the
    aperture's bounding box.  Returns the real part (the apertures are even)."""
    t = (np.arange(N) + 0.5) / N * 2.0 * rho - rho
    uu, vv = np.meshgrid(t, t, indexing="xy")
    cell = (2.0 * rho / N) ** 2
    if shape == 1:
        mask = (uu * uu + vv * vv) <= rho * rho
        area = math.pi * rho * rho
    elif shape == 2:
        mask = np.ones_like(uu, dtype=bool)
        area = 4.0 * rho * rho
    else:
        raise ValueError(shape)
    ph = np.cos(2.0 * math.pi * (uu * xi_x + vv * xi_y))
    return float(np.sum(ph[mask]) * cell / area)


def refocus_quadrature(layer_spec_bin: np.ndarray, d: np.ndarray, u0: float, v0: float,
                       s: float, shape: int, rho: float, wx: float, wy: float, N: int = 401) -> complex:
    """One bin of a refocused image from its defining integral (Eq. BsIntermediate):
    B(w) = int exp(-2 pi i s <u, w>) psi(u) L_{u0+u}(w) du, with the sub-aperture
    spectrum L_{u0+u}(w) = sum_k exp(2 pi i d_k <u0+u, w>) L_k(w) (Eq. FourierView),
    integrated by the midpoint rule over the aperture.  layer_spec_bin: [n]."""
    t = (np.arange(N) + 0.5) / N * 2.0 * rho - rho
    uu, vv = np.meshgrid(t, t, indexing="xy")
    if shape == 1:
        mask = (uu * uu + vv * vv) <= rho * rho
    else:
        mask = np.ones_like(uu, dtype=bool)
    uu = uu[mask]
    vv = vv[mask]
    acc = 0.0 + 0.0j
    for k in range(len(d)):
        ph = np.exp(2j * math.pi * (d[k] * ((u0 + uu) * wx + (v0 + vv) * wy) - s * (uu * wx + vv * wy)))
        acc += np.mean(ph) * layer_spec_bin[k]
    return complex(acc)
