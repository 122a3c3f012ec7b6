"""Seeded synthetic light-field material for the five workloads.

This module draws random numbers and shapes them into image statistics only:
layer images (blurred uniform noise or 1/f-spectrum images), view positions,
disparities, additive view noise, render requests, calibration start points
and frequency subsets.  It performs none of the Fourier Disparity Layer
arithmetic (no phase shifts, no layer sums, no solves): composing views from
layers is done by whichever side consumes this material.

Every generator takes an explicit ``numpy.random.Generator`` or seed and the
draws happen in a fixed order (layers -> positions/jitter -> noise ->
render/request parameters), so both the GPU path and the CPU checker see
identical arrays.

Conventions (Sec. III, two-plane parameterisation, generalised to 2D):
  * a view position is (u, v) = (horizontal, vertical) in view-grid units;
  * view j of a (2R+1)x(2R+1) grid has index j = (v+R)(2R+1) + (u+R);
  * disparities are in pixels per unit of view position.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

AP_PINHOLE = 0
AP_DISK = 1
AP_SQUARE = 2

REG_VIEW2 = 0
REG_LAYER2 = 1
REG_L2 = 2

LOSS_FIT = 0
LOSS_LOO = 1


@dataclasses.dataclass
class LightFieldSpec:
    """Raw material for one synthetic light field (no method arithmetic)."""

    layers: np.ndarray        # [n][C][H][W] float32, spatial layer images
    u: np.ndarray             # [m][2] float32 view positions (u, v)
    d: np.ndarray             # [n] float32 disparities
    noise: np.ndarray         # [m][C][H][W] float32 additive view noise
    lam: float
    eps: float
    reg: int
    views: np.ndarray         # [V][5] float32 render requests (u, v, focus, radius, shape)
    seed: int
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.u.shape[0])

    @property
    def n(self) -> int:
        return int(self.d.shape[0])

    @property
    def C(self) -> int:
        return int(self.layers.shape[1])

    @property
    def H(self) -> int:
        return int(self.layers.shape[2])

    @property
    def W(self) -> int:
        return int(self.layers.shape[3])


def grid_positions(R: int, jitter: float = 0.0, rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """(2R+1)^2 positions on the integer grid {-R..R}^2, optional uniform jitter."""
    g = np.arange(-R, R + 1, dtype=np.float64)
    vv, uu = np.meshgrid(g, g, indexing="ij")      # row index = v, column index = u
    pos = np.stack([uu.ravel(), vv.ravel()], axis=1)
    if jitter > 0.0:
        assert rng is not None
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    return pos.astype(np.float32)


def centered_grid_positions(g: int) -> np.ndarray:
    """g x g positions c - (g-1)/2, c = 0..g-1 on each axis (half-integers for even g)."""
    c = np.arange(g, dtype=np.float64) - (g - 1) / 2.0
    vv, uu = np.meshgrid(c, c, indexing="ij")
    return np.stack([uu.ravel(), vv.ravel()], axis=1).astype(np.float32)


def blurred_noise_layers(n: int, C: int, H: int, W: int, sigma_px: float,
                         rng: np.random.Generator) -> np.ndarray:
    """Uniform [0,1) noise, circularly blurred by a Gaussian of std ``sigma_px``.

    The blur is applied as the Gaussian's transfer function
    exp(-2 pi^2 sigma^2 |f|^2) on a full 2D FFT (an image-statistics filter,
    not part of the layer method).
    """
    x = rng.random((n, C, H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    tf = np.exp(-2.0 * math.pi ** 2 * sigma_px ** 2 * (fx ** 2 + fy ** 2))
    y = np.fft.ifft2(np.fft.fft2(x, axes=(-2, -1)) * tf, axes=(-2, -1)).real
    return y.astype(np.float32)


def pink_layers(n: int, C: int, H: int, W: int, rng: np.random.Generator) -> np.ndarray:
    """Random images with power spectrum ~ 1/|f|^2 (amplitude 1/|f|, DC zeroed),
    min-max scaled to [0, 1] per layer and channel."""
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    r = np.sqrt(fx ** 2 + fy ** 2)
    amp = np.zeros_like(r)
    amp[r > 0] = 1.0 / r[r > 0]
    white = rng.standard_normal((n, C, H, W))
    y = np.fft.ifft2(np.fft.fft2(white, axes=(-2, -1)) * amp, axes=(-2, -1)).real
    lo = y.min(axis=(-2, -1), keepdims=True)
    hi = y.max(axis=(-2, -1), keepdims=True)
    y = (y - lo) / np.maximum(hi - lo, 1e-30)
    return y.astype(np.float32)


def render_requests(V: int, rng: np.random.Generator, pos_range: float, radius_max: float,
                    focus_lo: float, focus_hi: float, shapes=(AP_DISK,)) -> np.ndarray:
    """[V][5] float32 rows (u, v, focus, radius, shape)."""
    out = np.zeros((V, 5), dtype=np.float32)
    out[:, 0:2] = rng.uniform(-pos_range, pos_range, size=(V, 2))
    out[:, 2] = rng.uniform(focus_lo, focus_hi, size=V)
    out[:, 3] = rng.uniform(0.0, radius_max, size=V)
    out[:, 4] = rng.choice(np.asarray(shapes, dtype=np.float32), size=V)
    return out


def frequency_subset(F: int, Q: int, rng: np.random.Generator) -> np.ndarray:
    """Q distinct half-spectrum bin indices drawn uniformly from [1, F)
    (the DC bin carries no gradient), sorted, int32."""
    Q = min(Q, F - 1)
    idx = rng.choice(np.arange(1, F, dtype=np.int64), size=Q, replace=False)
    return np.sort(idx).astype(np.int32)


# --------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------

def lf_5x5_128(seed: int = 0, H: int = 128, W: int = 128) -> LightFieldSpec:
    """5x5 integer grid, 128^2, 1 channel, 8 layers linspace(-2,2,8),
    blurred-noise layers (sigma 2 px), view noise 0.01, lambda 1e-2,
    16 pinhole renders at uniform positions in [-2,2]^2."""
    rng = np.random.default_rng(seed)
    n, C, R = 8, 1, 2
    layers = blurred_noise_layers(n, C, H, W, 2.0, rng)
    u = grid_positions(R)
    m = u.shape[0]
    noise = (0.01 * rng.standard_normal((m, C, H, W))).astype(np.float32)
    views = render_requests(16, rng, 2.0, 0.0, 0.0, 0.0, shapes=(AP_PINHOLE,))
    views[:, 2:4] = 0.0
    d = np.linspace(-2.0, 2.0, n).astype(np.float32)
    return LightFieldSpec(layers, u, d, noise, 1e-2, 1e-3, REG_VIEW2, views, seed, "lf_5x5_128")


def lf_9x9_512_rgb(seed: int = 2, H: int = 512, W: int = 512) -> LightFieldSpec:
    """9x9 jittered grid (+-0.05), 512^2 RGB, 30 layers linspace(-3,3,30),
    1/f^2-spectrum layers, view noise 0.005, lambda 1e-3; 81 disk-aperture
    renders at the input positions, radius U[0,2], focus U[-3,3]."""
    rng = np.random.default_rng(seed)
    n, C, R = 30, 3, 4
    layers = pink_layers(n, C, H, W, rng)
    u = grid_positions(R, 0.05, rng)
    m = u.shape[0]
    noise = (0.005 * rng.standard_normal((m, C, H, W))).astype(np.float32)
    views = np.zeros((m, 5), dtype=np.float32)
    views[:, 0:2] = u
    views[:, 2] = rng.uniform(-3.0, 3.0, size=m)
    views[:, 3] = rng.uniform(0.0, 2.0, size=m)
    views[:, 4] = AP_DISK
    d = np.linspace(-3.0, 3.0, n).astype(np.float32)
    return LightFieldSpec(layers, u, d, noise, 1e-3, 1e-3, REG_VIEW2, views, seed, "lf_9x9_512_rgb")


def uneven_light_field(i: int, base_seed: int = 3000, sizes=(128, 256, 384, 512)) -> LightFieldSpec:
    """Instance i of the 64 uneven light fields: grid 3..9, side from ``sizes``,
    8..32 layers linspace(-2,2,n), the generator of lf_5x5_128."""
    seed = base_seed + i
    rng = np.random.default_rng(seed)
    g = int(rng.integers(3, 10))
    side = int(rng.choice(np.asarray(sizes)))
    n = int(rng.integers(8, 33))
    C = 1
    layers = blurred_noise_layers(n, C, side, side, 2.0, rng)
    u = centered_grid_positions(g)
    m = u.shape[0]
    noise = (0.01 * rng.standard_normal((m, C, side, side))).astype(np.float32)
    views = np.zeros((0, 5), dtype=np.float32)
    d = np.linspace(-2.0, 2.0, n).astype(np.float32)
    return LightFieldSpec(layers, u, d, noise, 1e-2, 1e-3, REG_VIEW2, views, seed, f"uneven[{i}]")


def uneven_light_field_shape(i: int, base_seed: int = 3000, sizes=(128, 256, 384, 512)):
    """(grid side g, image side, layers n) of instance i -- the first three
    draws of :func:`uneven_light_field`, without generating the images."""
    rng = np.random.default_rng(base_seed + i)
    g = int(rng.integers(3, 10))
    side = int(rng.choice(np.asarray(sizes)))
    n = int(rng.integers(8, 33))
    return g, side, n


def lf_7x7_256_calib(seed: int = 5, H: int = 256, W: int = 256):
    """7x7 integer grid, 256^2, 1 channel, 16 layers linspace(-2,2,16),
    the generator of lf_5x5_128; returns (spec, u_init, d_init) with the start point
    perturbed by N(0,0.3^2) (positions) and N(0,0.2^2) (disparities)."""
    rng = np.random.default_rng(seed)
    n, C, R = 16, 1, 3
    layers = blurred_noise_layers(n, C, H, W, 2.0, rng)
    u = grid_positions(R)
    m = u.shape[0]
    noise = (0.01 * rng.standard_normal((m, C, H, W))).astype(np.float32)
    d = np.linspace(-2.0, 2.0, n).astype(np.float32)
    u0 = (u + 0.3 * rng.standard_normal(u.shape)).astype(np.float32)
    d0 = (d + 0.2 * rng.standard_normal(d.shape)).astype(np.float32)
    spec = LightFieldSpec(layers, u, d, noise, 1e-2, 1e-3, REG_LAYER2,
                          np.zeros((0, 5), np.float32), seed, "lf_7x7_256_calib")
    return spec, u0, d0


def shift_deviations(m: int, n: int, rng: np.random.Generator, frac: float = 0.1, amp: float = 0.5) -> np.ndarray:
    """Sparse departures from a rank-1 shift matrix, [m, n, 2] float32: a
    fraction ``frac`` of the (view, layer) pairs moves by N(0, amp^2) pixels
    per axis (a layer that some views see displaced, as an occlusion or a
    non-Lambertian surface would make it); every other entry is 0."""
    dev = (amp * rng.standard_normal((m, n, 2))).astype(np.float32)
    keep = rng.random((m, n)) < frac
    return dev * keep[:, :, None]


@dataclasses.dataclass
class Request:
    t_arrival: float      # seconds from stream start (scheduled arrival)
    kind: str             # "construct" or "render"
    lf: int               # light-field pool index
    view: np.ndarray      # [5] float32 (render only)


def serving_requests(rate: float = 200.0, duration: float = 60.0, pool: int = 8,
                     construct_frac: float = 0.2, seed: int = 4) -> List[Request]:
    """Open-loop Poisson stream: 20% construct, 80% render against a random
    resident light field, position U[-4,4]^2, disk or square (p=1/2),
    radius U[0,3], focus U[-3,3]."""
    rng = np.random.default_rng(seed)
    reqs: List[Request] = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        kind = "construct" if rng.random() < construct_frac else "render"
        lf = int(rng.integers(0, pool))
        view = np.zeros(5, dtype=np.float32)
        if kind == "render":
            view[0:2] = rng.uniform(-4.0, 4.0, size=2)
            view[2] = rng.uniform(-3.0, 3.0)
            view[3] = rng.uniform(0.0, 3.0)
            view[4] = AP_DISK if rng.random() < 0.5 else AP_SQUARE
        reqs.append(Request(t, kind, lf, view))
    return reqs


def scaled(spec_fn, H: int, W: int, **kw):
    """Same generator at a reduced resolution (for tests that must finish fast)."""
    return spec_fn(H=H, W=W, **kw)
