"""MI355X Fourier Disparity Layers: Python binding of libfdl.so.

Thin ctypes marshalling over the C ABI declared in ``include/fdl.h``: every
function takes torch CUDA tensors (device memory and the current stream are
the only things torch provides), checks dtypes/shapes/devices, and calls the
library entry point of the same name.  All arithmetic happens in the HIP
kernels; there is no CPU fallback -- if the library is missing the call
raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch  # must be imported before libfdl.so so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdl.so")

REG_VIEW2 = 0
REG_LAYER2 = 1
REG_L2 = 2
LOSS_FIT = 0
LOSS_LOO = 1
AP_PINHOLE = 0
AP_DISK = 1
AP_SQUARE = 2
AP_IMAGE = 3
MAX_LAYERS = 32
MAX_CHANNELS = 4

_lib = None


class FDLError(RuntimeError):
    def __init__(self, fn: str, code: int):
        self.code = code
        msg = lib().fdl_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{fn} failed: {msg} ({code})")


def lib():
    """Load libfdl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: run `python -m paper_1901_06919_amd.build` first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, f32, f64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double, ctypes.c_size_t
    L.fdl_status_string.restype = ctypes.c_char_p
    L.fdl_status_string.argtypes = [i32]
    L.fdl_version.restype = i32
    L.fdl_version.argtypes = []
    L.fdl_construct.restype = i32
    L.fdl_construct.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, i32, vp, vp, vp]
    L.fdl_construct_bins.restype = i32
    L.fdl_construct_bins.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, i32, i32, i32, vp, vp, vp]
    L.fdl_construct_views.restype = i32
    L.fdl_construct_views.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, i32, vp, vp, vp]
    L.fdl_render.restype = i32
    L.fdl_render.argtypes = [vp, vp, i32, i32, i32, i32, vp, i32, vp, vp]
    for name in ("fdl_rfft2", "fdl_irfft2"):
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.restype = i32
            fn.argtypes = [vp, vp, i32, i32, i32, vp]
    if hasattr(L, "fdl_calib_grad"):
        L.fdl_calib_workspace.restype = sz
        L.fdl_calib_workspace.argtypes = [i32, i32, i32]
        L.fdl_calib_grad.restype = i32
        L.fdl_calib_grad.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, i32, i32,
                                     vp, i32, vp, vp, vp, vp, vp, sz, vp]
        L.fdl_calib_grad_noalloc.restype = i32
        L.fdl_calib_grad_noalloc.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, i32, i32,
                                             vp, i32, vp, vp, vp, vp, vp]
        L.fdl_gd_step.restype = i32
        L.fdl_gd_step.argtypes = [vp, vp, vp, vp, i32, i32, f64, f64, vp]
    if hasattr(L, "fdl_batch_plan_create"):
        L.fdl_batch_plan_create.restype = i32
        L.fdl_batch_plan_create.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
        L.fdl_batch_plan_execute.restype = i32
        L.fdl_batch_plan_execute.argtypes = [vp, vp]
        L.fdl_batch_plan_info.restype = i32
        L.fdl_batch_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32),
                                          ctypes.POINTER(i32)]
        L.fdl_batch_plan_destroy.restype = i32
        L.fdl_batch_plan_destroy.argtypes = [vp]
        L.fdl_batch_plan_launches.restype = i32
        L.fdl_batch_plan_launches.argtypes = [vp]
        L.fdl_batch_plan_autotune.restype = i32
        L.fdl_batch_plan_autotune.argtypes = [vp, i32, vp, ctypes.POINTER(f32)]
        L.fdl_batch_plan_get_tuning.restype = i32
        L.fdl_batch_plan_get_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.fdl_batch_plan_set_tuning.restype = i32
        L.fdl_batch_plan_set_tuning.argtypes = [vp, i32, i32, i32]
    L.fdl_fma64_probe.restype = i32
    L.fdl_fma64_probe.argtypes = [vp, i32, i32, vp]
    L.fdl_construct_region.restype = i32
    L.fdl_construct_region.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, f32, vp, vp, vp]
    L.fdl_aperture_table.restype = i32
    L.fdl_aperture_table.argtypes = [vp, i32, i32, vp, vp]
    L.fdl_render_tabulated.restype = i32
    L.fdl_render_tabulated.argtypes = [vp, vp, i32, i32, i32, i32, vp, i32, vp, i32, i32, vp, vp]
    L.fdl_construct_relaxed.restype = i32
    L.fdl_construct_relaxed.argtypes = [vp, vp, i32, i32, i32, i32, i32, f32, f32, i32, vp, vp, vp]
    L.fdl_render_relaxed.restype = i32
    L.fdl_render_relaxed.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]
    L.fdl_calib_relaxed_workspace.restype = sz
    L.fdl_calib_relaxed_workspace.argtypes = [i32, i32, i32]
    L.fdl_calib_grad_relaxed.restype = i32
    L.fdl_calib_grad_relaxed.argtypes = [vp, vp, i32, i32, i32, i32, i32, f32, f32, i32, i32, vp, i32,
                                         vp, vp, vp, vp, sz, vp]
    L.fdl_gd_step_relaxed.restype = i32
    L.fdl_gd_step_relaxed.argtypes = [vp, vp, i32, i32, f64, f64, vp]
    _lib = L
    return L


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _check(t: torch.Tensor, dtype, shape, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _call(fn: str, *args):
    code = getattr(lib(), fn)(*args)
    if code != 0:
        raise FDLError(fn, code)


def view_records(views: torch.Tensor) -> torch.Tensor:
    """[V, 5] float rows (u, v, focus, radius, shape) -> device fdl_view records
    (the same 20 bytes per row, shape stored as int32)."""
    if getattr(views, "_fdl_records", False):
        return views
    v = views.to(torch.float32).contiguous().clone()
    v[:, 4] = views[:, 4].round().to(torch.int32).view(torch.float32)
    v._fdl_records = True
    return v


def rfft2(img: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """[..., H, W] float32 -> [..., H, W//2+1] complex64 (fdl_rfft2)."""
    H, W = img.shape[-2:]
    batch = img.numel() // (H * W)
    if out is None:
        out = torch.empty(img.shape[:-1] + (W // 2 + 1,), dtype=torch.complex64, device=img.device)
    _check(img, torch.float32, None, "img")
    _check(out, torch.complex64, img.shape[:-1] + (W // 2 + 1,), "out")
    _call("fdl_rfft2", img.data_ptr(), out.data_ptr(), batch, H, W, _stream(img))
    return out


def irfft2(spec: torch.Tensor, H: int, W: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """[..., H, W//2+1] complex64 -> [..., H, W] float32 (fdl_irfft2).  ``spec`` is
    used as scratch and overwritten (pass a clone to keep it)."""
    batch = spec.numel() // (H * (W // 2 + 1))
    if out is None:
        out = torch.empty(spec.shape[:-1] + (W,), dtype=torch.float32, device=spec.device)
    _check(spec, torch.complex64, spec.shape[:-2] + (H, W // 2 + 1), "spec")
    _check(out, torch.float32, spec.shape[:-1] + (W,), "out")
    _call("fdl_irfft2", spec.data_ptr(), out.data_ptr(), batch, H, W, _stream(spec))
    return out


def construct(view_spec: torch.Tensor, u: torch.Tensor, d: torch.Tensor, H: int, W: int,
              lam: float, eps: float, reg: int = REG_VIEW2, out: Optional[torch.Tensor] = None,
              status: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Layer spectra [n, C, H, W//2+1] from view spectra [m, C, H, W//2+1] (fdl_construct)."""
    m, C = view_spec.shape[:2]
    n = d.shape[0]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    _check(u, torch.float32, (m, 2), "u")
    if d.dtype != torch.float32 or d.dim() != 1:
        raise TypeError("d must be a 1-D float32 tensor")
    d_host = d.detach().to("cpu").contiguous()          # disparities travel by value
    if out is None:
        out = torch.empty((n, C, H, W // 2 + 1), dtype=torch.complex64, device=view_spec.device)
    _check(out, torch.complex64, (n, C, H, W // 2 + 1), "out")
    sp = 0
    if status is not None:
        _check(status, torch.int32, (1,), "status")
        sp = status.data_ptr()
    _call("fdl_construct", view_spec.data_ptr(), u.data_ptr(), d_host.data_ptr(), m, n, C, H, W,
          float(lam), float(eps), int(reg), out.data_ptr(), sp, _stream(view_spec))
    return out


def construct_bins(view_spec: torch.Tensor, u: torch.Tensor, d: torch.Tensor, H: int, W: int, lam: float,
                   eps: float, reg: int, bin_begin: int, bin_count: int, out: torch.Tensor,
                   status: Optional[torch.Tensor] = None) -> torch.Tensor:
    """fdl_construct_bins: the bins [bin_begin, bin_begin + bin_count) of
    :func:`construct` written into ``out`` (the other bins untouched)."""
    m, C = view_spec.shape[:2]
    n = d.shape[0]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    _check(u, torch.float32, (m, 2), "u")
    _check(out, torch.complex64, (n, C, H, W // 2 + 1), "out")
    d_host = d.detach().to("cpu").to(torch.float32).contiguous()
    _call("fdl_construct_bins", view_spec.data_ptr(), u.data_ptr(), d_host.data_ptr(), m, n, C, H, W,
          float(lam), float(eps), int(reg), int(bin_begin), int(bin_count), out.data_ptr(), _status_ptr(status),
          _stream(view_spec))
    return out


def construct_views(view_spec: torch.Tensor, views: torch.Tensor, d: torch.Tensor, H: int, W: int,
                    lam: float, eps: float, reg: int = REG_VIEW2, out: Optional[torch.Tensor] = None,
                    status: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Layer spectra [n, C, H, W//2+1] from view spectra [m, C, H, W//2+1] of
    input views with their own apertures (fdl_construct_views).  ``views``
    are [m, 5] float rows (u, v, focus, radius, shape) or records from
    :func:`view_records`, one per input view."""
    m, C = view_spec.shape[:2]
    n = d.shape[0]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    if not views.is_cuda:
        raise ValueError("views must be a device tensor")
    rec = views if getattr(views, "_fdl_records", False) else view_records(views)
    if rec.shape[0] != m:
        raise ValueError(f"views must describe the {m} input views, got {rec.shape[0]}")
    if d.dtype != torch.float32 or d.dim() != 1:
        raise TypeError("d must be a 1-D float32 tensor")
    d_host = d.detach().to("cpu").contiguous()          # disparities travel by value
    if out is None:
        out = torch.empty((n, C, H, W // 2 + 1), dtype=torch.complex64, device=view_spec.device)
    _check(out, torch.complex64, (n, C, H, W // 2 + 1), "out")
    sp = 0
    if status is not None:
        _check(status, torch.int32, (1,), "status")
        sp = status.data_ptr()
    _call("fdl_construct_views", view_spec.data_ptr(), rec.data_ptr(), d_host.data_ptr(), m, n, C, H, W,
          float(lam), float(eps), int(reg), out.data_ptr(), sp, _stream(view_spec))
    return out


def render(layer_spec: torch.Tensor, d: torch.Tensor, views: torch.Tensor, H: int, W: int,
           out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Rendered spectra [V, C, H, W//2+1] (fdl_render).  ``views`` are [V, 5]
    float rows (u, v, focus, radius, shape) or records from :func:`view_records`."""
    n, C = layer_spec.shape[:2]
    _check(layer_spec, torch.complex64, (n, C, H, W // 2 + 1), "layer_spec")
    _check(d, torch.float32, (n,), "d")
    if not views.is_cuda:
        raise ValueError("views must be a device tensor")
    rec = views if getattr(views, "_fdl_records", False) else view_records(views)
    V = rec.shape[0]
    if out is None:
        out = torch.empty((V, C, H, W // 2 + 1), dtype=torch.complex64, device=layer_spec.device)
    _check(out, torch.complex64, (V, C, H, W // 2 + 1), "out")
    _call("fdl_render", layer_spec.data_ptr(), d.data_ptr(), n, C, H, W, rec.data_ptr(), V,
          out.data_ptr(), _stream(layer_spec))
    return out


def _status_ptr(status: Optional[torch.Tensor]) -> int:
    if status is None:
        return 0
    _check(status, torch.int32, (1,), "status")
    return status.data_ptr()


def calib_workspace_bytes(m: int, n: int, Q: int) -> int:
    return int(lib().fdl_calib_workspace(m, n, Q))


def calib_grad(view_spec: torch.Tensor, u: torch.Tensor, d: torch.Tensor, H: int, W: int,
               lam: float, eps: float, reg: int, mode: int, freq_idx: Optional[torch.Tensor] = None,
               out: Optional[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = None,
               ws: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None):
    """(loss [1] f64, grad_u [m,2] f64, grad_d [n] f64) (fdl_calib_grad).
    ``status`` (int32 [1] on the device, optional) counts indices of
    ``freq_idx`` outside [0, F); the kernel clamps them."""
    m, C = view_spec.shape[:2]
    n = d.shape[0]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    _check(u, torch.float32, (m, 2), "u")
    _check(d, torch.float32, (n,), "d")
    dev = view_spec.device
    if freq_idx is not None:
        _check(freq_idx, torch.int32, None, "freq_idx")
        Q = freq_idx.numel()
        fp = freq_idx.data_ptr()
    else:
        Q = H * (W // 2 + 1)
        fp = 0
    if out is None:
        out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((m, 2), dtype=torch.float64, device=dev),
               torch.empty(n, dtype=torch.float64, device=dev))
    loss, gu, gd = out
    need = calib_workspace_bytes(m, n, Q)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _call("fdl_calib_grad", view_spec.data_ptr(), u.data_ptr(), d.data_ptr(), m, n, C, H, W, float(lam),
          float(eps), int(reg), int(mode), fp, Q, loss.data_ptr(), gu.data_ptr(), gd.data_ptr(),
          _status_ptr(status), ws.data_ptr(), ws.numel(), _stream(view_spec))
    return loss, gu, gd


def calib_grad_noalloc(view_spec: torch.Tensor, u: torch.Tensor, d: torch.Tensor, H: int, W: int,
                       lam: float, eps: float, reg: int, mode: int, freq_idx: Optional[torch.Tensor] = None,
                       out: Tuple[torch.Tensor, torch.Tensor, torch.Tensor] = None,
                       status: Optional[torch.Tensor] = None):
    """fdl_calib_grad_noalloc: :func:`calib_grad` without a workspace; the
    library keeps the partial sums in its static per-GPU array.  ``out`` =
    (loss [1], grad_u [m,2], grad_d [n]) float64 tensors is required, so the
    call allocates nothing."""
    m, C = view_spec.shape[:2]
    n = d.shape[0]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    _check(u, torch.float32, (m, 2), "u")
    _check(d, torch.float32, (n,), "d")
    if out is None:
        raise ValueError("calib_grad_noalloc needs caller-provided outputs")
    loss, gu, gd = out
    _check(loss, torch.float64, (1,), "loss")
    _check(gu, torch.float64, (m, 2), "grad_u")
    _check(gd, torch.float64, (n,), "grad_d")
    if freq_idx is not None:
        _check(freq_idx, torch.int32, None, "freq_idx")
        Q, fp = freq_idx.numel(), freq_idx.data_ptr()
    else:
        Q, fp = H * (W // 2 + 1), 0
    _call("fdl_calib_grad_noalloc", view_spec.data_ptr(), u.data_ptr(), d.data_ptr(), m, n, C, H, W, float(lam),
          float(eps), int(reg), int(mode), fp, Q, loss.data_ptr(), gu.data_ptr(), gd.data_ptr(),
          _status_ptr(status), _stream(view_spec))
    return loss, gu, gd


def gd_step(u: torch.Tensor, d: torch.Tensor, grad_u: torch.Tensor, grad_d: torch.Tensor,
            alpha: float = 0.2, eps_g: float = 1e-6) -> None:
    """In-place normalised gradient step on u [m,2] f32 and d [n] f32 (fdl_gd_step)."""
    m, n = u.shape[0], d.shape[0]
    _check(u, torch.float32, (m, 2), "u")
    _check(d, torch.float32, (n,), "d")
    _check(grad_u, torch.float64, (m, 2), "grad_u")
    _check(grad_d, torch.float64, (n,), "grad_d")
    _call("fdl_gd_step", u.data_ptr(), d.data_ptr(), grad_u.data_ptr(), grad_d.data_ptr(), m, n,
          float(alpha), float(eps_g), _stream(u))


def construct_region(view_spec: torch.Tensor, u: torch.Tensor, d: torch.Tensor, H: int, W: int, lam: float,
                     eps: float, region: float, out: Optional[torch.Tensor] = None,
                     status: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Layer spectra with the view regulariser over the camera-plane square of
    side ``region`` (fdl_construct_region); otherwise as :func:`construct`."""
    m, C = view_spec.shape[:2]
    n = d.shape[0]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    _check(u, torch.float32, (m, 2), "u")
    if d.dtype != torch.float32 or d.dim() != 1:
        raise TypeError("d must be a 1-D float32 tensor")
    d_host = d.detach().to("cpu").contiguous()
    if out is None:
        out = torch.empty((n, C, H, W // 2 + 1), dtype=torch.complex64, device=view_spec.device)
    _check(out, torch.complex64, (n, C, H, W // 2 + 1), "out")
    sp = 0
    if status is not None:
        _check(status, torch.int32, (1,), "status")
        sp = status.data_ptr()
    _call("fdl_construct_region", view_spec.data_ptr(), u.data_ptr(), d_host.data_ptr(), m, n, C, H, W,
          float(lam), float(eps), float(region), out.data_ptr(), sp, _stream(view_spec))
    return out


# ---- drawn apertures (Sec. VI) ----

def aperture_table(img: torch.Tensor, pad: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Spectrum samples [N, N] complex64, N = pad S, of a drawn aperture
    img [S, S] float32 (S odd) on the device (fdl_aperture_table)."""
    S = img.shape[0]
    N = pad * S
    _check(img, torch.float32, (S, S), "img")
    if out is None:
        out = torch.empty((N, N), dtype=torch.complex64, device=img.device)
    _check(out, torch.complex64, (N, N), "out")
    _call("fdl_aperture_table", img.data_ptr(), S, int(pad), out.data_ptr(), _stream(img))
    return out


def render_tabulated(layer_spec: torch.Tensor, d: torch.Tensor, views: torch.Tensor, H: int, W: int,
                     table: torch.Tensor, S: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """:func:`render` in which views of shape AP_IMAGE use the drawn aperture
    whose table (from :func:`aperture_table`, image side S) is given
    (fdl_render_tabulated)."""
    n, C = layer_spec.shape[:2]
    _check(layer_spec, torch.complex64, (n, C, H, W // 2 + 1), "layer_spec")
    _check(d, torch.float32, (n,), "d")
    N = table.shape[0]
    _check(table, torch.complex64, (N, N), "table")
    if not views.is_cuda:
        raise ValueError("views must be a device tensor")
    rec = views if getattr(views, "_fdl_records", False) else view_records(views)
    V = rec.shape[0]
    if out is None:
        out = torch.empty((V, C, H, W // 2 + 1), dtype=torch.complex64, device=layer_spec.device)
    _check(out, torch.complex64, (V, C, H, W // 2 + 1), "out")
    _call("fdl_render_tabulated", layer_spec.data_ptr(), d.data_ptr(), n, C, H, W, rec.data_ptr(), V,
          table.data_ptr(), N, int(S), out.data_ptr(), _stream(layer_spec))
    return out


# ---- relaxed model (Sec. VIII-B): a free shift pair per view and layer ----

def _check_shifts(shifts: torch.Tensor, rows: int, n: int):
    _check(shifts, torch.float32, (rows, n, 2), "shifts")


def construct_relaxed(view_spec: torch.Tensor, shifts: torch.Tensor, H: int, W: int, lam: float, eps: float,
                      reg: int = REG_LAYER2, out: Optional[torch.Tensor] = None,
                      status: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Layer spectra [n, C, H, W//2+1] of the relaxed model from view spectra
    [m, C, H, W//2+1] and shifts [m, n, 2] float32 (fdl_construct_relaxed)."""
    m, C = view_spec.shape[:2]
    n = shifts.shape[1]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    _check_shifts(shifts, m, n)
    if out is None:
        out = torch.empty((n, C, H, W // 2 + 1), dtype=torch.complex64, device=view_spec.device)
    _check(out, torch.complex64, (n, C, H, W // 2 + 1), "out")
    sp = 0
    if status is not None:
        _check(status, torch.int32, (1,), "status")
        sp = status.data_ptr()
    _call("fdl_construct_relaxed", view_spec.data_ptr(), shifts.data_ptr(), m, n, C, H, W, float(lam), float(eps),
          int(reg), out.data_ptr(), sp, _stream(view_spec))
    return out


def render_relaxed(layer_spec: torch.Tensor, shifts: torch.Tensor, H: int, W: int,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Spectra [V, C, H, W//2+1] of the views whose shift rows are
    shifts [V, n, 2] (fdl_render_relaxed)."""
    n, C = layer_spec.shape[:2]
    V = shifts.shape[0]
    _check(layer_spec, torch.complex64, (n, C, H, W // 2 + 1), "layer_spec")
    _check_shifts(shifts, V, n)
    if out is None:
        out = torch.empty((V, C, H, W // 2 + 1), dtype=torch.complex64, device=layer_spec.device)
    _check(out, torch.complex64, (V, C, H, W // 2 + 1), "out")
    _call("fdl_render_relaxed", layer_spec.data_ptr(), shifts.data_ptr(), n, C, H, W, V, out.data_ptr(),
          _stream(layer_spec))
    return out


def calib_relaxed_workspace_bytes(m: int, n: int, Q: int) -> int:
    return int(lib().fdl_calib_relaxed_workspace(m, n, Q))


def calib_grad_relaxed(view_spec: torch.Tensor, shifts: torch.Tensor, H: int, W: int, lam: float, eps: float,
                       reg: int, mode: int, freq_idx: Optional[torch.Tensor] = None,
                       out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, ws: Optional[torch.Tensor] = None,
                       status: Optional[torch.Tensor] = None):
    """(loss [1] f64, grad_shifts [m, n, 2] f64) (fdl_calib_grad_relaxed); ``status`` as
    :func:`calib_grad`."""
    m, C = view_spec.shape[:2]
    n = shifts.shape[1]
    _check(view_spec, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
    _check_shifts(shifts, m, n)
    dev = view_spec.device
    if freq_idx is not None:
        _check(freq_idx, torch.int32, None, "freq_idx")
        Q = freq_idx.numel()
        fp = freq_idx.data_ptr()
    else:
        Q = H * (W // 2 + 1)
        fp = 0
    if out is None:
        out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((m, n, 2), dtype=torch.float64, device=dev))
    loss, g = out
    _check(loss, torch.float64, (1,), "loss")
    _check(g, torch.float64, (m, n, 2), "grad_shifts")
    need = calib_relaxed_workspace_bytes(m, n, Q)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _call("fdl_calib_grad_relaxed", view_spec.data_ptr(), shifts.data_ptr(), m, n, C, H, W, float(lam), float(eps),
          int(reg), int(mode), fp, Q, loss.data_ptr(), g.data_ptr(), _status_ptr(status), ws.data_ptr(), ws.numel(),
          _stream(view_spec))
    return loss, g


def gd_step_relaxed(shifts: torch.Tensor, grad: torch.Tensor, alpha: float = 0.2, eps_g: float = 1e-6) -> None:
    """In-place normalised gradient step on shifts [m, n, 2] f32 (fdl_gd_step_relaxed)."""
    m, n = shifts.shape[:2]
    _check_shifts(shifts, m, n)
    _check(grad, torch.float64, (m, n, 2), "grad")
    _call("fdl_gd_step_relaxed", shifts.data_ptr(), grad.data_ptr(), m, n, float(alpha), float(eps_g),
          _stream(shifts))


def fma64_probe(out: torch.Tensor, iters: int) -> float:
    """Enqueue the FP64 multiply-add loop (fdl_fma64_probe) over out.numel()/256
    blocks; returns the flops it performs (16 per thread per iteration)."""
    _check(out, torch.float64, None, "out")
    if out.numel() % 256:
        raise ValueError("out must hold a multiple of 256 doubles")
    blocks = out.numel() // 256
    _call("fdl_fma64_probe", out.data_ptr(), blocks, int(iters), _stream(out))
    return 16.0 * out.numel() * iters


class LFDesc(ctypes.Structure):
    """Mirror of fdl_lf_desc."""
    _fields_ = [("view_spec", ctypes.c_void_p), ("u", ctypes.c_void_p), ("d", ctypes.c_void_p),
                ("layer_spec", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("C", ctypes.c_int32), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("reg", ctypes.c_int32), ("lam", ctypes.c_float), ("eps", ctypes.c_float)]


class BatchPlan:
    """Persistent batched construction over many light fields (fdl_batch_plan_*).

    ``items`` is a list of dicts with keys view_spec [m,C,H,W//2+1] c64, u [m,2]
    f32, d [n] f32 (device), out [n,C,H,W//2+1] c64, H, W, lam, eps, reg and
    optionally status [1] i32.  The tensors must stay alive while the plan is
    used (the plan stores their device pointers)."""

    def __init__(self, items, mode: int = 0):
        self._items = items
        arr = (LFDesc * len(items))()
        for i, it in enumerate(items):
            vs, u, d, out = it["view_spec"], it["u"], it["d"], it["out"]
            m, C = vs.shape[:2]
            n = d.shape[0]
            H, W = it["H"], it["W"]
            _check(vs, torch.complex64, (m, C, H, W // 2 + 1), "view_spec")
            _check(u, torch.float32, (m, 2), "u")
            _check(d, torch.float32, (n,), "d")
            _check(out, torch.complex64, (n, C, H, W // 2 + 1), "out")
            st = it.get("status")
            arr[i] = LFDesc(vs.data_ptr(), u.data_ptr(), d.data_ptr(), out.data_ptr(),
                            st.data_ptr() if st is not None else 0, m, n, C, H, W, int(it.get("reg", REG_VIEW2)),
                            float(it["lam"]), float(it["eps"]))
        self._descs = arr
        h = ctypes.c_void_p()
        _call("fdl_batch_plan_create", ctypes.cast(arr, ctypes.c_void_p), len(items), int(mode), ctypes.byref(h))
        self._h = h

    def execute(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _call("fdl_batch_plan_execute", self._h, s)

    def autotune(self, reps: int = 3) -> float:
        ms = ctypes.c_float()
        _call("fdl_batch_plan_autotune", self._h, int(reps), torch.cuda.current_stream().cuda_stream, ctypes.byref(ms))
        return float(ms.value)

    @property
    def launches(self) -> int:
        return int(lib().fdl_batch_plan_launches(self._h))

    def tuning(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _call("fdl_batch_plan_get_tuning", self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return {"mode": a.value, "chunk": b.value, "grid_per_cu": c.value}

    def set_tuning(self, mode: int, chunk: int = 1, grid_per_cu: int = 2):
        _call("fdl_batch_plan_set_tuning", self._h, int(mode), int(chunk), int(grid_per_cu))

    def info(self):
        tb, g, t = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _call("fdl_batch_plan_info", self._h, ctypes.byref(tb), ctypes.byref(g), ctypes.byref(t))
        return {"total_bins": tb.value, "grid": g.value, "launches": t.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fdl_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
