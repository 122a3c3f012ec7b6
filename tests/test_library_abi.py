"""CPU checks of the boundary: the shared library loads, exports every entry
point include/fdl.h declares, and rejects bad arguments on the host before
touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fdl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(fdl_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import paper_1901_06919_amd as fdl
    L = fdl.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), f"{n} declared in fdl.h but not exported"


def test_status_strings_and_version():
    import paper_1901_06919_amd as fdl
    L = fdl.lib()
    assert L.fdl_status_string(0) == b"ok"
    assert L.fdl_status_string(-2) == b"unsupported shape"
    assert L.fdl_version() >= 10000


def test_host_side_validation_without_gpu():
    import paper_1901_06919_amd as fdl
    L = fdl.lib()
    d = (ctypes.c_float * 4)(0, 1, 2, 3)
    fake = ctypes.c_void_p(0x1000)
    # n out of range, null pointers, bad sizes: rejected before any launch
    assert L.fdl_construct(fake, fake, d, 4, 40, 1, 8, 8, 0.01, 0.001, 0, fake, None, None) == -2
    assert L.fdl_construct(None, fake, d, 4, 4, 1, 8, 8, 0.01, 0.001, 0, fake, None, None) == -1
    assert L.fdl_construct(fake, fake, d, 4, 4, 1, 8, 7, 0.01, 0.001, 0, fake, None, None) == -2
    assert L.fdl_construct(fake, fake, d, 4, 4, 1, 8, 8, -1.0, 0.001, 0, fake, None, None) == -1
    assert L.fdl_rfft2(fake, fake, 1, 8, 10, None) == -2          # W/2 = 5 unsupported
    assert L.fdl_rfft2(fake, fake, 1, 7, 8, None) == -2           # H = 7 unsupported
    assert L.fdl_render(fake, fake, 33, 1, 8, 8, fake, 1, fake, None) == -2
    assert L.fdl_calib_grad(fake, fake, fake, 300, 4, 1, 8, 8, 0.01, 0.001, 1, 1, None, 0,
                            fake, fake, fake, None, fake, 1 << 20, None) == -2
    assert L.fdl_calib_workspace(49, 16, 4096) == 2048 * (1 + 98 + 16) * 8
    assert L.fdl_fma64_probe(None, 1, 1, None) == -1
    assert L.fdl_construct_views(None, fake, d, 4, 4, 1, 8, 8, 0.01, 0.001, 0, fake, None, None) == -1
    assert L.fdl_construct_views(fake, fake, d, 4, 40, 1, 8, 8, 0.01, 0.001, 0, fake, None, None) == -2
    # relaxed model: no view regulariser, shape limits, workspace size
    assert L.fdl_construct_relaxed(fake, fake, 4, 4, 1, 8, 8, 0.01, 0.001, 0, fake, None, None) == -1
    assert L.fdl_construct_relaxed(fake, None, 4, 4, 1, 8, 8, 0.01, 0.001, 1, fake, None, None) == -1
    assert L.fdl_construct_relaxed(fake, fake, 4, 33, 1, 8, 8, 0.01, 0.001, 1, fake, None, None) == -2
    assert L.fdl_render_relaxed(fake, fake, 33, 1, 8, 8, 1, fake, None) == -2
    assert L.fdl_render_relaxed(fake, fake, 4, 1, 8, 8, 0, fake, None) == -2
    assert L.fdl_calib_grad_relaxed(fake, fake, 4, 4, 1, 8, 8, 0.01, 0.001, 0, 0, None, 0,
                                    fake, fake, None, fake, 1 << 20, None) == -1
    assert L.fdl_calib_grad_relaxed(fake, fake, 300, 4, 1, 8, 8, 0.01, 0.001, 1, 0, None, 0,
                                    fake, fake, None, fake, 1 << 20, None) == -2
    assert L.fdl_calib_grad_relaxed(fake, fake, 4, 4, 1, 8, 8, 0.01, 0.001, 1, 0, None, 0,
                                    fake, fake, None, fake, 16, None) == -3
    assert L.fdl_calib_relaxed_workspace(49, 16, 4096) == 2048 * (1 + 2 * 49 * 16) * 8
    assert L.fdl_gd_step_relaxed(None, fake, 4, 4, 0.2, 1e-6, None) == -1
    # drawn apertures: odd image side, table size limits
    assert L.fdl_aperture_table(fake, 4, 2, fake, None) == -2
    assert L.fdl_aperture_table(fake, 255, 9, fake, None) == -2
    assert L.fdl_aperture_table(None, 5, 2, fake, None) == -1
    assert L.fdl_render_tabulated(fake, fake, 4, 1, 8, 8, fake, 1, fake, 12, 5, fake, None) == -2
    assert L.fdl_render_tabulated(fake, fake, 4, 1, 8, 8, fake, 1, None, 10, 5, fake, None) == -1
    # request server: argument checks before any device work
    h = ctypes.c_void_p()
    assert L.fdl_server_create(ctypes.c_size_t(0), 4, 4, 0, ctypes.byref(h)) == -1
    assert L.fdl_server_create(ctypes.c_size_t(1 << 30), 0, 4, 0, ctypes.byref(h)) == -1
    assert L.fdl_server_create(ctypes.c_size_t(1 << 30), 4, 65, 0, ctypes.byref(h)) == -1
    assert L.fdl_server_submit(None, None, None) == -1
    assert L.fdl_server_destroy(None) == -1
    # empty inputs are rejected, never launched: no views, layers, images, bins
    # or samples, an empty bin range, an empty batch
    assert L.fdl_construct(fake, fake, d, 0, 4, 1, 8, 8, 0.01, 0.001, 0, fake, None, None) == -2
    assert L.fdl_construct(fake, fake, d, 4, 0, 1, 8, 8, 0.01, 0.001, 0, fake, None, None) == -2
    assert L.fdl_construct_bins(fake, fake, d, 4, 4, 1, 8, 8, 0.01, 0.001, 0, 0, 0, fake, None, None) == -1
    assert L.fdl_construct_bins(fake, fake, d, 4, 4, 1, 8, 8, 0.01, 0.001, 0, 30, 11, fake, None, None) == -1
    assert L.fdl_construct_bins(fake, fake, d, 4, 4, 1, 8, 8, 0.01, 0.001, 0, -1, 4, fake, None, None) == -1
    assert L.fdl_rfft2(fake, fake, 0, 8, 8, None) == -2
    assert L.fdl_irfft2(fake, fake, 0, 8, 8, None) == -2
    assert L.fdl_render(fake, fake, 4, 1, 8, 8, fake, 0, fake, None) == -2
    assert L.fdl_calib_grad(fake, fake, fake, 4, 4, 1, 8, 8, 0.01, 0.001, 1, 1, fake, 0,
                            fake, fake, fake, None, fake, 1 << 20, None) == -1
    plan = ctypes.c_void_p()
    assert L.fdl_batch_plan_create(fake, 0, 0, ctypes.byref(plan)) == -1
    # finite-region view regulariser: the region side must be finite and positive
    assert L.fdl_construct_region(fake, fake, d, 4, 4, 1, 8, 8, 0.01, 0.001, 0.0, fake, None, None) == -1
    assert L.fdl_construct_region(fake, fake, d, 4, 40, 1, 8, 8, 0.01, 0.001, 2.0, fake, None, None) == -2
