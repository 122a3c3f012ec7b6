"""Python driver of the library's request server (fdl_server_* in the C ABI).

The server itself -- admission by HBM footprint from one budgeted device pool,
continuous batching of renders per light field, the worker thread that
retires finished work and launches arrived requests on its streams, and the
latency bookkeeping -- lives in libfdl (csrc/serve.cpp, policy in
csrc/serve_core.h).  This module only marshals arguments: it registers the
light fields, submits a request stream with its scheduled arrival times (all
ahead of time: the server starts each request no earlier than its arrival, so
no Python runs between arrival and completion), waits for the server to
drain, and reads back its statistics.

Requests are ``synth.Request`` objects (t_arrival, kind, lf, view); the
latency of a request is its completion, as seen by the server's worker
thread, minus its scheduled arrival (open loop, no coordinated omission).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Dict, List, Optional

import numpy as np
import torch

from . import FDLError, _check, lib

REQ_CONSTRUCT = 0
REQ_RENDER = 1
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_REJECTED = 0, 1, 2, 3


class _View(ctypes.Structure):
    _fields_ = [("u", ctypes.c_float), ("v", ctypes.c_float), ("focus", ctypes.c_float),
                ("radius", ctypes.c_float), ("shape", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lf", ctypes.c_int32), ("view", _View),
                ("image_dev", ctypes.c_void_p), ("t_arrival", ctypes.c_double)]


class _Summary(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("count", ctypes.c_int64 * 3), ("p50_ms", ctypes.c_double * 3), ("p99_ms", ctypes.c_double * 3),
                ("mean_ms", ctypes.c_double * 3), ("render_batches", ctypes.c_int64),
                ("mean_render_batch", ctypes.c_double), ("pool_high_water_bytes", ctypes.c_double),
                ("resident_bytes", ctypes.c_double), ("first_arrival_s", ctypes.c_double),
                ("last_completion_s", ctypes.c_double)]


class _SimRequest(ctypes.Structure):
    _fields_ = [("t_arrival", ctypes.c_double), ("kind", ctypes.c_int32), ("lf", ctypes.c_int32)]


class _SimResult(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("batch", ctypes.c_int32), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_declared = False


def _L():
    global _declared
    L = lib()
    if not _declared:
        vp, i32, f32, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_double, ctypes.c_size_t
        sigs = {
            "fdl_server_create": [sz, i32, i32, i32, ctypes.POINTER(vp)],
            "fdl_server_add_lightfield": [vp, vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, i32,
                                          ctypes.POINTER(i32)],
            "fdl_server_submit": [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_int64)],
            "fdl_server_poll": [vp, ctypes.c_int64, ctypes.POINTER(i32), ctypes.POINTER(f64)],
            "fdl_server_drain": [vp, f64],
            "fdl_server_now": [vp, ctypes.POINTER(f64)],
            "fdl_server_layers": [vp, i32, ctypes.POINTER(vp)],
            "fdl_server_stats": [vp, ctypes.POINTER(_Summary)],
            "fdl_server_destroy": [vp],
            "fdl_server_simulate": [sz, i32, i32, i32, i32, ctypes.POINTER(sz), ctypes.POINTER(sz), f64, f64,
                                    ctypes.POINTER(_SimRequest), i32, ctypes.POINTER(_SimResult),
                                    ctypes.POINTER(_Summary)],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.restype = i32
            fn.argtypes = args
        _declared = True
    return L


def _ok(fn: str, code: int):
    if code != 0:
        raise FDLError(fn, code)


def _summary_dict(s: _Summary, budget: int) -> dict:
    out = {"submitted": s.submitted, "completed": s.completed, "rejected": s.rejected,
           "throughput_rps": s.completed / max(s.last_completion_s - s.first_arrival_s, 1e-9),
           "max_reserved_MB": s.pool_high_water_bytes / 2 ** 20, "resident_MB": s.resident_bytes / 2 ** 20,
           "budget_MB": budget / 2 ** 20, "render_batches": s.render_batches,
           "mean_render_batch": s.mean_render_batch}
    for k, name in enumerate(("all", "construct", "render")):
        if s.count[k]:
            out[f"{name}_p50_ms"] = s.p50_ms[k]
            out[f"{name}_p99_ms"] = s.p99_ms[k]
            out[f"{name}_mean_ms"] = s.mean_ms[k]
            out[f"{name}_count"] = int(s.count[k])
    return out


@dataclasses.dataclass
class PoolEntry:
    view_spec: torch.Tensor      # [m, C, H, W//2+1] complex64 (resident)
    u: torch.Tensor              # [m, 2] f32 device
    d_host: torch.Tensor         # [n] f32 host
    d_dev: torch.Tensor          # [n] f32 device (for checks that render outside the server)
    H: int
    W: int
    lam: float
    eps: float
    reg: int


@dataclasses.dataclass
class ServeStats:
    completed: int
    rejected: int
    latency_ms: np.ndarray       # per completed request, in submission order
    summary_dict: dict
    max_reserved_bytes: int
    hbm_budget: int
    mean_render_batch: float

    def summary(self) -> dict:
        return dict(self.summary_dict)


class FDLServer:
    """Handle of one library server.  ``serial=True`` is the plain baseline
    (arrival order, one unit of work at a time on one stream, one view per
    render)."""

    def __init__(self, pool: List[PoolEntry], hbm_budget: int = 4 << 30, max_render_batch: int = 16,
                 max_inflight: int = 8, keep_outputs_every: int = 0, serial: bool = False):
        L = _L()
        self.pool = pool
        self.budget = int(hbm_budget)
        self.keep_every = int(keep_outputs_every)
        self.kept: Dict[int, torch.Tensor] = {}
        h = ctypes.c_void_p()
        _ok("fdl_server_create", L.fdl_server_create(self.budget, int(max_render_batch), int(max_inflight),
                                                      1 if serial else 0, ctypes.byref(h)))
        self.h = h
        self.lf_ids = []
        self._d_host = []
        for e in pool:
            m, C = e.view_spec.shape[:2]
            n = e.d_host.shape[0]
            _check(e.view_spec, torch.complex64, (m, C, e.H, e.W // 2 + 1), "view_spec")
            _check(e.u, torch.float32, (m, 2), "u")
            d = e.d_host.to(torch.float32).contiguous().cpu()
            self._d_host.append(d)
            lf = ctypes.c_int32()
            _ok("fdl_server_add_lightfield",
                L.fdl_server_add_lightfield(self.h, e.view_spec.data_ptr(), e.u.data_ptr(), d.data_ptr(), m, n, C,
                                            e.H, e.W, float(e.lam), float(e.eps), int(e.reg), ctypes.byref(lf)))
            self.lf_ids.append(lf.value)

    def now(self) -> float:
        t = ctypes.c_double()
        _ok("fdl_server_now", _L().fdl_server_now(self.h, ctypes.byref(t)))
        return t.value

    def run(self, requests, time_scale: float = 1.0, lead_s: float = 0.05, timeout_s: float = 600.0) -> ServeStats:
        """Submit ``requests`` (t_arrival, kind, lf, view, and an integer
        ``rid`` when outputs are kept) with arrivals ``lead_s`` after now,
        wait until the server has served them, and return the statistics."""
        L = _L()
        t0 = self.now() + lead_s
        ids = []
        images = {}
        for r in requests:
            req = _Request()
            req.kind = REQ_CONSTRUCT if r.kind == "construct" else REQ_RENDER
            req.lf = self.lf_ids[r.lf]
            v = r.view
            req.view = _View(float(v[0]), float(v[1]), float(v[2]), float(v[3]), int(round(float(v[4]))))
            img = None
            if req.kind == REQ_RENDER and self.keep_every and getattr(r, "rid", -1) % self.keep_every == 0:
                e = self.pool[r.lf]
                img = torch.empty((e.view_spec.shape[1], e.H, e.W), dtype=torch.float32, device=e.view_spec.device)
                images[r.rid] = img
            req.image_dev = img.data_ptr() if img is not None else None
            req.t_arrival = t0 + r.t_arrival * time_scale
            rid = ctypes.c_int64()
            code = L.fdl_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid))
            if code not in (0, -3):   # FDL_ENOMEM: rejected, still counted
                raise FDLError("fdl_server_submit", code)
            ids.append(rid.value)
        _ok("fdl_server_drain", L.fdl_server_drain(self.h, float(timeout_s)))
        lat = []
        for i in ids:
            st = ctypes.c_int32()
            ms = ctypes.c_double()
            _ok("fdl_server_poll", L.fdl_server_poll(self.h, i, ctypes.byref(st), ctypes.byref(ms)))
            if st.value == REQ_DONE:
                lat.append(ms.value)
        self.kept.update(images)
        return self.stats(np.asarray(lat))

    def stats(self, latency_ms: Optional[np.ndarray] = None) -> ServeStats:
        s = _Summary()
        _ok("fdl_server_stats", _L().fdl_server_stats(self.h, ctypes.byref(s)))
        d = _summary_dict(s, self.budget)
        return ServeStats(int(s.completed), int(s.rejected), latency_ms if latency_ms is not None else np.zeros(0), d,
                          int(s.pool_high_water_bytes), self.budget, float(s.mean_render_batch))

    def layers(self, lf: int) -> torch.Tensor:
        """A copy of the current resident layers of light field ``lf``
        ([n, C, H, W//2+1] complex64, on the device)."""
        e = self.pool[lf]
        n, C = e.d_host.shape[0], e.view_spec.shape[1]
        out = torch.empty((n, C, e.H, e.W // 2 + 1), dtype=torch.complex64, device=e.view_spec.device)
        p = ctypes.c_void_p()
        _ok("fdl_server_layers", _L().fdl_server_layers(self.h, self.lf_ids[lf], ctypes.byref(p)))
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.restype = ctypes.c_int
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        torch.cuda.synchronize(out.device)
        if hip.hipMemcpy(out.data_ptr(), p, out.numel() * 8, 3) != 0:   # device to device
            raise RuntimeError("hipMemcpy of the resident layers failed")
        return out

    def close(self):
        if self.h:
            _ok("fdl_server_destroy", _L().fdl_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(budget: int, layer_bytes, view_bytes, requests, construct_s: float, render_s_per_view: float,
             max_render_batch: int = 16, max_inflight: int = 8, serial: bool = False):
    """The server's scheduling policy on a simulated device (no GPU):
    ``requests`` = (t_arrival, kind, lf) tuples.  Returns (per-request
    [state, batch, t_admit, t_done] rows, summary dict)."""
    L = _L()
    nlf = len(layer_bytes)
    lb = (ctypes.c_size_t * nlf)(*[int(x) for x in layer_bytes])
    vb = (ctypes.c_size_t * nlf)(*[int(x) for x in view_bytes])
    reqs = (_SimRequest * max(1, len(requests)))()
    for i, (t, kind, lf) in enumerate(requests):
        reqs[i] = _SimRequest(float(t), int(kind), int(lf))
    res = (_SimResult * max(1, len(requests)))()
    s = _Summary()
    _ok("fdl_server_simulate", L.fdl_server_simulate(int(budget), int(max_render_batch), int(max_inflight),
                                                     1 if serial else 0, nlf, lb, vb, float(construct_s),
                                                     float(render_s_per_view), reqs, len(requests), res,
                                                     ctypes.byref(s)))
    rows = [(res[i].state, res[i].batch, res[i].t_admit, res[i].t_done) for i in range(len(requests))]
    return rows, _summary_dict(s, budget)
