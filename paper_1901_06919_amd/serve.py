"""Serving loop for mixed construct / render requests with continuous batching.

The server keeps a pool of light fields resident in HBM: their view spectra
(inputs of construction) and their current layer spectra (inputs of
rendering).  Requests arrive open-loop at their scheduled times:

* construct(lf): re-solve the layers of light field ``lf`` (fdl_construct)
  into a fresh buffer on the construct stream; when it completes, the new
  buffer becomes the resident layers of ``lf`` (renders already in flight keep
  reading the old buffer, so results never mix two versions);
* render(lf, view): one view (position, focus, aperture) of light field
  ``lf`` -> fdl_render + fdl_irfft2 -> an image.

Admission is by HBM footprint: each admitted unit of work reserves the bytes
of the buffers it allocates (new layer buffer for a construct; spectrum +
image per rendered view) against ``hbm_budget`` and releases them when its
completion event fires; work that does not fit waits in the queue (the server
never over-commits).  Continuous batching: every pass of the loop retires
finished work, then admits whatever has arrived while memory and in-flight
slots allow -- render requests for the same light field admitted together
share one fdl_render pass over the layers (up to ``max_render_batch`` views)
-- so requests that arrive while others run join the device queues at once;
renders and constructs run on different streams and overlap on the GPU.

Latency = completion observed on the host - scheduled arrival time, so queueing
delay is included (open loop, no coordinated omission).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import construct, irfft2, render, view_records


@dataclasses.dataclass
class PoolEntry:
    view_spec: torch.Tensor      # [m, C, H, W//2+1] complex64 (resident)
    u: torch.Tensor              # [m, 2] f32 device
    d_host: torch.Tensor         # [n] f32 host (construct takes disparities by value)
    d_dev: torch.Tensor          # [n] f32 device (render reads them on the device)
    H: int
    W: int
    lam: float
    eps: float
    reg: int
    layers: Optional[torch.Tensor] = None   # resident layer spectra


@dataclasses.dataclass
class Work:
    kind: str
    reqs: list
    event: torch.cuda.Event
    bytes: int
    lf: int
    outputs: object
    slot: int = -1               # pinned staging slot of the view parameters


@dataclasses.dataclass
class ServeStats:
    completed: int
    duration_s: float
    latency_ms: Dict[str, np.ndarray]
    max_reserved_bytes: int
    hbm_budget: int
    admitted_batches: int
    mean_render_batch: float

    def summary(self) -> dict:
        out = {"completed": self.completed, "throughput_rps": self.completed / max(self.duration_s, 1e-9),
               "max_reserved_MB": self.max_reserved_bytes / 2 ** 20, "budget_MB": self.hbm_budget / 2 ** 20,
               "mean_render_batch": self.mean_render_batch}
        for k, v in self.latency_ms.items():
            if len(v):
                out[f"{k}_p50_ms"] = float(np.percentile(v, 50))
                out[f"{k}_p99_ms"] = float(np.percentile(v, 99))
                out[f"{k}_count"] = int(len(v))
        return out


class FDLServer:
    def __init__(self, pool: List[PoolEntry], hbm_budget: int = 4 << 30, max_render_batch: int = 16,
                 max_inflight: int = 8, keep_outputs_every: int = 0, serial: bool = False):
        """serial=True is the plain baseline: one request at a time, in arrival
        order, on one stream (no batching, no overlap)."""
        self.pool = pool
        self.budget = int(hbm_budget)
        self.max_render_batch = int(max_render_batch)
        self.max_inflight = int(max_inflight)
        self.keep_every = int(keep_outputs_every)
        self.dev = pool[0].view_spec.device
        if serial:
            self.max_render_batch = 1
            self.max_inflight = 1
            one = torch.cuda.Stream(device=self.dev)
            self.render_streams = [one]
            self.construct_stream = one
        else:
            self.render_streams = [torch.cuda.Stream(device=self.dev) for _ in range(2)]
            self.construct_stream = torch.cuda.Stream(device=self.dev)
        self._rr = 0
        self.kept: Dict[int, torch.Tensor] = {}
        # view parameters travel through a ring of pinned host slots (freed when
        # the work that copied them completes), so uploads never block the loop
        nslots = self.max_inflight + 2
        self._pinned = torch.empty((nslots, self.max_render_batch, 5), dtype=torch.float32, pin_memory=True)
        self._dev_views = torch.empty((nslots, self.max_render_batch, 5), dtype=torch.float32, device=self.dev)
        self._free_slots = list(range(nslots))
        for e in pool:
            if e.layers is None:
                e.layers = construct(e.view_spec, e.u, e.d_host, e.H, e.W, e.lam, e.eps, e.reg)
        torch.cuda.synchronize(self.dev)

    # -- footprints -------------------------------------------------------------
    def _layer_bytes(self, e: PoolEntry) -> int:
        return e.layers.numel() * e.layers.element_size()

    def _render_bytes(self, e: PoolEntry, V: int) -> int:
        C = e.view_spec.shape[1]
        return V * C * e.H * ((e.W // 2 + 1) * 8 + e.W * 4)

    # -- work submission --------------------------------------------------------
    def _submit_construct(self, req) -> Work:
        e = self.pool[req.lf]
        with torch.cuda.stream(self.construct_stream):
            out = torch.empty_like(e.layers)
            construct(e.view_spec, e.u, e.d_host, e.H, e.W, e.lam, e.eps, e.reg, out=out)
            ev = torch.cuda.Event()
            ev.record(self.construct_stream)
        return Work("construct", [req], ev, self._layer_bytes(e), req.lf, out)

    def _submit_render(self, lf: int, reqs: list) -> Work:
        e = self.pool[lf]
        s = self.render_streams[self._rr % len(self.render_streams)]
        self._rr += 1
        layers = e.layers              # completed construct output (swapped in after its event fired)
        slot = self._free_slots.pop()
        V = len(reqs)
        host = self._pinned[slot, :V]
        host.copy_(torch.from_numpy(np.stack([r.view for r in reqs]).astype(np.float32)))
        with torch.cuda.stream(s):
            views = self._dev_views[slot, :V]
            views.copy_(host, non_blocking=True)
            rec = view_records(views)
            spec = render(layers, e.d_dev, rec, e.H, e.W)
            img = irfft2(spec, e.H, e.W)
            ev = torch.cuda.Event()
            ev.record(s)
        layers.record_stream(s)
        return Work("render", reqs, ev, self._render_bytes(e, V), lf, img, slot)

    # -- main loop --------------------------------------------------------------
    def run(self, requests, time_scale: float = 1.0) -> ServeStats:
        """Serve ``requests`` (objects with t_arrival, kind, lf, view, and an
        integer ``rid``) in real time; returns latency statistics."""
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        queue: collections.deque = collections.deque()
        inflight: List[Work] = []
        reserved = 0
        max_reserved = 0
        lat = {"render": [], "construct": [], "all": []}
        batches = 0
        rendered = 0
        t0 = time.perf_counter()
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].t_arrival * time_scale <= now:
                queue.append(pending.popleft())
            # retire finished work (in any order)
            still = []
            for w in inflight:
                if w.event.query():
                    done = time.perf_counter() - t0
                    reserved -= w.bytes
                    for r in w.reqs:
                        ms = (done - r.t_arrival * time_scale) * 1e3
                        lat[w.kind].append(ms)
                        lat["all"].append(ms)
                    if w.slot >= 0:
                        self._free_slots.append(w.slot)
                    if w.kind == "construct":
                        self.pool[w.lf].layers = w.outputs        # swap in the new layers
                    elif self.keep_every:
                        for i, r in enumerate(w.reqs):
                            if r.rid % self.keep_every == 0:
                                self.kept[r.rid] = w.outputs[i].clone()
                else:
                    still.append(w)
            inflight = still
            # admit: constructs individually, renders grouped by light field
            progressed = False
            while queue and len(inflight) < self.max_inflight and self._free_slots:
                head = queue[0]
                if head.kind == "construct":
                    need = self._layer_bytes(self.pool[head.lf])
                    if reserved + need > self.budget:
                        break
                    queue.popleft()
                    w = self._submit_construct(head)
                else:
                    lf = head.lf
                    group = [r for r in queue if r.kind == "render" and r.lf == lf][: self.max_render_batch]
                    need = self._render_bytes(self.pool[lf], len(group))
                    while group and reserved + need > self.budget:
                        group.pop()
                        need = self._render_bytes(self.pool[lf], len(group))
                    if not group:
                        break
                    ids = {id(r) for r in group}
                    queue = collections.deque(r for r in queue if id(r) not in ids)
                    w = self._submit_render(lf, group)
                    batches += 1
                    rendered += len(group)
                reserved += w.bytes
                max_reserved = max(max_reserved, reserved)
                inflight.append(w)
                progressed = True
            if not progressed and inflight:
                time.sleep(20e-6)
            elif not progressed and not inflight and pending:
                wait = pending[0].t_arrival * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        torch.cuda.synchronize(self.dev)
        dur = time.perf_counter() - t0
        return ServeStats(len(lat["all"]), dur, {k: np.asarray(v) for k, v in lat.items()}, max_reserved, self.budget,
                          batches, rendered / max(batches, 1))
