#!/usr/bin/env python3
"""Benchmark of the Fourier Disparity Layer hot path on one MI355X.

One step = every stage of the path over one batch of synthetic input,
inputs resident in HBM before the timed region:
  a1  rfft2 of the 81 views x 3 channels (512^2)              -> view spectra
  a2-a6  layer construction, 30 layers, 131,584 bins x 3 ch   -> layer spectra
  a7  render 81 disk-aperture views at the input positions    -> view spectra
  a8  irfft2 of the 243 rendered spectra                      -> images
  a9  calibration loss + leave-one-out adjoint, 4096 bins of the 7x7 / 256^2 /
      16-layer calibration workload
  a10 normalised gradient step on (u, d)
The workload is the 9x9-view, 512x512 RGB, 30-layer light field (jittered
grid, 1/f^2 layers, noise 0.005, lambda 1e-3); its views are synthesised on the
GPU by the library's own forward model (untimed set-up).

value  = layer-construction frequency solves per second of the whole step
         (131,584 bins per step; each bin's system serves the 3 channels).
Also reported: rendered views/s, per-stage times, the roofline of the
dominant kernel (construction, FP64 VALU-bound), and the FP64 CPU oracle
timed on a bounded sample of the same construction.

Measured beside them on the same device: the achievable HBM bandwidth (a
plain 1 GiB device copy) and FP64 VALU rate (fdl_fma64_probe), and, when the
committed rocprofv3 counters match the kernel source, the construction
kernel's executed-instruction issue fraction.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64 (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
PEAK_HBM_GBS = 8000.0


def construct_flops_per_bin(m: int, n: int, C: int) -> int:
    """Algorithmic FP64 flops of one bin with the Toeplitz Gram (d uniform):
    Gram 8 m (n-1), right-hand sides 8 m n C, Cholesky (4/3) n^3, two
    triangular solves 8 n^2 C (1 complex multiply-add = 8 flops)."""
    return 8 * m * (n - 1) + 8 * m * n * C + (4 * n ** 3) // 3 + 8 * n * n * C


def _code_only(text: str) -> str:
    """C++ source with comments removed and whitespace collapsed, so that the
    hash below changes with the code and not with its comments."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the construction kernel's code (comments and layout ignored);
    the committed counter record is used only while it matches."""
    h = hashlib.sha256()
    for name in ("construct_team.h", "construct_plain.h", "construct_c3.hip", "fdl_device.h"):
        with open(os.path.join(ROOT, "paper_1901_06919_amd", "csrc", name)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def load_counters():
    """The committed rocprofv3 counter record of the construction kernel (HBM
    bytes and VALU instructions per launch), or {} when the kernel source
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "construct_9x9_512rgb_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return {}
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return {}
    return rec


def achievable(fdl, dev):
    """Achievable HBM bandwidth (1 GiB device-to-device copy, bytes read +
    written) and FP64 VALU rate (fdl_fma64_probe over 8 blocks per CU)."""
    import torch

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3 / reps

    src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    t_copy = timed(lambda: dst.copy_(src))
    hbm = 2 * src.numel() * 4 / t_copy / 1e9
    del src, dst
    out = torch.empty(256 * 8 * 256, dtype=torch.float64, device=dev)
    flops = [0.0]

    def fma():
        flops[0] = fdl.fma64_probe(out, 4096)

    t_fma = timed(fma)
    return {"hbm_copy_GBs": hbm, "fp64_fma_TFLOPs": flops[0] / t_fma / 1e12}


def cpu_baseline(views_img, u, d, lam, eps, reg, render_views, calib):
    """The FP64 oracle (unchanged), timed on the host cores on the benchmark's
    own inputs, stage by stage: forward DFT of the 243 view images, the
    construction of all 131,584 bins (from the oracle's own spectra), the
    disk-aperture render of 16 of the 81 views (from the oracle's layers)
    and the leave-one-out calibration gradient on 256 of the 4096 sampled
    bins of the calibration workload.  Work is split over worker threads
    (numpy's FFT, LAPACK and ufuncs release the GIL; BLAS pinned to one
    thread each); every stage runs once to warm up, then 5 times, and the
    median is reported, scaled to the benchmark's units."""
    import concurrent.futures

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fdl_oracle as O

    m, C, H, W = views_img.shape
    F = H * (W // 2 + 1)
    workers = max(1, min(16, os.cpu_count() or 1))

    def med(fn):
        fn()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    with threadpool_limits(limits=1), concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        flat = views_img.reshape(m * C, H, W)
        img_chunks = np.array_split(np.arange(m * C), workers)
        spec = np.empty((m * C, H, W // 2 + 1), dtype=np.complex128)

        def fft():
            def one(ix):
                spec[ix] = O.rfft2(flat[ix])
            list(ex.map(one, img_chunks))

        t_fft = med(fft)
        spec4 = spec.reshape(m, C, H, W // 2 + 1)
        bins = np.array_split(np.arange(F), workers * 4)
        layers = np.empty((len(d), C, F), dtype=np.complex128)

        def construct():
            def one(ix):
                layers[:, :, ix] = O.construct(spec4, u, d, H, W, lam, eps, reg, freq_index=ix)
            list(ex.map(one, bins))

        t_con = med(construct)
        lay4 = layers.reshape(len(d), C, H, W // 2 + 1)
        rv = render_views[:16]

        def render():
            list(ex.map(lambda v: O.render(lay4, d, rv[v:v + 1], H, W), range(rv.shape[0])))

        t_ren = med(render)
        (cs, cu, cd, cH, cW, clam, ceps, creg, cidx) = calib
        sample = np.array_split(cidx[:256], workers)

        def calib_grad():
            list(ex.map(lambda ix: O.calib_loss_grad(cs, cu, cd, cH, cW, clam, ceps, creg, O.LOSS_LOO, ix), sample))

        t_cal = med(calib_grad) * (cidx.shape[0] / 256.0)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": F / t_con, "unit": "bins/s", "cores": workers, "kind": "oracle",
            "sample": (f"FP64 oracle on the benchmark's inputs, {workers} threads, median of 5 after a warm-up: "
                       f"rfft2 of {m * C} images {H}x{W} ({t_fft:.2f} s), construction of all {F} bins "
                       f"({t_con:.2f} s), disk render of {rv.shape[0]} of the views ({t_ren:.2f} s), LOO gradient on "
                       f"256 of {cidx.shape[0]} bins of the 7x7/256^2 calibration workload (scaled)"),
            "stages": {"rfft2_images_per_s": m * C / t_fft, "construct_bins_per_s": F / t_con,
                       "render_views_per_s": rv.shape[0] / t_ren, "calib_grad_steps_per_s": 1.0 / t_cal},
            "host_cpus": os.cpu_count(), "cpu_model": model}


def systems(fdl, synth, dev, serve_seconds: float):
    """Batching: 64 uneven light fields (grids 3..9, 128^2..512^2 incl. 384,
    8..32 layers, 1 channel) -- plain per-light-field calls vs the autotuned
    batched plan vs the plan replayed from a HIP graph.  Serving: open-loop
    Poisson stream at 200 req/s (20% construct, 80% render) against 8 resident
    9x9 / 512^2 RGB / 30-layer light fields, HBM-footprint admission."""
    import numpy as np
    import torch

    out = {}
    g = torch.Generator(device=dev).manual_seed(3)
    items = []
    print("bench: generating the 64 uneven light fields", file=sys.stderr, flush=True)
    for i in range(64):
        # instance i of the uneven-light-field generator (seed 3000 + i): its
        # views are rendered from its layers at its positions (untimed set-up)
        lf = synth.uneven_light_field(i)
        side, n = lf.H, lf.n
        u = torch.from_numpy(lf.u).to(dev)
        m = u.shape[0]
        d = torch.from_numpy(lf.d)
        pin = torch.zeros((m, 5), dtype=torch.float32)
        pin[:, 0:2] = torch.from_numpy(lf.u)
        lsp = fdl.rfft2(torch.from_numpy(lf.layers).to(dev))
        img_i = fdl.irfft2(fdl.render(lsp, d.to(dev), fdl.view_records(pin.to(dev)), side, side), side, side)
        spec = fdl.rfft2(img_i + torch.from_numpy(lf.noise).to(dev))
        del lsp, img_i
        items.append(dict(view_spec=spec, u=u, d=d.to(dev), d_host=d, H=side, W=side, lam=1e-2, eps=1e-3, reg=0,
                          out=torch.empty((n, 1, side, side // 2 + 1), dtype=torch.complex64, device=dev)))
    bins = sum(it["H"] * (it["W"] // 2 + 1) for it in items)

    def plain():
        for it in items:
            fdl.construct(it["view_spec"], it["u"], it["d_host"], it["H"], it["W"], it["lam"], it["eps"], it["reg"],
                          out=it["out"])

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    t_plain = timed(plain)
    plan = fdl.BatchPlan(items, mode=1)
    plan.autotune(reps=2)
    t_batch = timed(plan.execute)
    gr = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream(device=dev)
    st.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(st):
        with torch.cuda.graph(gr, stream=st):
            plan.execute()
    torch.cuda.current_stream(dev).wait_stream(st)
    t_graph = timed(gr.replay)
    out["batching"] = {"light_fields": 64, "bins": bins, "plain_ms": t_plain, "batched_ms": t_batch,
                       "graph_ms": t_graph, "speedup_vs_plain": t_plain / min(t_batch, t_graph),
                       "tuning": plan.tuning(), "launches": plan.launches}
    plan.close()
    del items
    torch.cuda.empty_cache()

    # calibration loop (7x7 / 256^2 / 16 layers, LOO loss, 4096 bins per step):
    # 200 steps issued eagerly vs the same steps captured once in a HIP graph
    lfc, u5_0, d5_0 = synth.lf_7x7_256_calib()
    l5 = fdl.rfft2(torch.from_numpy(lfc.layers).to(dev))
    p5 = torch.zeros((lfc.m, 5), dtype=torch.float32)
    p5[:, 0:2] = torch.from_numpy(lfc.u)
    v5 = fdl.irfft2(fdl.render(l5, torch.from_numpy(lfc.d).to(dev), fdl.view_records(p5.to(dev)), lfc.H, lfc.W),
                    lfc.H, lfc.W) + torch.from_numpy(lfc.noise).to(dev)
    b5 = fdl.rfft2(v5)
    F5 = lfc.H * (lfc.W // 2 + 1)
    nsteps = 200
    rng = np.random.default_rng(5)
    subs = torch.from_numpy(np.stack([synth.frequency_subset(F5, 4096, rng) for _ in range(nsteps)])).to(dev)
    u5 = torch.from_numpy(u5_0).to(dev)
    d5 = torch.from_numpy(d5_0).to(dev)
    g5 = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((lfc.m, 2), dtype=torch.float64, device=dev),
          torch.empty(lfc.n, dtype=torch.float64, device=dev))
    ws = torch.empty(fdl.calib_workspace_bytes(lfc.m, lfc.n, 4096), dtype=torch.uint8, device=dev)

    def loop():
        for i in range(nsteps):
            fdl.calib_grad(b5, u5, d5, lfc.H, lfc.W, lfc.lam, lfc.eps, lfc.reg, fdl.LOSS_LOO, subs[i], out=g5, ws=ws)
            fdl.gd_step(u5, d5, g5[1], g5[2], 0.2, 1e-6)

    t_eager = timed(loop, reps=2)
    gr5 = torch.cuda.CUDAGraph()
    st5 = torch.cuda.Stream(device=dev)
    st5.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(st5):
        with torch.cuda.graph(gr5, stream=st5):
            loop()
    torch.cuda.current_stream(dev).wait_stream(st5)
    t_graph5 = timed(gr5.replay, reps=2)
    out["calibration"] = {"steps": nsteps, "eager_steps_per_s": nsteps / (t_eager * 1e-3),
                          "graph_steps_per_s": nsteps / (t_graph5 * 1e-3), "graph_speedup": t_eager / t_graph5}
    del gr5, b5, subs, ws

    # relaxed model (free shift per view and layer) on the same light field,
    # whose views now follow rank-1 shifts plus sparse deviations: 200 relaxed
    # gradient steps (FIT objective, 4096 bins each) from the rank-1 shifts,
    # then the denoising pass (layers over all bins with the final shifts, the
    # 49 input views rendered back, inverse DFT)
    P_true = (torch.from_numpy(lfc.d)[None, :, None] * torch.from_numpy(lfc.u)[:, None, :]
              + torch.from_numpy(synth.shift_deviations(lfc.m, lfc.n, np.random.default_rng(57))))
    P_true = P_true.to(dev).contiguous()
    vr = fdl.irfft2(fdl.render_relaxed(l5, P_true, lfc.H, lfc.W), lfc.H, lfc.W) + torch.from_numpy(lfc.noise).to(dev)
    br = fdl.rfft2(vr)
    P0 = (torch.from_numpy(lfc.d)[None, :, None] * torch.from_numpy(lfc.u)[:, None, :]).to(dev).contiguous()
    Pw = P0.clone()
    rsteps = 200
    rsubs = torch.from_numpy(np.stack([synth.frequency_subset(F5, 4096, rng) for _ in range(rsteps)])).to(dev)
    gr_out = (torch.empty(1, dtype=torch.float64, device=dev),
              torch.empty((lfc.m, lfc.n, 2), dtype=torch.float64, device=dev))
    wsr = torch.empty(fdl.calib_relaxed_workspace_bytes(lfc.m, lfc.n, 4096), dtype=torch.uint8, device=dev)

    def relaxed_loop():
        Pw.copy_(P0)
        for i in range(rsteps):
            fdl.calib_grad_relaxed(br, Pw, lfc.H, lfc.W, lfc.lam, lfc.eps, lfc.reg, fdl.LOSS_FIT, rsubs[i], out=gr_out,
                                   ws=wsr)
            fdl.gd_step_relaxed(Pw, gr_out[1], 0.2, 1e-6)

    lay_r = torch.empty((lfc.n, 1, lfc.H, lfc.W // 2 + 1), dtype=torch.complex64, device=dev)
    out_r = torch.empty((lfc.m, 1, lfc.H, lfc.W // 2 + 1), dtype=torch.complex64, device=dev)
    img_r = torch.empty((lfc.m, 1, lfc.H, lfc.W), dtype=torch.float32, device=dev)

    def denoise():
        fdl.construct_relaxed(br, Pw, lfc.H, lfc.W, lfc.lam, lfc.eps, lfc.reg, out=lay_r)
        fdl.render_relaxed(lay_r, Pw, lfc.H, lfc.W, out=out_r)
        fdl.irfft2(out_r, lfc.H, lfc.W, out=img_r)

    t_rloop = timed(relaxed_loop, reps=2)
    t_den = timed(denoise, reps=5)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(5):
        fdl.construct_relaxed(br, Pw, lfc.H, lfc.W, lfc.lam, lfc.eps, lfc.reg, out=lay_r)
    ev[1].record()
    for _ in range(5):
        fdl.render_relaxed(lay_r, Pw, lfc.H, lfc.W, out=out_r)
    ev[2].record()
    torch.cuda.synchronize()
    # denoising error against the noise-free relaxed-model views, with the
    # fitted shifts, the rank-1 start and the true shifts
    clean = vr - torch.from_numpy(lfc.noise).to(dev)

    def err(img):
        return float(torch.linalg.vector_norm(img - clean) / torch.linalg.vector_norm(clean))

    err_in = err(vr)
    err_out = err(img_r)
    P_fit = Pw.clone()
    errs = {}
    for name, Pq in (("rank1_start", P0), ("true_shifts", P_true)):
        Pw.copy_(Pq)
        denoise()
        errs[name] = err(img_r)
    torch.cuda.synchronize()
    shift_err = float(torch.linalg.vector_norm(P_fit - P_true) / torch.linalg.vector_norm(P0 - P_true))
    out["relaxed"] = {"workload": "7x7 views 256x256, 16 layers, rank-1 shifts + 10% deviations N(0, 0.5^2), "
                                  "noise sigma 0.01; 200 FIT steps of 4096 bins, then construct + render 49 views",
                      "steps_per_s": rsteps / (t_rloop * 1e-3), "denoise_ms": t_den,
                      "construct_relaxed_ms": ev[0].elapsed_time(ev[1]) / 5,
                      "render_relaxed_ms": ev[1].elapsed_time(ev[2]) / 5,
                      "construct_bins_per_s": F5 / (ev[0].elapsed_time(ev[1]) / 5 * 1e-3),
                      "rel_err_input": err_in, "rel_err_denoised": err_out,
                      "rel_err_denoised_rank1_shifts": errs["rank1_start"],
                      "rel_err_denoised_true_shifts": errs["true_shifts"],
                      "shift_err_vs_start": shift_err}
    del br, vr, rsubs, wsr, lay_r, out_r, img_r
    torch.cuda.empty_cache()

    if serve_seconds > 0:
        from paper_1901_06919_amd.serve import FDLServer, PoolEntry
        lfb = synth.lf_9x9_512_rgb(H=8, W=8)          # positions / disparities only
        pool = []
        d = torch.from_numpy(lfb.d)
        for i in range(8):
            spec = torch.randn((81, 3, 512, 257), dtype=torch.complex64, device=dev, generator=g)
            pool.append(PoolEntry(spec, torch.from_numpy(lfb.u).to(dev), d, d.to(dev), 512, 512, 1e-3, 1e-3, 0))
        # the serving workload: 200 req/s for serve_seconds (60 s: about 12,000
        # requests); a shorter stream at 1000 req/s shows the tail under load
        for rate, seconds in ((200.0, serve_seconds), (1000.0, min(serve_seconds, 6.0))):
            reqs = synth.serving_requests(rate=rate, duration=seconds, pool=8, seed=4)
            res = {"requests": len(reqs), "seconds": seconds}
            for name, serial in (("continuous", False), ("serial_fifo", True)):
                srv = FDLServer(pool, hbm_budget=2 << 30, max_render_batch=16, max_inflight=8, serial=serial)
                srv.run(reqs[: max(1, len(reqs) // 20)])          # warm-up slice
                res[name] = srv.run(reqs, timeout_s=seconds + 120.0).summary()
                srv.close()
                print(f"bench: serving {rate:.0f} req/s {name}: p50 {res[name].get('all_p50_ms', 0):.3f} ms "
                      f"p99 {res[name].get('all_p99_ms', 0):.3f} ms", file=sys.stderr, flush=True)
            out["serving" if rate == 200.0 else f"serving_{int(rate)}rps"] = res
        del pool
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-systems", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the FDL path runs on one MI355X; more than one GPU is not supported "
              "(the sharding is designed, not implemented). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_06919_amd as fdl
    from paper_1901_06919_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # ---- set-up (untimed): synthetic workload resident in HBM ----
    lfb = synth.lf_9x9_512_rgb()
    H, W = lfb.H, lfb.W
    m, n, C = lfb.m, lfb.n, lfb.C
    F = H * (W // 2 + 1)
    layers = torch.from_numpy(lfb.layers).to(dev)
    u = torch.from_numpy(lfb.u).to(dev)
    d_dev = torch.from_numpy(lfb.d).to(dev)
    d_host = torch.from_numpy(lfb.d).clone()
    pin = torch.zeros((m, 5), dtype=torch.float32)
    pin[:, 0:2] = torch.from_numpy(lfb.u)
    pin_rec = fdl.view_records(pin.to(dev))
    views_rec = fdl.view_records(torch.from_numpy(lfb.views).to(dev))
    lspec = fdl.rfft2(layers)
    vspec = fdl.render(lspec, d_dev, pin_rec, H, W)
    views = fdl.irfft2(vspec, H, W) + torch.from_numpy(lfb.noise).to(dev)
    del lspec, vspec, layers

    lfc, u5_0, d5_0 = synth.lf_7x7_256_calib()
    l5 = fdl.rfft2(torch.from_numpy(lfc.layers).to(dev))
    p5 = torch.zeros((lfc.m, 5), dtype=torch.float32)
    p5[:, 0:2] = torch.from_numpy(lfc.u)
    v5 = fdl.irfft2(fdl.render(l5, torch.from_numpy(lfc.d).to(dev), fdl.view_records(p5.to(dev)), lfc.H, lfc.W),
                    lfc.H, lfc.W) + torch.from_numpy(lfc.noise).to(dev)
    b5 = fdl.rfft2(v5)
    del l5, v5
    u5 = torch.from_numpy(u5_0).to(dev)
    d5 = torch.from_numpy(d5_0).to(dev)
    F5 = lfc.H * (lfc.W // 2 + 1)
    Q5 = 4096
    rng = np.random.default_rng(5)
    nsub = args.warmup + args.steps
    subsets = torch.from_numpy(np.stack([synth.frequency_subset(F5, Q5, rng) for _ in range(nsub)])).to(dev)
    g_out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((lfc.m, 2), dtype=torch.float64, device=dev),
             torch.empty(lfc.n, dtype=torch.float64, device=dev))
    ws5 = torch.empty(fdl.calib_workspace_bytes(lfc.m, lfc.n, Q5), dtype=torch.uint8, device=dev)

    spec = torch.empty((m, C, H, W // 2 + 1), dtype=torch.complex64, device=dev)
    lay = torch.empty((n, C, H, W // 2 + 1), dtype=torch.complex64, device=dev)
    rend = torch.empty((m, C, H, W // 2 + 1), dtype=torch.complex64, device=dev)
    img = torch.empty((m, C, H, W), dtype=torch.float32, device=dev)
    V = int(views_rec.shape[0])

    stages = ["rfft2", "construct", "render", "irfft2", "calib_grad", "gd_step"]
    ev = {s: [] for s in stages}

    def step(i, record):
        marks = []

        def mark():
            if record:
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                marks.append(e)

        mark()
        fdl.rfft2(views, out=spec)
        mark()
        fdl.construct(spec, u, d_host, H, W, lfb.lam, lfb.eps, lfb.reg, out=lay)
        mark()
        fdl.render(lay, d_dev, views_rec, H, W, out=rend)
        mark()
        fdl.irfft2(rend, H, W, out=img)
        mark()
        fdl.calib_grad(b5, u5, d5, lfc.H, lfc.W, lfc.lam, lfc.eps, lfc.reg, fdl.LOSS_LOO, subsets[i], out=g_out, ws=ws5)
        mark()
        fdl.gd_step(u5, d5, g_out[1], g_out[2], 0.2, 1e-6)
        mark()
        if record:
            for s, a, b in zip(stages, marks[:-1], marks[1:]):
                ev[s].append((a, b))

    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    stage_us = {s: float(np.mean([a.elapsed_time(b) for a, b in ev[s]]) * 1e3) for s in stages}
    step_ms = [ev[stages[0]][i][0].elapsed_time(ev[stages[-1]][i][1]) for i in range(args.steps)]

    flops = construct_flops_per_bin(m, n, C) * F
    t_con = stage_us["construct"] * 1e-6
    achieved = flops / t_con / 1e12
    cnt = load_counters()
    ach = achievable(fdl, dev)
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": cnt.get("hbm_bytes_per_launch"),
            "kernel": "k_construct<3,true,30>", "flops_per_launch": flops,
            "achievable_peak": ach["fp64_fma_TFLOPs"], "frac_of_achievable": achieved / ach["fp64_fma_TFLOPs"]}
    if cnt:
        # traffic and instruction counts are not observed in this run: they
        # come from the committed counter record of the same kernel source
        roof["counters_source"] = ("committed rocprofv3 record profiles/construct_9x9_512rgb_traffic.json "
                                   f"(kernel source {cnt.get('kernel_source_hash')}, {cnt.get('source')})")
    if cnt.get("valu_insts_per_launch"):
        # time the counted VALU instructions need at one wave instruction per
        # 4 cycles on each of the 1024 SIMDs at 2.4 GHz, over the measured time
        t_issue = cnt["valu_insts_per_launch"] * 4.0 / (1024 * 2.4e9)
        roof["executed_valu_insts"] = cnt["valu_insts_per_launch"]
        roof["executed_issue_frac"] = t_issue / t_con

    # wider path (inputs with their own apertures): a hybrid focal-stack input of
    # 9 centre disk views (radius 1.5, focus through the scene) + 3x3
    # sub-aperture views, 30 layers, 512^2 RGB, same spectra layout
    hv = np.zeros((18, 5), np.float32)
    hv[:9, 2] = np.linspace(-3, 3, 9)
    hv[:9, 3] = 1.5
    hv[:9, 4] = 1
    gg = np.arange(-1, 2)
    hy, hx = np.meshgrid(gg, gg, indexing="ij")
    hv[9:, 0] = hx.ravel()
    hv[9:, 1] = hy.ravel()
    hrec = fdl.view_records(torch.from_numpy(hv).to(dev))
    hspec = spec[:18]
    fdl.construct_views(hspec, hrec, d_host, H, W, lfb.lam, lfb.eps, lfb.reg, out=lay)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        fdl.construct_views(hspec, hrec, d_host, H, W, lfb.lam, lfb.eps, lfb.reg, out=lay)
    e1.record()
    torch.cuda.synchronize()
    t_views = e0.elapsed_time(e1) / 5
    views_row = {"workload": "18 input views (9 centre disks r=1.5 focused over [-3,3] + 3x3 pinholes), "
                             "30 layers, 512x512 RGB", "ms": t_views, "bins_per_s": F / (t_views * 1e-3)}

    # drawn aperture: the 81 rendered views of the step with a hexagonal
    # aperture drawn as a 63x63 image, spectrum table zero-padded 8x (504^2),
    # against the same views with the analytic disk
    S_ap, pad_ap = 63, 8
    cc = (np.arange(S_ap) - (S_ap - 1) / 2) * (2.0 / S_ap)
    ax, ay = np.abs(cc)[None, :], np.abs(cc)[:, None]
    hexa = ((ay <= math.sqrt(3) / 2) & (math.sqrt(3) * ax + ay <= math.sqrt(3))).astype(np.float32)
    img_ap = torch.from_numpy(hexa).to(dev)
    tab = fdl.aperture_table(img_ap, pad_ap)
    hv_img = torch.from_numpy(lfb.views).clone()
    hv_img[:, 4] = fdl.AP_IMAGE
    rec_img = fdl.view_records(hv_img.to(dev))
    fdl.render_tabulated(lay, d_dev, rec_img, H, W, tab, S_ap, out=rend)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(5):
        fdl.aperture_table(img_ap, pad_ap, out=tab)
    e[1].record()
    for _ in range(5):
        fdl.render_tabulated(lay, d_dev, rec_img, H, W, tab, S_ap, out=rend)
    e[2].record()
    for _ in range(5):
        fdl.render(lay, d_dev, views_rec, H, W, out=rend)
    e[3].record()
    torch.cuda.synchronize()
    # finite-region view regulariser (camera-plane square of side 8, the
    # extent of the 9x9 grid) on the benchmark construction
    fdl.rfft2(views, out=spec)
    fdl.construct_region(spec, u, d_host, H, W, lfb.lam, lfb.eps, 8.0, out=lay)
    torch.cuda.synchronize()
    er = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    er[0].record()
    for _ in range(5):
        fdl.construct_region(spec, u, d_host, H, W, lfb.lam, lfb.eps, 8.0, out=lay)
    er[1].record()
    torch.cuda.synchronize()
    t_reg = er[0].elapsed_time(er[1]) / 5
    region_row = {"workload": "benchmark construction (9x9 views, 512x512 RGB, 30 layers) with the view "
                              "regulariser over the camera-plane square of side 8", "ms": t_reg,
                  "bins_per_s": F / (t_reg * 1e-3)}

    # the small configuration (5x5 views, 128^2, 1 channel, 8 layers, 16 pinhole
    # renders): the whole path as plain launches and replayed from a HIP graph
    lf1 = synth.lf_5x5_128()
    H1, W1 = lf1.H, lf1.W
    u1 = torch.from_numpy(lf1.u).to(dev)
    d1h = torch.from_numpy(lf1.d).clone()
    d1 = d1h.to(dev)
    p1 = torch.zeros((lf1.m, 5), dtype=torch.float32)
    p1[:, 0:2] = torch.from_numpy(lf1.u)
    l1 = fdl.rfft2(torch.from_numpy(lf1.layers).to(dev))
    img1 = fdl.irfft2(fdl.render(l1, d1, fdl.view_records(p1.to(dev)), H1, W1), H1, W1) + \
        torch.from_numpy(lf1.noise).to(dev)
    r1 = fdl.view_records(torch.from_numpy(lf1.views).to(dev))
    V1 = int(r1.shape[0])
    spec1 = torch.empty((lf1.m, lf1.C, H1, W1 // 2 + 1), dtype=torch.complex64, device=dev)
    lay1 = torch.empty((lf1.n, lf1.C, H1, W1 // 2 + 1), dtype=torch.complex64, device=dev)
    rsp1 = torch.empty((V1, lf1.C, H1, W1 // 2 + 1), dtype=torch.complex64, device=dev)
    out1 = torch.empty((V1, lf1.C, H1, W1), dtype=torch.float32, device=dev)

    def small_step():
        fdl.rfft2(img1, out=spec1)
        fdl.construct(spec1, u1, d1h, H1, W1, lf1.lam, lf1.eps, lf1.reg, out=lay1)
        fdl.render(lay1, d1, r1, H1, W1, out=rsp1)
        fdl.irfft2(rsp1, H1, W1, out=out1)

    def timed_ms(fn, reps=50):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_small = timed_ms(small_step)
    g1 = torch.cuda.CUDAGraph()
    s1 = torch.cuda.Stream(device=dev)
    s1.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s1):
        with torch.cuda.graph(g1, stream=s1):
            small_step()
    torch.cuda.current_stream(dev).wait_stream(s1)
    t_small_g = timed_ms(g1.replay)
    e_s = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    fdl.rfft2(img1, out=spec1)
    e_s[0].record()
    for _ in range(20):
        fdl.construct(spec1, u1, d1h, H1, W1, lf1.lam, lf1.eps, lf1.reg, out=lay1)
    e_s[1].record()
    torch.cuda.synchronize()
    small_row = {"workload": "5x5 views, 128x128, 1 channel, 8 layers linspace(-2,2), 16 pinhole renders "
                             "(rfft2, construct, render, irfft2)",
                 "plain_ms": t_small, "graph_ms": t_small_g, "graph_speedup": t_small / t_small_g,
                 "construct_us": e_s[0].elapsed_time(e_s[1]) / 20 * 1e3,
                 "bins_per_s_graph": H1 * (W1 // 2 + 1) / (t_small_g * 1e-3)}
    del g1, l1, img1, spec1, lay1, rsp1, out1

    drawn_row = {"workload": f"{V} views of 512x512 RGB, 30 layers, drawn hexagonal aperture {S_ap}x{S_ap} "
                             f"padded to {S_ap * pad_ap}^2, bilinear reads",
                 "table_ms": e[0].elapsed_time(e[1]) / 5, "render_ms": e[1].elapsed_time(e[2]) / 5,
                 "analytic_render_ms": e[2].elapsed_time(e[3]) / 5}

    views_host = views.cpu().numpy() if not args.no_cpu_baseline else None
    b5_host = b5.cpu().numpy().astype(np.complex128) if not args.no_cpu_baseline else None
    lfc_u0, lfc_d0 = u5_0.astype(np.float64), d5_0.astype(np.float64)
    subsets_host = subsets.cpu().numpy()
    sysres = None
    if not args.no_systems:
        del spec, lay, rend, img, views, b5
        torch.cuda.empty_cache()
        sysres = systems(fdl, synth, dev, args.serve_seconds)

    base = None
    if not args.no_cpu_baseline:
        print("bench: timing the FP64 oracle on the host cores", file=sys.stderr, flush=True)
        calib_in = (b5_host, lfc_u0, lfc_d0, lfc.H, lfc.W, lfc.lam, lfc.eps, lfc.reg, subsets_host[0])
        base = cpu_baseline(views_host, lfb.u.astype(np.float64), lfb.d.astype(np.float64), lfb.lam, lfb.eps, lfb.reg,
                            lfb.views.astype(np.float64), calib_in)
        gpu_rates = {"rfft2_images_per_s": m * C / (stage_us["rfft2"] * 1e-6),
                     "construct_bins_per_s": F / (stage_us["construct"] * 1e-6),
                     "render_views_per_s": V / (stage_us["render"] * 1e-6),
                     "calib_grad_steps_per_s": 1.0 / (stage_us["calib_grad"] * 1e-6)}
        base["gpu_stages"] = gpu_rates
        base["gpu_over_cpu"] = {k: gpu_rates[k] / base["stages"][k] for k in gpu_rates}

    out = {
        "metric": "layer-construction frequency solves/s",
        "value": F / (ms_per_step * 1e-3),
        "unit": "bins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "9x9 views, 512x512 RGB, 30 layers linspace(-3,3), 81 disk renders; "
                               "calibration rows on 7x7 views 256x256, 16 layers, 4096 bins",
                   "bins": F, "views": m, "layers": n, "channels": C, "rendered_views": V},
        "rendered_views_per_s": V / (ms_per_step * 1e-3),
        "median_step_ms": float(np.median(step_ms)),
        "stage_us": stage_us,
        "achievable": ach,
        "construct_views": views_row,
        "drawn_aperture": drawn_row,
        "construct_region": region_row,
        "small_config": small_row,
        "roofline": roof,
        "cpu_baseline": base,
        "construct_bins_per_s": F / (stage_us["construct"] * 1e-6),
    }
    if sysres is not None:
        out["batching"] = sysres.get("batching")
        sv = sysres.get("serving")
        if sv:
            out["serving"] = sv
            out["p50_request_ms"] = sv["continuous"].get("all_p50_ms")
            out["p99_request_ms"] = sv["continuous"].get("all_p99_ms")
        if sysres.get("serving_1000rps"):
            out["serving_1000rps"] = sysres["serving_1000rps"]
        if sysres.get("calibration"):
            out["calibration"] = sysres["calibration"]
        if sysres.get("relaxed"):
            out["relaxed"] = sysres["relaxed"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
