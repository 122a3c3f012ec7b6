"""Batching pattern: many uneven light fields in one plan (flat, flat single
and persistent launches, autotuned, HIP-graph replayed) must reproduce the
plain per-light-field fdl_construct calls, and the oracle on sampled bins."""
import numpy as np
import pytest
import torch

from oracle import fdl_oracle as O
from paper_1901_06919_amd import synth

pytestmark = pytest.mark.gpu


def fdl():
    import paper_1901_06919_amd as m
    return m


def _items(count, sizes=(128, 256, 384, 512), seed=0):
    """Uneven light fields shaped like the 64-instance batching workload
    (grids 3..9, sides from `sizes`, 8..32 layers), random view spectra."""
    rng = np.random.default_rng(seed)
    items = []
    for i in range(count):
        g, side, n = synth.uneven_light_field_shape(i, sizes=sizes)
        u = synth.centered_grid_positions(g)
        m = u.shape[0]
        H = W = side
        spec = (rng.standard_normal((m, 1, H, W // 2 + 1)) + 1j * rng.standard_normal((m, 1, H, W // 2 + 1)))
        spec = spec.astype(np.complex64)
        d = np.linspace(-2.0, 2.0, n).astype(np.float32)
        items.append(dict(spec_np=spec, u_np=u, d_np=d, H=H, W=W, lam=1e-2, eps=1e-3, reg=0,
                          view_spec=torch.from_numpy(spec).cuda(), u=torch.from_numpy(u).cuda(),
                          d=torch.from_numpy(d).cuda(),
                          out=torch.empty((n, 1, H, W // 2 + 1), dtype=torch.complex64, device="cuda")))
    return items


def _plain(items):
    return [fdl().construct(it["view_spec"], it["u"], it["d"], it["H"], it["W"], it["lam"], it["eps"], it["reg"])
            for it in items]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_batched_matches_plain_calls(mode):
    items = _items(12, sizes=(128, 256, 384), seed=mode)
    ref = _plain(items)
    plan = fdl().BatchPlan(items, mode=mode)
    plan.execute()
    torch.cuda.synchronize()
    worst = 0.0
    exact = True
    for it, r in zip(items, ref):
        diff = (it["out"] - r).abs().max().item()
        exact &= diff == 0.0
        e = O.rel_l2(it["out"].cpu().numpy(), r.cpu().numpy())
        worst = max(worst, e) if e == e else float("inf")   # NaN counts as a failure
    print(f"mode {mode}: launches {plan.launches}, worst rel_l2 vs plain {worst:.2e}, bitwise {exact}")
    assert worst < 1e-6
    # a second execution (queue reset by the last block) gives the same result
    for it in items:
        it["out"].zero_()
    plan.execute()
    torch.cuda.synchronize()
    for it, r in zip(items, ref):
        assert O.rel_l2(it["out"].cpu().numpy(), r.cpu().numpy()) < 1e-6


def _mixed_items(seed):
    """A batch that spans every batched kernel class: 1, 2, 3 and 4 channels,
    uniform and general disparities, exact and jittered view grids (lattice
    and table paths), 5 to 32 layers."""
    rng = np.random.default_rng(seed)
    items = []
    for i, (g, side, n, C, uniform, jitter) in enumerate([
            (3, 64, 5, 1, True, False), (4, 96, 12, 2, True, True), (5, 64, 20, 3, False, True),
            (3, 128, 32, 4, True, False), (5, 96, 27, 1, False, False), (4, 64, 16, 4, False, True),
            (3, 96, 30, 3, True, True), (2, 64, 8, 2, False, False), (4, 128, 24, 1, True, True),
            (3, 64, 29, 4, True, True)]):
        u = synth.centered_grid_positions(g)
        if jitter:
            u = (u + rng.uniform(-0.05, 0.05, u.shape)).astype(np.float32)
        m = u.shape[0]
        H = W = side
        spec = (rng.standard_normal((m, C, H, W // 2 + 1)) + 1j * rng.standard_normal((m, C, H, W // 2 + 1)))
        spec = spec.astype(np.complex64)
        d = (np.linspace(-2.0, 2.0, n) if uniform else np.sort(rng.uniform(-2.0, 2.0, n))).astype(np.float32)
        items.append(dict(spec_np=spec, u_np=u, d_np=d, H=H, W=W, lam=1e-2, eps=1e-3, reg=0,
                          view_spec=torch.from_numpy(spec).cuda(), u=torch.from_numpy(u).cuda(),
                          d=torch.from_numpy(d).cuda(),
                          out=torch.empty((n, C, H, W // 2 + 1), dtype=torch.complex64, device="cuda")))
    return items


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_batched_mixed_classes_match_plain_calls(mode):
    items = _mixed_items(40 + mode)
    print(f"mixed batch mode {mode}: {len(items)} light fields", flush=True)
    ref = _plain(items)
    plan = fdl().BatchPlan(items, mode=mode)
    plan.execute()
    torch.cuda.synchronize()
    worst = 0.0
    for it, r in zip(items, ref):
        e = O.rel_l2(it["out"].cpu().numpy(), r.cpu().numpy())
        worst = max(worst, e) if e == e else float("inf")   # NaN counts as a failure
    print(f"  launches {plan.launches}, worst rel_l2 vs plain {worst:.2e}")
    assert worst < 1e-6
    # one light field of each kind against the oracle on a few bins
    rng = np.random.default_rng(7)
    for it in items[:4]:
        F = it["H"] * (it["W"] // 2 + 1)
        idx = np.unique(np.concatenate([[0, F - 1], rng.choice(F, 24, replace=False)]))
        refo = O.construct(it["spec_np"].astype(np.complex128), it["u_np"].astype(np.float64),
                           it["d_np"].astype(np.float64), it["H"], it["W"], it["lam"], it["eps"], it["reg"],
                           freq_index=idx)
        n, C = it["out"].shape[:2]
        got = it["out"].cpu().numpy().reshape(n, C, F)[:, :, idx]
        assert O.rel_l2(got, refo) < 1e-4


def test_batched_matches_oracle_on_sampled_bins():
    items = _items(6, sizes=(128, 384, 512), seed=11)
    plan = fdl().BatchPlan(items, mode=1)
    plan.execute()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for it in items:
        H, W = it["H"], it["W"]
        F = H * (W // 2 + 1)
        idx = np.sort(rng.choice(F, 256, replace=False))
        ref = O.construct(it["spec_np"].astype(np.complex128), it["u_np"].astype(np.float64),
                          it["d_np"].astype(np.float64), H, W, it["lam"], it["eps"], it["reg"], freq_index=idx)
        got = it["out"].cpu().numpy().reshape(len(it["d_np"]), 1, -1)[:, :, idx]
        err = O.rel_l2(got, ref)
        print(f"  H={H} m={it['u_np'].shape[0]} n={len(it['d_np'])}: rel_l2 {err:.2e}")
        assert err < 1e-4


def test_batched_graph_replay_matches_eager():
    items = _items(10, sizes=(128, 256), seed=21)
    plan = fdl().BatchPlan(items, mode=1)
    plan.execute()
    torch.cuda.synchronize()
    eager = [it["out"].clone() for it in items]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.execute()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for it in items:
            it["out"].zero_()            # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for it, e in zip(items, eager):
            assert torch.equal(it["out"], e), f"replay {rep} differs"


def test_autotune_keeps_results():
    items = _items(8, sizes=(128, 256), seed=31)
    ref = _plain(items)
    plan = fdl().BatchPlan(items, mode=0)
    ms = plan.autotune(reps=2)
    print(f"autotuned: {plan.tuning()} in {ms:.3f} ms")
    plan.execute()
    torch.cuda.synchronize()
    for it, r in zip(items, ref):
        assert O.rel_l2(it["out"].cpu().numpy(), r.cpu().numpy()) < 1e-6
