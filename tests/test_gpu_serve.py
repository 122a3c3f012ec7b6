"""Serving pattern through the library's request server (fdl_server_*):
an open-loop Poisson mix of construct and render requests with HBM-footprint
admission and continuous batching; every checked result must equal the same
request computed alone, the constructions in the mix must leave layers equal
to a fresh construction, and admission must stay inside the budget."""
import numpy as np
import pytest
import torch

from paper_1901_06919_amd import synth

pytestmark = pytest.mark.gpu


def _pool(k, H=128, W=128, seed=40):
    from paper_1901_06919_amd.serve import PoolEntry
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(k):
        u = synth.grid_positions(4, 0.05, rng)
        m, C, n = u.shape[0], 3, 30
        spec = (rng.standard_normal((m, C, H, W // 2 + 1)) + 1j * rng.standard_normal((m, C, H, W // 2 + 1)))
        d = np.linspace(-3, 3, n).astype(np.float32)
        pool.append(PoolEntry(torch.from_numpy(spec.astype(np.complex64)).cuda(), torch.from_numpy(u).cuda(),
                              torch.from_numpy(d), torch.from_numpy(d).cuda(), H, W, 1e-3, 1e-3, 0))
    return pool


@pytest.mark.parametrize("serial", [False, True])
def test_serving_results_equal_alone_and_admission_respects_budget(serial):
    import paper_1901_06919_amd as fdl
    from paper_1901_06919_amd.serve import FDLServer
    print(f"serving mix through fdl_server_*: serial={serial}", flush=True)
    pool = _pool(3)
    reqs = synth.serving_requests(rate=400.0, duration=1.0, pool=3, seed=4)
    for i, r in enumerate(reqs):
        r.rid = i
    # budget deliberately tight: the three resident layer sets, then room for
    # one construction and a few rendered views at a time
    e = pool[0]
    per_view = 256 * (-(-3 * e.H * (e.W // 2 + 1) * 8 // 256) + -(-3 * e.H * e.W * 4 // 256) + 1)
    layer_bytes = 30 * 3 * e.H * (e.W // 2 + 1) * 8
    budget = 4 * layer_bytes + 6 * per_view
    srv = FDLServer(pool, hbm_budget=budget, max_render_batch=8, max_inflight=6, keep_outputs_every=5,
                    serial=serial)
    stats = srv.run(reqs)
    summ = stats.summary()
    print(summ, flush=True)
    assert stats.completed == len(reqs) and stats.rejected == 0
    assert stats.max_reserved_bytes <= budget
    if not serial:
        assert summ["render_batches"] < summ["render_count"]   # some renders shared a launch
    checked = 0
    for rid, img in srv.kept.items():
        r = reqs[rid]
        e = pool[r.lf]
        layers = srv.layers(r.lf)
        alone = fdl.irfft2(fdl.render(layers, e.d_dev, torch.from_numpy(r.view[None].copy()).cuda(), e.H, e.W),
                           e.H, e.W)[0]
        assert torch.equal(alone, img), f"request {rid} differs alone vs in the mix"
        checked += 1
    assert checked > 10
    # the constructions in the mix left layers equal to a fresh construction
    for i, e in enumerate(pool):
        fresh = fdl.construct(e.view_spec, e.u, e.d_host, e.H, e.W, e.lam, e.eps, e.reg)
        assert torch.equal(fresh, srv.layers(i))
    srv.close()


def test_server_rejects_a_request_larger_than_the_budget():
    from paper_1901_06919_amd.serve import FDLServer
    print("serving: over-budget request rejected at submit", flush=True)
    pool = _pool(1, H=64, W=64)
    e = pool[0]
    layer_bytes = 30 * 3 * e.H * (e.W // 2 + 1) * 8
    # room for the resident layers and one rendered view, not for a second layer set
    srv = FDLServer(pool, hbm_budget=layer_bytes + (1 << 20), max_render_batch=4, max_inflight=4)
    reqs = [synth.Request(0.0, "construct", 0, np.zeros(5, np.float32)),
            synth.Request(0.001, "render", 0, np.array([0.5, -0.5, 0.0, 1.0, 1.0], np.float32))]
    stats = srv.run(reqs)
    assert stats.rejected == 1 and stats.completed == 1
    srv.close()
