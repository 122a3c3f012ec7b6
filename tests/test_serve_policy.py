"""Host-side tests of the request server's scheduling policy
(fdl_server_simulate: the library's own scheduler on a simulated device with
fixed service times, no GPU): rejection of requests that can never fit,
termination, no head-of-line blocking, the starvation guard, render
grouping, one construction per light field at a time, the serial baseline,
and the budget bound."""
import numpy as np
import pytest

MB = 2 ** 20
DONE, REJECTED = 2, 3
CONSTRUCT, RENDER = 0, 1


def sim(*a, **k):
    from paper_1901_06919_amd import serve
    return serve.simulate(*a, **k)


def test_request_that_can_never_fit_is_rejected_at_submit_and_the_rest_is_served():
    # 10 MB pool, two light fields of 3 MB layers: 4 MB left for work.  A
    # light field whose rendered view needs 5 MB can never be served.
    reqs = [(0.0, RENDER, 1), (0.0, RENDER, 0), (0.001, CONSTRUCT, 0), (0.002, RENDER, 1)]
    rows, s = sim(10 * MB, [3 * MB, 3 * MB], [1 * MB, 5 * MB], reqs, 0.01, 0.001)
    assert [r[0] for r in rows] == [REJECTED, DONE, DONE, REJECTED]
    assert s["rejected"] == 2 and s["completed"] == 2
    assert s["max_reserved_MB"] <= s["budget_MB"]


def test_no_head_of_line_blocking_behind_a_construct_waiting_for_memory():
    # 9 MB pool: resident 3 + 3, so a construct (3 MB) must wait while two
    # 1 MB renders run; a render that arrives after the construct starts first
    reqs = [(0.0, RENDER, 0), (0.0, RENDER, 1), (0.0001, CONSTRUCT, 1), (0.0002, RENDER, 0)]
    rows, s = sim(9 * MB, [3 * MB, 3 * MB], [1 * MB, 1 * MB], reqs, 0.01, 0.004, max_render_batch=1)
    st, batch, t_admit, t_done = zip(*rows)
    assert all(x == DONE for x in st)
    assert t_admit[2] > t_admit[3]              # the later render overtook the blocked construct
    assert t_admit[2] >= min(t_done[0], t_done[1]) - 1e-12   # the construct started once memory was freed


def test_starvation_guard_stops_overtaking_after_50_ms():
    # an overload of renders of light field 0 (one every 0.5 ms, 2 ms each on
    # two streams) keeps the 4 MB of free pool full, so the construct of light
    # field 1 (3 MB) could wait forever behind later renders; after 50 ms
    # nothing may overtake it, the renders in flight drain, and it starts
    reqs = [(0.0, RENDER, 0), (0.0, RENDER, 0), (0.0001, CONSTRUCT, 1)]
    reqs += [(0.0002 + 0.0005 * i, RENDER, 0) for i in range(300)]
    rows, s = sim(10 * MB, [3 * MB, 3 * MB], [1 * MB, 1 * MB], reqs, 0.001, 0.002, max_render_batch=1)
    assert all(r[0] == DONE for r in rows)
    wait = rows[2][2] - reqs[2][0]
    assert 0.05 <= wait <= 0.05 + 0.005
    # without the guard it would have waited for the whole render stream
    assert wait < 0.2 * max(r[3] for r in rows)


def test_arrived_renders_of_one_light_field_share_a_launch():
    reqs = [(0.0, RENDER, 0)] * 5 + [(0.0, RENDER, 1)] * 2
    rows, s = sim(64 * MB, [3 * MB, 3 * MB], [1 * MB, 1 * MB], reqs, 0.01, 0.001, max_render_batch=4)
    batches = [r[1] for r in rows]
    assert batches[:4] == [batches[0]] * 4 and batches[4] != batches[0]
    assert batches[5] == batches[6] and batches[5] not in batches[:5]
    assert s["render_batches"] == 3 and abs(s["mean_render_batch"] - 7 / 3) < 1e-12


def test_one_construction_per_light_field_at_a_time():
    reqs = [(0.0, CONSTRUCT, 0), (0.0, CONSTRUCT, 0), (0.0, CONSTRUCT, 1)]
    rows, s = sim(64 * MB, [3 * MB, 3 * MB], [1 * MB, 1 * MB], reqs, 0.01, 0.001)
    assert all(r[0] == DONE for r in rows)
    assert rows[1][2] >= rows[0][3] - 1e-12      # second construct of lf 0 after the first ends


def test_serial_baseline_is_strict_arrival_order_one_view_per_render():
    rng = np.random.default_rng(1)
    t = np.cumsum(rng.exponential(0.002, 50))
    reqs = [(float(ti), CONSTRUCT if rng.random() < 0.2 else RENDER, int(rng.integers(0, 3))) for ti in t]
    rows, s = sim(64 * MB, [3 * MB] * 3, [1 * MB] * 3, reqs, 0.004, 0.001, serial=True)
    admits = [r[2] for r in rows]
    assert all(r[0] == DONE for r in rows)
    assert admits == sorted(admits)
    for a, b in zip(rows, rows[1:]):
        assert b[2] >= a[3] - 1e-12              # one unit of work at a time
    assert s["mean_render_batch"] == 1.0


def test_random_stream_terminates_within_budget_and_continuous_beats_serial_at_the_tail():
    rng = np.random.default_rng(7)
    t = np.cumsum(rng.exponential(1 / 800.0, 2000))
    reqs = [(float(ti), CONSTRUCT if rng.random() < 0.2 else RENDER, int(rng.integers(0, 8))) for ti in t]
    lb, vb = [95 * MB] * 8, [4 * MB] * 8
    rows, cont = sim(2048 * MB, lb, vb, reqs, 1.0e-3, 0.25e-3)
    rows_s, ser = sim(2048 * MB, lb, vb, reqs, 1.0e-3, 0.25e-3, serial=True)
    assert cont["completed"] == ser["completed"] == len(reqs)
    assert cont["max_reserved_MB"] <= 2048
    assert cont["all_p99_ms"] < ser["all_p99_ms"]


def test_simulate_rejects_bad_arguments():
    from paper_1901_06919_amd import FDLError
    with pytest.raises(FDLError):
        sim(64 * MB, [3 * MB], [1 * MB], [(0.0, RENDER, 5)], 0.01, 0.001)   # unknown light field
    with pytest.raises(FDLError):
        sim(1 * MB, [3 * MB], [1 * MB], [(0.0, RENDER, 0)], 0.01, 0.001)   # layers larger than the pool
