"""CPU tests of the serving scheduler (simulated executor: a batch holds its slot for q * cost ns).

Admission is in arrival order, only into a free slot, and only when the batch's device buffers fit
in what the memory budget has left; a request larger than the whole budget is rejected; latencies are
completion - arrival; the statistics agree with the completions. Waiting requests are coalesced into
one batch, in arrival order, while their total stays within the coalescing size (off: coalesce=1).
"""
import numpy as np
import pytest

import paper_2505_03372_amd as wt


def _reqs(sizes, arrivals):
    return [dict(q=int(q), arrival_s=float(a)) for q, a in zip(sizes, arrivals)]


def _mixed_scratch(q):
    """Device scratch of one mixed batch (class offsets; then class counts and classes below 2^16
    queries, else bucket ids, the sort passes and the bucket starts; then the slot order)."""
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    if q <= 16384:
        return 0
    if q < 1 << 16:
        return r(4 * 18) + r(4 * 64) + r(q) + r(4 * q)
    nblk = -(-q // (1024 * 256))
    return r(4 * 18) + r(2 * q) + r(r(nblk * 32768 * 4) + r(4 * 32768)) + r(4 * 32768) + r(4 * q)


def _request_bytes(q):
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    return r(4 * q) + r(q) + r(4 * q) + r(8 * q) + r(8 * q) + r(_mixed_scratch(q))


def test_fifo_single_slot():
    s = wt.Server(None, slots=1, sim_ns_per_query=200.0, coalesce=1)
    sizes = [1000, 10, 5000, 1, 3000]
    comps, st = s.run(_reqs(sizes, [0.0] * len(sizes)))
    admits = [c["admit_s"] for c in comps]
    assert admits == sorted(admits)
    for a, b in zip(comps, comps[1:]):
        assert b["admit_s"] >= a["done_s"] - 1e-9
    for q, c in zip(sizes, comps):
        assert c["status"] == wt.WT_OK and c["slot"] == 0
        assert c["done_s"] - c["admit_s"] >= q * 200e-9 * 0.999
    assert st["peak_in_flight"] == 1 and st["queries"] == sum(sizes) and st["rejected"] == 0
    s.close()


def test_slots_bound_concurrency():
    s = wt.Server(None, slots=4, sim_ns_per_query=1000.0, coalesce=1)
    comps, st = s.run(_reqs([2000] * 12, [0.0] * 12))
    assert st["peak_in_flight"] == 4
    slots = [c["slot"] for c in comps]
    assert set(slots) == {0, 1, 2, 3}
    # never more than 4 requests overlap
    ev = sorted([(c["admit_s"], 1) for c in comps] + [(c["done_s"], -1) for c in comps], key=lambda x: (x[0], x[1]))
    live = peak = 0
    for _, d in ev:
        live += d
        peak = max(peak, live)
    assert peak <= 4
    s.close()


def test_memory_budget_admission_and_rejection():
    q = 100000
    budget = 2 * _request_bytes(q) + 1000  # room for two such requests at once
    s = wt.Server(None, slots=8, mem_budget=budget, sim_ns_per_query=20.0, coalesce=1)
    sizes = [q] * 6 + [10 * q] + [q]  # the 10q request exceeds the whole budget
    comps, st = s.run(_reqs(sizes, [0.0] * len(sizes)))
    assert st["peak_bytes"] <= budget
    assert st["peak_in_flight"] == 2
    assert comps[6]["status"] == wt.WT_ERR_OOM and comps[6]["slot"] == 0xFFFFFFFF
    assert st["rejected"] == 1 and st["queries"] == 7 * q
    assert all(c["status"] == wt.WT_OK for i, c in enumerate(comps) if i != 6)
    s.close()


def test_arrivals_and_latency_stats():
    rng = np.random.default_rng(5)
    n = 300
    arr = np.cumsum(rng.exponential(200e-6, n))
    sizes = rng.integers(1, 2000, n)
    s = wt.Server(None, slots=3, sim_ns_per_query=100.0, coalesce=1)
    comps, st = s.run(_reqs(sizes, arr))
    lat = np.array([c["done_s"] - c["arrival_s"] for c in comps])
    assert np.all(np.array([c["admit_s"] for c in comps]) >= arr - 1e-9)
    assert np.all(lat >= sizes * 100e-9 * 0.999)
    srt = np.sort(lat)
    assert abs(st["lat_p50_s"] - srt[int(0.5 * (n - 1) + 0.5)]) < 1e-12
    assert abs(st["lat_p99_s"] - srt[int(0.99 * (n - 1) + 0.5)]) < 1e-12
    assert st["lat_max_s"] == pytest.approx(srt[-1])
    assert st["queries"] == int(sizes.sum())
    assert st["qps"] == pytest.approx(st["queries"] / st["makespan_s"])
    s.close()


def test_unsorted_arrivals_rejected():
    s = wt.Server(None, slots=2, sim_ns_per_query=10.0)
    with pytest.raises(wt.WTError) as ei:
        s.run(_reqs([1, 1], [0.5, 0.1]))
    assert ei.value.status == wt.WT_ERR_ARG
    s.close()


def test_server_needs_forest_without_simulation():
    with pytest.raises(wt.WTError) as ei:
        wt.Server(None, slots=2)
    assert ei.value.status == wt.WT_ERR_ARG


def test_coalescing_groups_waiting_requests_in_order():
    """With one slot, requests waiting at the same time go out as batches of consecutive requests whose
    total stays within the coalescing size; a request above it goes alone; each batch completes at once
    after its total cost."""
    s = wt.Server(None, slots=1, sim_ns_per_query=100.0, coalesce=4000)
    sizes = [1000, 1500, 1000, 600, 5000, 10, 20]  # batches: [0..2] (3500), [3] (600 + 5000 > 4000), [4], [5, 6]
    comps, st = s.run(_reqs(sizes, [0.0] * len(sizes)))
    groups = [[0, 1, 2], [3], [4], [5, 6]]
    assert st["batches"] == len(groups) and st["queries"] == sum(sizes)
    for g in groups:
        assert len({comps[i]["admit_s"] for i in g}) == 1 and len({comps[i]["done_s"] for i in g}) == 1
        cost = sum(sizes[i] for i in g) * 100e-9
        assert comps[g[0]]["done_s"] - comps[g[0]]["admit_s"] >= cost * 0.999
    for a, b in zip(groups, groups[1:]):
        assert comps[b[0]]["admit_s"] >= comps[a[0]]["done_s"] - 1e-9
    assert st["peak_in_flight"] == 3  # the first batch
    s.close()


def test_coalescing_default_size_and_slot_default():
    """Default: 8 slots and batches of up to 16384 queries; 128 requests of 1000 queries waiting at once
    fill eight batches of 16 requests (16000 queries each)."""
    s = wt.Server(None, sim_ns_per_query=50.0)
    comps, st = s.run(_reqs([1000] * 128, [0.0] * 128))
    assert st["batches"] == 8 and st["peak_in_flight"] == 128
    assert sorted({c["slot"] for c in comps}) == list(range(8))
    s.close()
