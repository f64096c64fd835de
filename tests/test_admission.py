"""Admission and scheduling policy of the serving loop, on a fake clock with a
stub executor (host-only; no GPU)."""
import numpy as np
import pytest

from paper_1211_6193_amd.server import Admission, Request, estimate_bytes, simulate
from paper_1211_6193_amd import workloads as W


def _arrivals(n, rate, seed, lo=1 << 20, hi=1 << 26):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    b = rng.integers(lo, hi, n)
    return list(zip(t.tolist(), b.tolist()))


@pytest.mark.parametrize("slots", [1, 2, 4])
@pytest.mark.parametrize("budget", [1 << 27, 1 << 30])
def test_budget_never_exceeded_and_all_served(slots, budget):
    arr = _arrivals(500, 2000.0, slots * 7 + budget % 97)
    res, peak = simulate(arr, lambda nbytes: 1e-4 + nbytes / 4e11, budget, slots)
    assert peak <= budget
    assert all(d >= s >= a for a, s, d in res)          # every request admitted after arrival, finished after


def test_fifo_order_of_admission():
    arr = _arrivals(300, 5000.0, 3)
    res, _ = simulate(arr, lambda nbytes: 2e-4, 1 << 28, 2)
    starts = [s for _, s, _ in res]
    assert starts == sorted(starts)                      # requests are admitted in arrival order


def test_oversized_request_rejected():
    adm = Admission(1000, 2)
    with pytest.raises(ValueError):
        adm.arrive(Request(0, 0.0, None, 2000))


def test_take_respects_slots():
    adm = Admission(1 << 20, 1)
    for i in range(5):
        adm.arrive(Request(i, 0.0, None, 100))
    b = adm.take()
    assert len(b) == 5 and adm.take() == []
    adm.finish(b)
    assert adm.in_use == 0 and adm.inflight == 0


def test_estimate_covers_memory_and_log():
    job = W.family_job("STENCIL", 4, 128, np.random.default_rng(0))
    est = estimate_bytes(job)
    assert est >= 2 * 4 * len(job.memory) + 8 * 6 * 4 * 128


def test_longest_fitting_prefix_with_a_batch_cost():
    # a batch costs a fixed part plus its requests' bytes (the shape of the
    # library's footprint): the longest prefix that fits is taken, in order
    cost = lambda rs: (50 + sum(r.bytes for r in rs)) if rs else 0
    adm = Admission(1000, 2, cost=cost)
    for i, b in enumerate([600, 300, 200, 10]):
        adm.arrive(Request(i, 0.0, None, b))
    first = adm.take()
    assert [r.rid for r in first] == [0, 1] and adm.in_use == 950
    assert adm.take() == []                      # 200 more does not fit next to 950
    adm.finish(first)
    second = adm.take()
    assert [r.rid for r in second] == [2, 3] and adm.in_use == 260
    with pytest.raises(ValueError):
        adm.arrive(Request(9, 0.0, None, 960))   # 1010 with the fixed part
