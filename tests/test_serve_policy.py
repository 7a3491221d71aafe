"""Admission policy of the serving loop under a virtual clock (no device):
the same FIFO queue and first-fit arena as the server, fake executions."""
import numpy as np
import pytest

from paper_2309_09072_amd import lcs as L


def run(seed, count=300, slots=6, budget=1 << 26):
    r = np.random.default_rng(seed)
    arrival = np.cumsum(r.exponential(0.01, count))
    foot = (r.integers(1, 24, count) << 20).astype(np.uint64)
    service = r.uniform(0.005, 0.08, count)
    ta, td, peak = L.server_simulate(budget, slots, arrival, foot, service)
    return arrival, foot, service, ta, td, peak


@pytest.mark.parametrize("seed", range(6))
def test_invariants(seed):
    budget, slots = 1 << 26, 6
    arrival, foot, service, ta, td, peak = run(seed, slots=slots, budget=budget)
    assert peak <= budget
    assert np.all(ta >= arrival - 1e-12)                 # never admitted before arrival
    assert np.all(np.diff(ta) >= -1e-12)                  # arrival order (FIFO)
    assert np.allclose(td, ta + service)
    # at every admission instant, concurrency and memory stay within limits
    for t in ta:
        live = (ta <= t) & (td > t)
        assert live.sum() <= slots
        assert int(foot[live].sum()) <= budget


def test_continuous_batching_overlaps_arrivals():
    """Requests that arrive while others run are admitted before those finish."""
    arrival = np.array([0.0, 0.01, 0.02, 0.03])
    foot = np.array([1 << 20] * 4, np.uint64)
    service = np.array([1.0, 1.0, 1.0, 1.0])
    ta, td, peak = L.server_simulate(1 << 24, 4, arrival, foot, service)
    assert np.allclose(ta, arrival)
    assert peak == 4 << 20


def test_memory_budget_queues_and_rejects():
    arrival = np.array([0.0, 0.0, 0.0])
    foot = np.array([6 << 20, 6 << 20, 6 << 20], np.uint64)
    service = np.array([1.0, 1.0, 1.0])
    ta, td, peak = L.server_simulate(13 << 20, 8, arrival, foot, service)
    assert np.allclose(ta, [0.0, 0.0, 1.0]) and peak == 12 << 20
    with pytest.raises(L.LcsError):
        L.server_simulate(4 << 20, 8, arrival, foot, service)   # larger than the budget
