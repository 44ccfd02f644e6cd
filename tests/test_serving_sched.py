"""Serving scheduler logic on the CPU with a simulated executor: continuous
FIFO admission bounded by executor slots and an HBM budget."""
import numpy as np
import pytest

from paper_2511_06407_amd import serving as sv


def run_sim(requests, budget, slots, per_move=1e-3):
    clock = sv.SimClock()
    ex = sv.SimulatedExecutor(lambda r: per_move * r.n_moves * (r.D / 100.0) ** 2, clock)
    sch = sv.Scheduler(ex, budget, slots, clock=clock)
    sch.run(requests)
    return sch, clock.t


def test_request_stream_shape():
    reqs = sv.make_requests(20.0, 30.0, seed=1)
    assert 450 < len(reqs) < 750                      # Poisson(600)
    D = np.array([r.D for r in reqs])
    assert D.min() >= 34 and D.max() <= 1038
    # log-uniform: median near the geometric mean of the range
    assert abs(np.log(np.median(D)) - 0.5 * (np.log(34) + np.log(1038))) < 0.3
    assert set(r.kind for r in reqs) == {"gp_logistic", "mkl"}


def test_all_complete_and_latency_bounds():
    reqs = sv.make_requests(5.0, 10.0, d_max=300, moves=(5, 20), seed=2)
    sch, t_end = run_sim(reqs, budget=40e9, slots=4)
    for r in reqs:
        assert r.done_s is not None and r.admit_s >= r.arrival_s - 1e-12
        service = 1e-3 * r.n_moves * (r.D / 100.0) ** 2
        assert r.latency_s >= service - 1e-9
    assert sch.max_running <= 4


def test_memory_budget_is_respected_and_blocks_fifo():
    reqs = sv.make_requests(50.0, 2.0, d_min=400, d_max=1038, moves=(5, 10), seed=3)
    fps = [sv.request_footprint(r) for r in reqs]
    budget = 2.5 * max(fps)
    sch, _ = run_sim(reqs, budget=budget, slots=16)
    assert sch.max_in_use <= budget
    # FIFO: admission order follows arrival order
    order = sorted(reqs, key=lambda r: r.admit_s)
    assert [r.rid for r in order] == sorted(r.rid for r in reqs)


def test_oversized_request_is_refused():
    reqs = [sv.Request(0, 0.0, "mkl", 1038, 5, 0)]
    with pytest.raises(ValueError):
        run_sim(reqs, budget=1e6, slots=1)


def test_footprint_grows_with_dimension():
    assert sv.footprint_bytes(1024, 14) > 10 * sv.footprint_bytes(256, 14)
    assert sv.footprint_bytes(1024, 14) < 8e9
