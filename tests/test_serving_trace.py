"""Host logic of the serving and batched workloads (no GPU): the seeded job traces."""

import math

import numpy as np

from paper_1412_3655_amd import serving


def test_serving_trace_draws():
    """Poisson arrivals at 20/s, L even in [8, 32] from V log-uniform in [8^4, 32^4], eps uniform in
    [0.4, 1], about 30 % with a 500-sweep anneal, job seed 2000 + k; rounding eps to buckets changes
    nothing else."""
    jobs = serving.serving_trace(1000, 20.0, 5)
    b = serving.serving_trace(1000, 20.0, 5, eps_buckets=(0.4, 0.7, 1.0))
    t = np.array([j.arrival for j in jobs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 20.0) < 0.1 / 20.0  # exponential inter-arrivals, mean 1/rate
    L = np.array([j.dims[0] for j in jobs])
    assert all(j.dims == (j.dims[0],) * 4 for j in jobs)
    assert L.min() >= 8 and L.max() <= 32 and np.all(L % 2 == 0)
    logv = 4 * np.log(L)
    assert abs(np.median(logv) - 0.5 * (math.log(8 ** 4) + math.log(32 ** 4))) < 0.5
    eps = np.array([j.eps for j in jobs])
    assert eps.min() >= 0.4 and eps.max() <= 1.0 and len(set(eps.tolist())) == len(jobs)
    assert abs(eps.mean() - 0.7) < 0.03
    frac = np.mean([j.anneal == 500 for j in jobs])
    assert 0.25 < frac < 0.35 and all(j.anneal in (0, 500) for j in jobs)
    assert [j.seed for j in jobs] == [2000 + k for k in range(1000)]
    for x, y in zip(jobs, b):
        assert (x.arrival, x.dims, x.anneal, x.seed) == (y.arrival, y.dims, y.anneal, y.seed)
        assert y.eps in (0.4, 0.7, 1.0) and abs(y.eps - x.eps) <= 0.15 + 1e-12


def test_batched_jobs_draws():
    jobs = serving.batched_jobs(64, 4)
    shapes = {(12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32), (24, 24, 24, 48)}
    assert all(j.dims in shapes for j in jobs)
    assert [j.seed for j in jobs] == [1000 + i for i in range(64)]
    assert all(0.4 <= j.eps <= 1.0 for j in jobs)
    assert sum(serving.volume(j.dims) for j in jobs) == 12719104


def test_compare_finals():
    """Per-result comparison of a mixed-precision run with a float64 run of the same jobs: only
    jobs converged in both count; |dF| above 1e-9 marks another maximum."""
    a = serving.RunStats(3, 0, 1.0)
    b = serving.RunStats(3, 0, 1.0)
    a.finals = {1: (True, 1e-13, 0.5), 2: (True, 2e-13, 0.6), 3: (False, 1e-7, 0.7), 4: (True, 1e-13, 0.1)}
    b.finals = {1: (True, 3e-13, 0.5 + 1e-12), 2: (True, 2e-13, 0.6 + 1e-5), 3: (True, 1e-13, 0.7)}
    c = serving.compare_finals(a, b)
    assert c["jobs_converged_in_both"] == 2
    assert c["jobs_same_maximum_dF_le_1e-9"] == 1
    assert abs(c["max_abs_dF"] - 1e-5) < 1e-12 and abs(c["max_abs_dF_same_maximum"] - 1e-12) < 1e-15
    assert abs(c["max_abs_dtheta"] - 2e-13) < 1e-20
    assert serving.compare_finals(serving.RunStats(0, 0, 1.0), b) == {"jobs_converged_in_both": 0}
