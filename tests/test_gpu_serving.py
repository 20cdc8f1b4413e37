"""Continuous batching: jobs admitted while others are part-way through their
sweeps give, alone and in the mix, the same result.

A pool job runs exactly the state machine of gf_anneal + gf_fix_until on a lone
lattice (same per-site code, same reduction order, same switch and stall
rules), so its links, sweep counts, theta and F must equal its solo run
bitwise (the stated bound is 1e-12).  Here jobs arrive while the resident ones
are mid-anneal or mid-fix, and the request loop (serving.run_pool) runs under a
budget small enough that jobs wait in its queue and are backfilled.
"""

import sys

import numpy as np
import pytest

import gauge_inputs as gi
from paper_1412_3655_amd import gf, serving

pytestmark = pytest.mark.gpu

CE = 5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    gf.lib()


FIX = dict(omega=1.7, mode=gf.GF_OR_EXACT, theta_target=1e-12, max_sweeps=3000, check_every=CE,
           reunit_every=4 * CE, theta_switch=-1.0)


def solo(dims, links, prec, anneal, seed, T_end=0.01, storage=12):
    with gf.Lattice(dims, prec, storage=storage) as lat:
        lat.set_links(links)
        if anneal:
            lat.anneal(anneal, 1.25, T_end, seed)
        r = lat.fix_until(**FIX)
        return r, lat.get_links()


# (dims, eps, link seed, anneal sweeps, pool steps to run before admitting the job)
WAVES = [
    ((6, 6, 6, 6), 0.6, 31, 0, 0),
    ((4, 8, 6, 4), 0.7, 32, 40, 0),    # anneals over the first 8 steps while the others fix
    ((8, 8, 8, 8), 0.5, 33, 0, 0),
    ((6, 4, 4, 10), 0.6, 34, 25, 3),   # arrives with every resident job mid-run; anneals beside their fix
    ((4, 4, 4, 4), 0.6, 35, 0, 3),
    ((10, 6, 6, 6), 0.65, 36, 0, 7),   # arrives later still, some jobs near convergence
    ((2, 4, 6, 8), 0.6, 37, 10, 7),
]


@pytest.mark.parametrize("prec,overlap", [(gf.GF_MIXED, False), (gf.GF_FP64, False), (gf.GF_MIXED, True),
                                          (gf.GF_FP64, True)])
def test_admission_while_others_run_equals_solo(prec, overlap):
    """overlap=True: every admission, fetch and release happens while a step is in flight
    (gf_pool_step_async), on the pool's transfer stream."""
    say(f"mid-run admission vs solo, prec={prec} overlap={overlap}")
    inputs = [gi.gen_links(d, e, s) for (d, e, s, _, _) in WAVES]
    ref = [solo(d, u, prec, a, 500 + i) for i, ((d, e, s, a, _), u) in enumerate(zip(WAVES, inputs))]
    done = {}
    with gf.Pool(1 << 34, 16, prec=prec, check_every=CE) as pool:
        step = 0
        pending = list(enumerate(WAVES))
        admitted_mid_run = 0
        while len(done) < len(WAVES):
            while pending and pending[0][1][4] <= step:
                i, (d, e, s, a, _) = pending.pop(0)
                active, _, _ = pool.stats()
                admitted_mid_run += active > 0
                assert pool.admit(700 + i, d, inputs[i], anneal_sweeps=a, T_start=1.25, T_end=0.01,
                                  seed=500 + i, **{k: v for k, v in FIX.items() if k != "check_every"})
            active, _, _ = pool.stats()
            if active and overlap:
                pool.step_async()  # completes the previous step, launches this one
            elif active:
                pool.step()
            step += 1
            for r in pool.poll():
                done[r["job_id"]] = (r, pool.fetch_links(r["job_id"]))
            assert step < 5000
        pool.sync()
        assert admitted_mid_run >= 4
        for i, ((dims, e, s, a, at), (r_solo, l_solo)) in enumerate(zip(WAVES, ref)):
            d, links = done[700 + i]
            r = d["result"]
            say(f"  job {i} {dims} anneal {a} admitted at step {at}: pool sweeps {r.sweeps} "
                f"({r.sweeps_fp32}/{r.sweeps_fp64}) theta {r.theta:.3e}; solo {r_solo.sweeps}")
            assert d["status"] == gf.GF_OK
            assert r == r_solo
            assert np.array_equal(links, l_solo)
        assert pool.stats() == (0, 0, 0)


@pytest.mark.parametrize("overlap,reals32", [(True, 12), (False, 12), (True, 8)])
def test_run_pool_queues_backfills_and_equals_solo(overlap, reals32):
    """The request loop under a budget of two of the largest jobs: a burst of 8 arrivals at
    t = 0, then staggered ones, queue (max queue depth > 0), are backfilled as jobs retire,
    every job finishes with its solo result, latencies are non-negative and the pool never
    holds more than the budget; with the host's work overlapping the steps and without."""
    say(f"serving.run_pool under a tight budget, overlap={overlap}, reals32={reals32}")
    shapes = [(4, 4, 4, 4), (6, 4, 4, 4), (4, 6, 4, 6), (6, 6, 6, 6)]
    rng = np.random.default_rng(11)
    jobs = []
    t = 0.0
    for k in range(14):
        if k >= 8:
            t += float(rng.exponential(0.005))
        d = shapes[int(rng.integers(0, len(shapes)))]
        jobs.append(serving.Job(k, d, float(rng.uniform(0.4, 0.7)), 3000 + k, t,
                                anneal=20 if k % 3 == 0 else 0))
    inputs = {j.job_id: gi.gen_links(j.dims, j.eps, 40 + j.job_id) for j in jobs}
    budget = 2 * gf.gf_pool_job_bytes((6, 6, 6, 6), gf.GF_MIXED, reals32)
    st = serving.run_pool(jobs, lambda j: inputs[j.job_id], prec=gf.GF_MIXED, check_every=CE, max_slots=8,
                          hbm_budget=budget, fix=FIX, collect=True, overlap=overlap, reals32=reals32)
    s = st.summary()
    say(f"  {s['converged']}/{s['jobs']} converged, max queue {s['max_queue_depth']}, "
        f"max resident {s['max_resident_jobs']}, peak bytes {s['peak_hbm_bytes']} of {budget}")
    assert s["jobs"] == len(jobs) and len(st.results) == len(jobs) and s["failed"] == 0
    assert s["max_queue_depth"] > 0
    assert 0 < s["peak_hbm_bytes"] <= budget
    assert min(st.latencies) >= 0.0
    for j in jobs:
        d, links = st.results[j.job_id]
        r_solo, l_solo = solo(j.dims, inputs[j.job_id], gf.GF_MIXED, j.anneal, j.seed, storage=reals32)
        assert d["result"] == r_solo, (j, d["result"], r_solo)
        assert np.array_equal(links, l_solo)
