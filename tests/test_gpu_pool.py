"""The batched pool: every job's result equals the same job run alone.

A job in the pool runs the same fix-until iteration (and annealing prelude)
as gf_anneal + gf_fix_until on a lone lattice, with the same per-site code and
the same reduction order, so links, sweep counts, theta and F must agree
bitwise; tolerance is therefore 0 (the stated bound is 1e-12).
"""

import sys

import numpy as np
import pytest

import gauge_inputs as gi
import oracle
from paper_1412_3655_amd import gf

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    gf.lib()


JOBS = [
    # (dims, eps, seed, anneal sweeps)
    ((4, 4, 4, 4), 0.6, 1, 0),
    ((6, 4, 4, 8), 0.8, 2, 7),
    ((8, 8, 8, 8), 0.5, 3, 0),
    ((2, 4, 6, 8), 0.9, 4, 3),
    ((6, 10, 6, 6), 0.7, 5, 0),
    ((4, 6, 8, 4), 1.0, 6, 12),
]


def fix_kw(check_every):
    return dict(omega=1.7, mode=gf.GF_OR_EXACT, theta_target=1e-12, max_sweeps=4000, check_every=check_every,
                reunit_every=2 * check_every, theta_switch=1e-8)


def solo(dims, links, prec, anneal, seed, check_every, storage=12):
    with gf.Lattice(dims, prec, storage=storage) as lat:
        lat.set_links(links)
        if anneal:
            lat.anneal(anneal, 1.25, 0.05, seed)
        r = lat.fix_until(**fix_kw(check_every))
        return r, lat.get_links()


@pytest.mark.parametrize("prec,reals32,cache32,cache64", [(gf.GF_MIXED, 12, 0, 0), (gf.GF_FP64, 12, 0, 0),
                                                         (gf.GF_MIXED, 8, 0, 0), (gf.GF_MIXED, 8, 2, 1),
                                                         (gf.GF_MIXED, 12, 2, 1), (gf.GF_FP64, 12, 0, 1)])
def test_pool_equals_solo(prec, reals32, cache32, cache64):
    """reals32 = 8: the pool's float32 links in 8 reals, against solo GF_MIXED lattices stored the
    same way.  cache32 / cache64: the cache policy of the pool's overrelaxation sweeps (default
    plain for float32 and non-temporal for float64; 1 plain, 2 non-temporal), which changes
    neither the order of updates within a colour's result nor the links."""
    ce = 5
    say(f"pool vs solo prec={prec} reals32={reals32} cache {cache32}/{cache64}")
    inputs = [gi.gen_links(d, e, s) for (d, e, s, _) in JOBS]
    ref = [solo(d, u, prec, a, 100 + i, ce, reals32) for i, ((d, e, s, a), u) in enumerate(zip(JOBS, inputs))]
    with gf.Pool(1 << 34, 16, prec=prec, check_every=ce, reals32=reals32, cache32=cache32,
                 cache64=cache64) as pool:
        assert pool.cache == (cache32 or (2 if reals32 == 8 else 1), cache64 or 2)
        for i, ((d, e, s, a), u) in enumerate(zip(JOBS, inputs)):
            assert pool.admit(1000 + i, d, u, anneal_sweeps=a, T_start=1.25, T_end=0.05, seed=100 + i,
                              **{k: v for k, v in fix_kw(ce).items() if k not in ("check_every", "mode")})
        done = {}
        for _ in range(2000):
            pool.step()
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == len(JOBS):
                break
        assert len(done) == len(JOBS)
        for i, ((dims, e, s, a), (r_solo, l_solo)) in enumerate(zip(JOBS, ref)):
            d = done[1000 + i]
            r = d["result"]
            say(f"  job {i} {dims}: pool sweeps {r.sweeps} ({r.sweeps_fp32}/{r.sweeps_fp64}) theta {r.theta:.3e}; "
                f"solo {r_solo.sweeps} ({r_solo.sweeps_fp32}/{r_solo.sweeps_fp64}) theta {r_solo.theta:.3e}")
            assert d["status"] == gf.GF_OK
            assert r == r_solo
            links = pool.fetch_links(1000 + i)
            assert np.array_equal(links, l_solo)
        assert pool.stats() == (0, 0, 0)
    if reals32 == 8:
        with pytest.raises(gf.GFError) as e:
            gf.Pool(1 << 30, 4, prec=gf.GF_FP64, reals32=8)
        assert e.value.status == gf.GF_E_ARG


def test_pool_admission_backfill_and_failures():
    say("pool admission, budget, backfill, failures")
    dims = (4, 4, 4, 4)
    need = gf.gf_pool_job_bytes(dims, gf.GF_MIXED)
    u = gi.gen_links(dims, 0.6, 9)
    bad = u.copy()
    bad[5, 2, 1, 1, 0] = np.nan
    with gf.Pool(3 * need, 8, prec=gf.GF_MIXED, check_every=5) as pool:
        assert pool.admit(1, dims, u)
        assert pool.admit(2, dims, bad)  # fails numerically at its first measurement
        assert pool.admit(3, dims, u)
        assert not pool.admit(4, dims, u)  # budget exhausted: nothing changes
        with pytest.raises(gf.GFError) as e:
            pool.admit(1, dims, u)
        assert e.value.status in (gf.GF_E_ARG, gf.GF_E_FULL)
        with pytest.raises(gf.GFError) as e:
            pool.release(3)  # not finished yet
        assert e.value.status == gf.GF_E_STATE
        with pytest.raises(gf.GFError):
            gf.gf_pool_admit(pool.handle, 5, dims, u, check_every=7)  # cadence differs from the pool's
        done = {}
        for _ in range(500):
            pool.step()
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == 3:
                break
        assert done[2]["status"] == gf.GF_E_NUMERIC
        assert done[1]["status"] == gf.GF_OK and done[1]["result"].converged
        assert done[3]["result"] == done[1]["result"]
        pool.release(2)
        assert pool.admit(4, dims, u)  # backfill into the freed budget
        for _ in range(500):
            pool.step()
            got = pool.poll()
            if got:
                assert got[0]["job_id"] == 4 and got[0]["result"] == done[1]["result"]
                break
        a, f, b = pool.stats()
        assert a == 0 and f == 3 and b == 3 * need


def test_pool_many_shapes_fill():
    """64 lattices of uneven volume in one pool converge, each equal to its solo run."""
    say("pool 64 uneven lattices")
    shapes = [(4, 4, 4, 4), (6, 4, 4, 4), (4, 6, 6, 4), (8, 4, 4, 6)]
    rng = np.random.default_rng(4)
    picks = rng.integers(0, len(shapes), 64)
    with gf.Pool(1 << 34, 64, prec=gf.GF_MIXED, check_every=10) as pool:
        inputs = {}
        for i, p in enumerate(picks):
            d = shapes[p]
            inputs[i] = (d, gi.gen_links(d, 0.4 + 0.6 * rng.random(), 1000 + i))
            assert pool.admit(i, d, inputs[i][1], theta_target=1e-12, max_sweeps=3000, reunit_every=100,
                              theta_switch=1e-8)
        done = {}
        for _ in range(1000):
            pool.step()
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == 64:
                break
        assert len(done) == 64
        for i in (0, 17, 63):
            d, u = inputs[i]
            with gf.Lattice(d, gf.GF_MIXED) as lat:
                lat.set_links(u)
                r = lat.fix_until(omega=1.7, mode=0, theta_target=1e-12, max_sweeps=3000, check_every=10,
                                  reunit_every=100, theta_switch=1e-8)
            assert done[i]["result"] == r
        assert all(v["result"].converged for v in done.values())


def test_pool_cancel_mid_run():
    """Cancelling a job mid-run: it is polled with GF_E_CANCELLED and its last theta, takes no
    further steps, and every other job still equals its solo run bitwise."""
    say("pool cancel mid-run")
    ce = 5
    jobs = [((8, 8, 8, 8), 0.6, 31), ((6, 10, 6, 6), 0.7, 32), ((4, 4, 4, 8), 0.5, 33)]
    inputs = [gi.gen_links(d, e, s) for (d, e, s) in jobs]
    ref = {i: solo(d, u, gf.GF_MIXED, 0, 0, ce) for i, ((d, e, s), u) in enumerate(zip(jobs, inputs))}
    kw = {k: v for k, v in fix_kw(ce).items() if k not in ("check_every", "mode")}
    with gf.Pool(1 << 34, 8, prec=gf.GF_MIXED, check_every=ce) as pool:
        for i, ((d, e, s), u) in enumerate(zip(jobs, inputs)):
            assert pool.admit(i, d, u, **kw)
        for _ in range(3):
            pool.step()
        assert pool.poll() == []
        pool.cancel(1)
        with pytest.raises(gf.GFError) as e:
            pool.cancel(1)  # already finished (cancelled)
        assert e.value.status == gf.GF_E_STATE
        with pytest.raises(gf.GFError) as e:
            pool.cancel(99)
        assert e.value.status == gf.GF_E_ARG
        done = {}
        for _ in range(2000):
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == len(jobs):
                break
            pool.step()
        assert len(done) == len(jobs)
        c = done[1]
        assert c["status"] == gf.GF_E_CANCELLED and not c["result"].converged
        assert c["result"].sweeps == 3 * ce and np.isfinite(c["result"].theta)
        for i in (0, 2):
            assert done[i]["status"] == gf.GF_OK
            assert done[i]["result"] == ref[i][0]
            assert np.array_equal(pool.fetch_links(i), ref[i][1])
        pool.release(1)
        assert pool.stats() == (0, 0, 0)


def test_pool_step_in_flight_release_cancel_and_budget():
    """With a step in flight (gf_pool_step_async): a finished job's lattice released meanwhile
    still counts against the budget until the step is completed (gf_pool_sync), an admission
    that needs its bytes is refused until then, cancelling a job completes the step first, and
    every job that ran to the end equals its solo run bitwise."""
    say("pool step in flight: release, budget, cancel")
    ce = 5
    small, big = (4, 4, 4, 4), (8, 8, 8, 8)
    u_small = gi.gen_links(small, 0.3, 41)
    u_big = gi.gen_links(big, 0.8, 42)
    need_s = gf.gf_pool_job_bytes(small, gf.GF_MIXED)
    need_b = gf.gf_pool_job_bytes(big, gf.GF_MIXED)
    ref_small = solo(small, u_small, gf.GF_MIXED, 0, 0, ce)
    ref_big = solo(big, u_big, gf.GF_MIXED, 0, 0, ce)
    kw = {k: v for k, v in fix_kw(ce).items() if k not in ("check_every", "mode")}
    with gf.Pool(2 * need_b, 8, prec=gf.GF_MIXED, check_every=ce) as pool:
        assert pool.admit(1, small, u_small, **kw)
        assert pool.admit(2, big, u_big, **kw)
        done = {}
        for _ in range(2000):
            pool.step_async()
            for d in pool.poll():
                done[d["job_id"]] = d
            if 1 in done:
                break
        assert 1 in done and 2 not in done, "the small job finishes first"
        assert done[1]["result"] == ref_small[0]
        # job 2 is in the step in flight: job 1's lattice comes out beside it
        assert np.array_equal(pool.fetch_links(1), ref_small[1])
        assert pool.stats() == (1, 0, need_s + need_b)  # released, not yet freed
        assert not pool.admit(3, big, u_big, **kw)  # needs job 1's bytes
        pool.sync()
        assert pool.stats()[2] == need_b
        assert pool.admit(3, big, u_big, **kw)  # joins job 2 mid-run
        for _ in range(3):
            pool.step_async()
        pool.cancel(3)  # completes the step in flight first
        for _ in range(4000):
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == 3:
                break
            pool.step_async()
        pool.sync()
        assert done[3]["status"] == gf.GF_E_CANCELLED and done[3]["result"].sweeps == 3 * ce
        assert done[2]["status"] == gf.GF_OK and done[2]["result"] == ref_big[0]
        assert np.array_equal(pool.fetch_links(2), ref_big[1])
        pool.release(3)
        assert pool.stats() == (0, 0, 0)


BATCH_SHAPES = [(12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32), (24, 24, 24, 48)]


@pytest.mark.timeout(900)
def test_pool_full_size_batched_shapes():
    """The batched workload's four lattice shapes at full size, in the pool's launch shapes
    (128-thread blocks; 1 or 2 lanes per site for float64 and 2 for float32, the autotuner's
    picks on MI355X): a float64 pool doing one sweep per job against the oracle's sweep of each
    lattice (1e-12), then a mixed pool (one job with a heat-bath prelude) against each job's solo
    gf_anneal + gf_fix_until run (bitwise)."""
    eps = (0.5, 0.7, 0.9, 1.0)
    inputs = [gi.gen_links(d, e, 1000 + i) for i, (d, e) in enumerate(zip(BATCH_SHAPES, eps))]
    refs = [oracle.sweep(u.copy(), d, 1, 1.7, oracle.OR_EXACT) for d, u in zip(BATCH_SHAPES, inputs)]
    for tps64 in (1, 2):
        say(f"pool full-size shapes, float64, one sweep, tps64={tps64}")
        with gf.Pool(1 << 36, 8, prec=gf.GF_FP64, check_every=1, tps64=tps64) as pool:
            for i, (d, u) in enumerate(zip(BATCH_SHAPES, inputs)):
                assert pool.admit(i, d, u, theta_target=0.0, max_sweeps=1, reunit_every=0)
            pool.step()
            done = {d["job_id"]: d for d in pool.poll()}
            assert sorted(done) == [0, 1, 2, 3]
            for i, d in enumerate(BATCH_SHAPES):
                assert done[i]["status"] == gf.GF_OK and done[i]["result"].sweeps == 1
                diff = float(np.abs(pool.fetch_links(i) - refs[i]).max())
                say(f"  {d}: max|pool - oracle| = {diff:.2e}")
                assert diff <= 1e-12
    say("pool full-size shapes, mixed, against solo runs")
    kw = dict(omega=1.7, mode=gf.GF_OR_EXACT, theta_target=1e-12, max_sweeps=100, check_every=10,
              reunit_every=50, theta_switch=-1.0)
    anneal = (0, 0, 0, 20)
    solo_res = []
    for i, (d, u) in enumerate(zip(BATCH_SHAPES, inputs)):
        with gf.Lattice(d, gf.GF_MIXED) as lat:
            lat.set_links(u)
            if anneal[i]:
                lat.anneal(anneal[i], 1.25, 0.01, 77)
            solo_res.append((lat.fix_until(**kw), lat.get_links()))
    with gf.Pool(1 << 36, 8, prec=gf.GF_MIXED, check_every=10, tps32=2, tps64=2) as pool:
        for i, (d, u) in enumerate(zip(BATCH_SHAPES, inputs)):
            assert pool.admit(i, d, u, anneal_sweeps=anneal[i], T_start=1.25, T_end=0.01, seed=77,
                              **{k: v for k, v in kw.items() if k not in ("check_every", "mode")})
        done = {}
        for _ in range(40):
            pool.step()
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == 4:
                break
        assert sorted(done) == [0, 1, 2, 3]
        for i in range(4):
            r, links = solo_res[i]
            assert done[i]["result"] == r
            assert np.array_equal(pool.fetch_links(i), links)


def test_pool_large_slot_table_uses_the_search_fallback():
    """A pool of more than 511 slots (work-list segments longer than one wave's strided read)
    finds tiles by binary search; its jobs still equal their solo runs."""
    say("pool with 600 slots")
    ce = 5
    jobs = [((6, 4, 4, 8), 0.6, 41), ((4, 4, 4, 4), 0.5, 42), ((8, 8, 8, 8), 0.7, 43)]
    inputs = [gi.gen_links(d, e, s) for (d, e, s) in jobs]
    ref = [solo(d, u, gf.GF_MIXED, 0, 0, ce) for (d, e, s), u in zip(jobs, inputs)]
    kw = {k: v for k, v in fix_kw(ce).items() if k not in ("check_every", "mode")}
    with gf.Pool(1 << 34, 600, prec=gf.GF_MIXED, check_every=ce) as pool:
        for i, ((d, e, s), u) in enumerate(zip(jobs, inputs)):
            assert pool.admit(i, d, u, **kw)
        done = {}
        for _ in range(2000):
            pool.step()
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == len(jobs):
                break
        for i in range(len(jobs)):
            assert done[i]["result"] == ref[i][0]
            assert np.array_equal(pool.fetch_links(i), ref[i][1])


@pytest.mark.parametrize("reals32", [12, 8])
def test_pool_autotune_keeps_results(reals32):
    """gf_pool_autotune times every (lanes, block) shape of the pool's sweeps on copies of the
    resident jobs, applies the fastest, and leaves the jobs' links alone: results still equal
    the solo runs bitwise.  A shape outside {1, 2, 4} x {64, 128, 256} is rejected."""
    ce = 5
    say("pool autotune keeps results")
    jobs = JOBS[:4]
    inputs = [gi.gen_links(d, e, s) for (d, e, s, _) in jobs]
    ref = [solo(d, u, gf.GF_MIXED, a, 200 + i, ce, reals32) for i, ((d, e, s, a), u) in enumerate(zip(jobs, inputs))]
    with pytest.raises(gf.GFError):
        gf.Pool(1 << 30, 4, prec=gf.GF_MIXED, tps32=8)
    with pytest.raises(gf.GFError):
        gf.Pool(1 << 30, 4, prec=gf.GF_MIXED, block64=512)
    with pytest.raises(gf.GFError):
        gf.Pool(1 << 30, 4, prec=gf.GF_MIXED, cache32=3)
    with gf.Pool(1 << 34, 8, prec=gf.GF_MIXED, check_every=ce, block32=64, block64=256, reals32=reals32) as pool:
        # default lanes per site of the float32 sweeps: 1 with 8-real links, 2 with 12-real links
        assert pool.shape == (1 if reals32 == 8 else 2, 64, 1, 256)
        with pytest.raises(gf.GFError) as e:
            pool.autotune(gf.GF_FP32)
        assert e.value.status == gf.GF_E_STATE  # nothing resident
        for i, ((d, e_, s, a), u) in enumerate(zip(jobs, inputs)):
            assert pool.admit(300 + i, d, u, anneal_sweeps=a, T_start=1.25, T_end=0.05, seed=200 + i,
                              **{k: v for k, v in fix_kw(ce).items() if k not in ("check_every", "mode")})
        pool.step()
        (t32, b32, n32), rows32 = pool.autotune(gf.GF_FP32, 2)
        (t64, b64, n64), rows64 = pool.autotune(gf.GF_FP64, 2)
        say(f"  float32 {t32}/{b32} of {len(rows32)} shapes, float64 {t64}/{b64} of {len(rows64)}")
        assert len(rows32) == 18 and len(rows64) == 18  # 3 lanes x 3 blocks x 2 cache policies
        assert pool.shape == (t32, b32, t64, b64)
        assert pool.cache == (n32 + 1, n64 + 1)  # the chosen policy: 0 plain, 1 non-temporal
        assert min(r[3] for r in rows32) == [r[3] for r in rows32 if (r[0], r[1]) == (t32, b32)][0]
        done = {}
        for _ in range(2000):
            pool.step()
            for d in pool.poll():
                done[d["job_id"]] = d
            if len(done) == len(jobs):
                break
        for i, (r_solo, l_solo) in enumerate(ref):
            assert done[300 + i]["result"] == r_solo
            assert np.array_equal(pool.fetch_links(300 + i), l_solo)
    with gf.Pool(1 << 34, 4, prec=gf.GF_FP64, check_every=ce) as pool:
        assert pool.admit(1, jobs[0][0], inputs[0], **{k: v for k, v in fix_kw(ce).items()
                                                        if k not in ("check_every", "mode")})
        with pytest.raises(gf.GFError) as e:
            pool.autotune(gf.GF_FP32)
        assert e.value.status == gf.GF_E_ARG
