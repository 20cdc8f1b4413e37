"""Request loop over the native job pool (gf_pool_*): continuous batching of
gauge-fixing jobs.

The pool (C ABI, include/gf.h) owns the device work: admission by HBM
footprint, resident lattices, batched sweeps (one launch per kernel kind over
every lattice) captured in hipGraphs, retirement.  This module is the arrival-side driver: it releases jobs into a
FIFO queue at their arrival times, admits from the head of the queue whenever
the pool has room (slots and bytes), steps the pool, and retires finished
jobs (freeing their lattices, which lets queued jobs in); by default the host
work of a pass (retiring, downloading, admitting) runs while the next step is
on the GPU.  Latency of a job = completion of the pool step in which it
finished - its arrival, on the library's steady clock.

`run_fifo` is the comparison path: one lattice at a time, in arrival order,
with gf_anneal + gf_fix_until on a lone lattice of the given precision.
"""

from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import gf


@dataclass
class Job:
    job_id: int
    dims: tuple
    eps: float
    seed: int
    arrival: float = 0.0  # seconds after the start of the run
    anneal: int = 0       # heat-bath sweeps before the fix-until iteration (T 1.25 -> 0.01)


@dataclass
class RunStats:
    jobs: int
    converged: int
    seconds: float
    latencies: list = field(default_factory=list)        # every finished job
    conv_latencies: list = field(default_factory=list)   # converged jobs only
    results: dict = field(default_factory=dict)          # job_id -> (result, links) when collected
    finals: dict = field(default_factory=dict)           # job_id -> (converged, theta, F) of every finished job
    sweeps: int = 0
    sweeps_fp32: int = 0     # fix-phase sweeps in float32 (mixed precision)
    sweeps_fp64: int = 0     # fix-phase sweeps in float64
    site_updates: float = 0.0
    site_updates_fp32: float = 0.0  # fix-phase site updates in float32
    site_updates_fp64: float = 0.0  # fix-phase site updates in float64
    site_updates_anneal: float = 0.0
    failed: int = 0
    max_queue: int = 0       # most jobs waiting for admission at once
    max_resident: int = 0    # most jobs resident in the pool at once
    peak_bytes: int = 0      # most device bytes the pool held for job lattices
    shape: tuple = ()        # (tps32, block32, tps64, block64) of the pool's sweeps
    cache: tuple = ()        # (cache32, cache64): 1 plain, 2 non-temporal link accesses
    tuning: dict = field(default_factory=dict)  # autotuner tables (kernel -> rows), when tuned

    def summary(self) -> dict:
        def pct(v, q):
            return float(np.percentile(v, q)) if v else None

        return {
            "jobs": self.jobs,
            "converged": self.converged,
            "failed": self.failed,
            "seconds": self.seconds,
            "converged_lattices_per_s": self.converged / self.seconds if self.seconds > 0 else None,
            "lattices_per_s": self.jobs / self.seconds if self.seconds > 0 else None,
            "p50_latency_s_converged": pct(self.conv_latencies, 50),
            "p99_latency_s_converged": pct(self.conv_latencies, 99),
            # every job, a job that stopped at its sweep cap unconverged counted at
            # the time it stopped: its time to theta < 1e-12 is censored there, so
            # these are lower bounds of the percentiles over all jobs
            "p50_latency_s_censored": pct(self.latencies, 50),
            "p99_latency_s_censored": pct(self.latencies, 99),
            "site_updates_per_s": self.site_updates / self.seconds if self.seconds > 0 else None,
            "sweeps": self.sweeps,
            "fix_sweeps_fp32": self.sweeps_fp32,
            "fix_sweeps_fp64": self.sweeps_fp64,
            "site_updates": self.site_updates,
            "fix_site_updates_fp32": self.site_updates_fp32,
            "fix_site_updates_fp64": self.site_updates_fp64,
            "anneal_site_updates": self.site_updates_anneal,
            "max_queue_depth": self.max_queue,
            "max_resident_jobs": self.max_resident,
            "peak_hbm_bytes": self.peak_bytes,
            "pool_shape_tps32_block32_tps64_block64": list(self.shape) or None,
            "pool_cache32_cache64": list(self.cache) or None,
            "pool_autotune_us_per_sweep": self.tuning or None,
        }


def volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


def batched_jobs(n=64, master_seed=4):
    """The batched workload: n lattices with shapes uniform over {12^4, 16^4, 16^3x32, 24^3x48},
    eps uniform in [0.4, 1.0] (drawn from a seeded stream), link seed 1000 + i."""
    shapes = [(12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32), (24, 24, 24, 48)]
    rng = np.random.default_rng(master_seed)
    out = []
    for i in range(n):
        d = shapes[int(rng.integers(0, len(shapes)))]
        out.append(Job(i, d, float(rng.uniform(0.4, 1.0)), 1000 + i))
    return out


def serving_trace(n=1000, rate=20.0, master_seed=5, anneal_fraction=0.3, anneal_sweeps=500,
                  eps_buckets=None):
    """The serving workload: Poisson arrivals at `rate` per second; V log-uniform between 8^4 and
    32^4 with L = even extent nearest V^(1/4); eps uniform in [0.4, 1.0] (rounded to the nearest
    of `eps_buckets` when given, so that a long trace can generate one input per (L, eps) and
    reuse it); a fraction of the jobs with an annealing prelude; job seed 2000 + k.  The random
    draws do not depend on `eps_buckets`: arrivals, extents and preludes are the same either way."""
    rng = np.random.default_rng(master_seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate))
        logv = rng.uniform(math.log(8 ** 4), math.log(32 ** 4))
        L = int(round(math.exp(logv / 4.0) / 2.0)) * 2
        L = min(32, max(8, L))
        eps = float(rng.uniform(0.4, 1.0))
        if eps_buckets:
            eps = min(eps_buckets, key=lambda e: abs(e - eps))
        anneal = anneal_sweeps if rng.random() < anneal_fraction else 0
        out.append(Job(k, (L, L, L, L), eps, 2000 + k, t, anneal))
    return out


def run_pool(jobs, links_of, prec=gf.GF_MIXED, check_every=10, max_slots=256, hbm_budget=None,
             fix=None, open_loop=True, tps32=0, tps64=0, log=None, collect=False, autotune=False,
             overlap=True, reals32=12):
    """Run `jobs` through a pool; links_of(job) -> canonical host links.  collect=True
    downloads every finished job's links into stats.results[job_id] = (result, links)
    (the download is inside the timed run).  autotune=True runs gf_pool_autotune on the jobs
    resident before the first step (inside the timed run), for the float32 sweeps of a
    mixed pool and the float64 sweeps.

    overlap=True: each pass completes the step in flight, frees the lattices of the jobs
    that finished in it, launches the next step and, while it runs, downloads finished
    jobs (collect=True) and admits queued ones, which join the step after it.
    overlap=False: step, retire and admit one after another with the GPU idle between
    steps.  Every job's result is the same either way.  reals32 = 8: the pool's float32 links
    in 8 reals (a GF_MIXED pool)."""
    fix = dict(fix or {})
    import torch

    free, total = torch.cuda.mem_get_info()
    if hbm_budget is None:
        hbm_budget = int(free * 0.8)
    stats = RunStats(jobs=len(jobs), converged=0, seconds=0.0)
    arrivals = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    queue = collections.deque()
    by_id = {}
    with gf.Pool(hbm_budget, max_slots, prec=prec, check_every=check_every, mode=fix.get("mode", 0),
                 tps32=tps32, tps64=tps64, reals32=reals32) as pool:
        t0 = gf.gf_clock()
        done = 0

        def admit_queued():
            now = gf.gf_clock() - t0
            while arrivals and (not open_loop or arrivals[0].arrival <= now):
                queue.append(arrivals.popleft())
            while queue:
                j = queue[0]
                ok = pool.admit(j.job_id, j.dims, links_of(j), anneal_sweeps=j.anneal, T_start=1.25, T_end=0.01,
                                seed=j.seed, **fix)
                if not ok:
                    break
                by_id[j.job_id] = j
                queue.popleft()
            active, finished, held = pool.stats()
            stats.max_queue = max(stats.max_queue, len(queue))
            stats.max_resident = max(stats.max_resident, active + finished)
            stats.peak_bytes = max(stats.peak_bytes, held)
            return active

        def record(d, links=None):
            nonlocal done
            j = by_id.pop(d["job_id"])
            if collect:
                stats.results[d["job_id"]] = (d, links)
            lat = d["t_done"] - t0 - j.arrival if open_loop else d["t_done"] - t0
            r = d["result"]
            stats.latencies.append(lat)
            stats.sweeps += r.sweeps + j.anneal
            stats.sweeps_fp32 += r.sweeps_fp32
            stats.sweeps_fp64 += r.sweeps_fp64
            stats.site_updates += (r.sweeps + j.anneal) * volume(j.dims)
            stats.site_updates_fp32 += r.sweeps_fp32 * volume(j.dims)
            stats.site_updates_fp64 += r.sweeps_fp64 * volume(j.dims)
            stats.site_updates_anneal += j.anneal * volume(j.dims)
            if d["status"] == gf.GF_OK:
                stats.finals[j.job_id] = (bool(r.converged), r.theta, r.F)
            if d["status"] != gf.GF_OK:
                stats.failed += 1
            elif r.converged:
                stats.converged += 1
                stats.conv_latencies.append(lat)
            done += 1
            if log:
                log(f"  job {j.job_id} {j.dims} eps={j.eps:.2f} anneal={j.anneal}: sweeps {r.sweeps} "
                    f"({r.sweeps_fp32}/{r.sweeps_fp64}) theta {r.theta:.2e} latency {lat:.2f} s")

        def tune_once(active):
            if active and autotune and not stats.tuning:
                held = pool.stats()[2]
                kinds = [gf.GF_FP32, gf.GF_FP64] if prec == gf.GF_MIXED else [gf.GF_FP64]
                for k in kinds:
                    _, rows = pool.autotune(k, 3, scratch_bytes=min(held, 16 << 30))
                    stats.tuning["fp32" if k == gf.GF_FP32 else "fp64"] = [
                        [t, b, nt, round(us, 1)] for (t, b, nt, us) in rows]
                stats.shape = pool.shape
                stats.cache = pool.cache

        def idle(active, finished):
            if active or finished:
                return
            if arrivals and not queue:
                time.sleep(max(0.0, min(0.05, arrivals[0].arrival - (gf.gf_clock() - t0))))
            elif queue:
                raise RuntimeError(f"job {queue[0].job_id} {queue[0].dims} does not fit the pool budget")

        while done < len(jobs):
            if overlap:
                pool.sync()
                ended = pool.poll()
                if not collect:
                    for d in ended:
                        pool.release(d["job_id"])  # nothing in flight: freed now, room for admissions
                active, finished, _ = pool.stats()
                tune_once(active)
                if active:
                    pool.step_async()
                for d in ended:
                    record(d, pool.fetch_links(d["job_id"]) if collect else None)
                active = admit_queued()
                idle(active, pool.stats()[1])
            else:
                active = admit_queued()
                tune_once(active)
                finished = pool.stats()[1]
                if active:
                    pool.step()
                else:
                    idle(active, finished)
                for d in pool.poll():
                    if collect:
                        record(d, pool.fetch_links(d["job_id"]))
                    else:
                        pool.release(d["job_id"])
                        record(d)
        pool.sync()
        stats.seconds = gf.gf_clock() - t0
        stats.shape = pool.shape
        stats.cache = pool.cache
    return stats


def run_fifo(jobs, links_of, prec=gf.GF_FP64, fix=None, open_loop=True, tps=0, block=0, nt=0, log=None):
    """One lattice at a time in arrival order (gf_anneal + gf_fix_until on a lone lattice)."""
    fix = dict(fix or {})
    stats = RunStats(jobs=len(jobs), converged=0, seconds=0.0)
    t0 = gf.gf_clock()
    for j in sorted(jobs, key=lambda j: j.arrival):
        if open_loop:
            wait = j.arrival - (gf.gf_clock() - t0)
            if wait > 0:
                time.sleep(wait)
        u = links_of(j)
        with gf.Lattice(j.dims, prec) as lat:
            if tps:
                lat.set_sweep_config(tps, block, nt)
            lat.set_links(u)
            if j.anneal:
                lat.anneal(j.anneal, 1.25, 0.01, j.seed)
            try:
                r = lat.fix_until(**fix)
                ok = True
            except gf.GFError:
                ok = False
        t_done = gf.gf_clock() - t0
        lat_s = t_done - j.arrival if open_loop else t_done
        stats.latencies.append(lat_s)
        if not ok:
            stats.failed += 1
            continue
        stats.finals[j.job_id] = (bool(r.converged), r.theta, r.F)
        stats.sweeps += r.sweeps + j.anneal
        stats.sweeps_fp32 += r.sweeps_fp32
        stats.sweeps_fp64 += r.sweeps_fp64
        stats.site_updates += (r.sweeps + j.anneal) * volume(j.dims)
        stats.site_updates_fp32 += r.sweeps_fp32 * volume(j.dims)
        stats.site_updates_fp64 += r.sweeps_fp64 * volume(j.dims)
        stats.site_updates_anneal += j.anneal * volume(j.dims)
        if r.converged:
            stats.converged += 1
            stats.conv_latencies.append(lat_s)
        if log:
            log(f"  fifo job {j.job_id} {j.dims} eps={j.eps:.2f}: sweeps {r.sweeps} theta {r.theta:.2e} "
                f"latency {lat_s:.2f} s")
    stats.seconds = gf.gf_clock() - t0
    return stats


def compare_finals(mixed: RunStats, ref: RunStats) -> dict:
    """Per-job final theta and F of a run (mixed precision) against a float64 reference run of the
    same jobs: over the jobs that converged in both, the largest and the median |dF| and |dtheta|,
    and how many landed on another maximum (|dF| > 1e-9: rough inputs whose trajectories part)."""
    both = [k for k, v in mixed.finals.items() if v[0] and k in ref.finals and ref.finals[k][0]]
    if not both:
        return {"jobs_converged_in_both": 0}
    dF = np.array([abs(mixed.finals[k][2] - ref.finals[k][2]) for k in both])
    dth = np.array([abs(mixed.finals[k][1] - ref.finals[k][1]) for k in both])
    same = dF <= 1e-9
    return {"jobs_converged_in_both": len(both), "max_abs_dF": float(dF.max()), "median_abs_dF": float(np.median(dF)),
            "max_abs_dtheta": float(dth.max()), "jobs_same_maximum_dF_le_1e-9": int(same.sum()),
            "max_abs_dF_same_maximum": float(dF[same].max()) if same.any() else None}
