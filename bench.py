"""Benchmark of the checkerboard SU(3) overrelaxation sweep on one MI355X.

Workload (the bandwidth configuration): a 32^4 periodic lattice, links
exp(i eps H) with eps = 0.8 and a Haar gauge rotation (seed 0), overrelaxation
omega = 1.7 (exact SU(2) power), float64 links in the 12-real layout.  One
step = one sweep = the black half-sweep then the white half-sweep = V site
updates; the timed region holds `--steps` sweeps with the links resident in
HBM.  Prints one JSON line.

Extra legs (reported inside the same line): the float32 sweep rate, the 32^4
run to theta < 1e-12 in float64 and in mixed precision (capped; it is also
run on a smoother input of the same generator, eps = 0.6, which converges), a
cpu_baseline of the FP64 CPU oracle on a bounded number of sweeps of the same
lattice (all host cores, and one core), and the serving workload (Poisson arrivals of jobs of mixed volume,
continuous-batching pool in mixed precision vs float64 one lattice at a time:
converged lattices/s and p50/p99 time to theta < 1e-12; `--no-serve` skips
it).  `--batched` and `--fullsize` add the 64-lattice and the 48^3 x 96
workloads.  `--copy-probe` adds a plain device copy of known size (the library's
streaming probe, 1 GiB read + 1 GiB written per dispatch, one warm-up and one
timed dispatch) before the timed region, so that a `rocprofv3 --pmc` run of
this script can scale the HBM counters of the sweep kernel.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published peak
BYTES_PER_SITE = {"f64": 1536, "f32": 768}  # 8 links x 12 reals, read + write
METRIC = "SU(3) OR site-updates/s + HBM GB/s (% peak); converged lattices/s, p99 to θ<1e-12"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "or_sweep_f64_32x4_traffic.md")
SWEEP_SOURCES = ["gf_sweep.hip", "gf_site.h", "gf_device.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_1412_3655_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    or None when it is missing or the sweep kernel changed since."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    src = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not src or not val or src.group(1) != sweep_source_hash():
        return None
    return float(val.group(1))


def time_run(lat, torch, stream, steps, omega, mode, chunk=10):
    """Time `steps` sweeps issued as gf_sweep_or calls of `chunk` sweeps on this stream (2*chunk
    half-sweep kernels per call: launched directly on lattices of >= 2^16 sites per colour, a
    replayed hipGraph below), with a HIP event pair around the whole region and around every
    call.  Returns (region seconds, wall seconds, mean half-sweep kernel seconds = event time
    of a call / its 2*chunk launches)."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.sweep(n, omega, mode)
        e1.record(stream)
        marks.append((e0, e1, n))
        done += n
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches = sum(2 * n for (_, _, n) in marks)
    kernel_s = sum(a.elapsed_time(b) / 1e3 for (a, b, _) in marks)
    return start.elapsed_time(stop) / 1e3, wall, kernel_s / launches


def copy_bandwidth(gf, nbytes=1 << 30, reps=10):
    """Best GB/s (read + write bytes) of the library's plain streaming copy probe over a few
    launch shapes, with and without non-temporal accesses: the practical HBM ceiling."""
    best = {}
    for nt in (False, True):
        for blocks in (1024, 4096, 16384, nbytes // 16 // 256):
            g = gf.gf_probe_copy(nbytes, reps, nt, blocks)
            key = "nontemporal" if nt else "plain"
            best[key] = max(best.get(key, 0.0), g)
    return best


def fix_until_leg(gf, torch, stream, links, dims, args, eps):
    """The run of one input to theta < 1e-12: plain FP64 and FP32-bulk / FP64-polish (GF_MIXED)."""
    out = {"eps": eps}
    kw = dict(omega=args.omega, mode=args.mode, theta_target=1e-12, max_sweeps=args.fix_max_sweeps,
              check_every=10, reunit_every=100, theta_switch=args.theta_switch)
    P0 = None
    for name, prec in (("fp64", gf.GF_FP64), ("mixed", gf.GF_MIXED)):
        with gf.Lattice(dims, prec, stream=stream) as lat:
            lat.set_sweep_config(args.tps, args.block, args.nt, kernel=gf.GF_FP64)
            lat.set_links(links)
            if prec == gf.GF_MIXED:
                # the float32 sweeps of a mixed lattice also update g(x): tuned as their own kernel
                if args.no_tune:
                    lat.set_sweep_config(args.tps32, args.block32, args.nt32, kernel=gf.GF_FP32)
                    out["mixed_fp32_config"] = [args.tps32, args.block32, args.nt32]
                else:
                    out["mixed_fp32_config"] = list(lat.autotune(gf.GF_FP32, n_sweeps=5)[0])
                log(f"fix_until eps={eps}: mixed float32 sweeps with g tracking at {out['mixed_fp32_config']}")
            if P0 is None:
                P0 = lat.plaquette()  # of the float64 input (a mixed lattice starts on float32 links)
            if prec == gf.GF_MIXED:
                floor, sw = lat.tune_switch(1e-12)
                out["fp32_theta_floor"] = floor
                out["theta_switch"] = sw if args.theta_switch < 0 else args.theta_switch
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = lat.fix_until(**kw)
            dt = time.perf_counter() - t0
            P1 = lat.plaquette()
        out[name] = {"seconds": dt, "converged": r.converged, "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_fp32,
                     "sweeps_fp64": r.sweeps_fp64, "theta": r.theta, "F": r.F, "plaquette_drift": abs(P1 - P0)}
        log(f"fix_until eps={eps} {name}: {dt:.2f} s, sweeps {r.sweeps} ({r.sweeps_fp32}/{r.sweeps_fp64}), "
            f"theta {r.theta:.3e}, F {r.F:.12f}")
    out["mixed"]["dF_vs_fp64"] = out["mixed"]["F"] - out["fp64"]["F"]
    out["speedup_mixed_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    return out


def batched_leg(gf, gi, stream, args):
    """64 lattices of uneven volume to theta < 1e-12: mixed-precision pool vs FP64 one at a time."""
    from paper_1412_3655_amd import serving

    jobs = serving.batched_jobs(64, 4)
    t0 = time.perf_counter()
    links = {j.job_id: gi.gen_links(j.dims, j.eps, j.seed) for j in jobs}
    log(f"batched: generated 64 lattices ({sum(serving.volume(j.dims) for j in jobs)} sites) in "
        f"{time.perf_counter() - t0:.1f} s")
    fix = dict(omega=args.omega, mode=args.mode, theta_target=1e-12, max_sweeps=args.job_max_sweeps, check_every=10,
               reunit_every=100, theta_switch=args.theta_switch)
    t32, t64 = args.pool_tps32, args.pool_tps64
    out = {"jobs": 64, "max_sweeps": args.job_max_sweeps, "pool_tps32": t32, "pool_tps64": t64}
    for name, fn in (
        ("pool_mixed", lambda: serving.run_pool(jobs, lambda j: links[j.job_id], gf.GF_MIXED, 10, 64, None, fix,
                                                False, t32, t64)),
        ("pool_fp64", lambda: serving.run_pool(jobs, lambda j: links[j.job_id], gf.GF_FP64, 10, 64, None, fix,
                                               False, t32, t64)),
        ("fifo_fp64", lambda: serving.run_fifo(jobs, lambda j: links[j.job_id], gf.GF_FP64, fix, False, args.tps,
                                               args.block, args.nt)),
    ):
        st = fn()
        out[name] = st.summary()
        log(f"batched {name}: {st.converged}/64 converged in {st.seconds:.2f} s")
    out["speedup_converged_per_s_pool_mixed_vs_fifo_fp64"] = (
        (out["pool_mixed"]["converged_lattices_per_s"] or 0) / out["fifo_fp64"]["converged_lattices_per_s"]
        if out["fifo_fp64"]["converged_lattices_per_s"] else None)
    return out


def serving_leg(gf, gi, stream, args):
    """Poisson arrivals (20/s) of jobs of mixed volume: continuous batching vs FP64 FIFO."""
    from paper_1412_3655_amd import serving

    jobs = serving.serving_trace(args.serve_jobs, 20.0, 5)
    t0 = time.perf_counter()
    bank = {}
    for j in jobs:
        key = (j.dims, j.eps)
        if key not in bank:
            bank[key] = gi.gen_links(j.dims, j.eps, 3000 + len(bank))
    log(f"serving: {len(jobs)} jobs, {len(bank)} distinct inputs generated in {time.perf_counter() - t0:.1f} s")
    fix = dict(omega=args.omega, mode=args.mode, theta_target=1e-12, max_sweeps=args.job_max_sweeps, check_every=10,
               reunit_every=100, theta_switch=args.theta_switch)
    t32, t64 = args.pool_tps32, args.pool_tps64
    links_of = lambda j: bank[(j.dims, j.eps)]
    out = {"jobs": len(jobs), "rate_per_s": 20.0, "max_sweeps": args.job_max_sweeps,
           "distinct_inputs": len(bank), "last_arrival_s": jobs[-1].arrival, "pool_tps32": t32, "pool_tps64": t64}
    budget = int(args.serve_budget_gb * 1e9) if args.serve_budget_gb > 0 else None
    out["hbm_budget_bytes"] = budget
    st = serving.run_pool(jobs, links_of, gf.GF_MIXED, 10, 256, budget, fix, True, t32, t64)
    out["pool_mixed"] = st.summary()
    log(f"serving pool: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s")
    st = serving.run_fifo(jobs, links_of, gf.GF_FP64, fix, True, args.tps, args.block, args.nt)
    out["fifo_fp64"] = st.summary()
    log(f"serving fifo: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s")
    a, b = out["pool_mixed"]["converged_lattices_per_s"], out["fifo_fp64"]["converged_lattices_per_s"]
    out["speedup_converged_per_s_pool_mixed_vs_fifo_fp64"] = a / b if a and b else None
    if args.serve_closed:
        # the same jobs all queued at t = 0: peak throughput, latency counted from t = 0
        closed = {}
        st = serving.run_pool(jobs, links_of, gf.GF_MIXED, 10, 256, budget, fix, False, t32, t64)
        closed["pool_mixed"] = st.summary()
        log(f"serving closed loop pool: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s")
        st = serving.run_fifo(jobs, links_of, gf.GF_FP64, fix, False, args.tps, args.block, args.nt)
        closed["fifo_fp64"] = st.summary()
        log(f"serving closed loop fifo: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s")
        a, b = closed["pool_mixed"]["converged_lattices_per_s"], closed["fifo_fp64"]["converged_lattices_per_s"]
        closed["speedup_converged_per_s_pool_mixed_vs_fifo_fp64"] = a / b if a and b else None
        out["closed_loop"] = closed
    return out


def fullsize_leg(gf, gi, torch, stream, args):
    """The 48^3 x 96 workload (eps = 1.0, seed 0) in mixed precision: 2000 float32 heat-bath sweeps
    on g(x) with T falling linearly from 1.25 to 0.01 (Philox per site), then overrelaxation to
    theta < 1e-13 with float32 bulk, float64 polish and reunitarisation every 100 sweeps."""
    dims = (48, 48, 48, 96)
    V = gi.volume(dims)
    t0 = time.perf_counter()
    u = gi.gen_links(dims, 1.0, 0)
    log(f"fullsize: generated {dims} in {time.perf_counter() - t0:.1f} s")
    out = {"workload": "48x48x48x96, eps=1.0, seed 0; anneal 2000 (T 1.25 -> 0.01), then OR to theta < 1e-13",
           "max_sweeps": args.full_max_sweeps}
    with gf.Lattice(dims, gf.GF_FP64, stream=stream) as lat:
        lat.set_links(u)
        P0 = lat.plaquette()
    with gf.Lattice(dims, gf.GF_MIXED, stream=stream) as lat:
        lat.set_links(u)
        del u
        cfg = {}
        for kernel, name in ((gf.GF_FP32, "f32"), (gf.GF_FP64, "f64")):
            chosen, _ = lat.autotune(kernel, n_sweeps=3)
            cfg[name] = list(chosen)
        chosen, _ = lat.autotune_anneal(gf.GF_FP32, n_sweeps=2)
        cfg["hb_f32"] = list(chosen)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.anneal(2000, 1.25, 0.01, 0)
        th_a, F_a = lat.measure()
        t_anneal = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = lat.fix_until(omega=args.omega, mode=args.mode, theta_target=1e-13, max_sweeps=args.full_max_sweeps,
                          check_every=10, reunit_every=100, theta_switch=args.theta_switch)
        t_fix = time.perf_counter() - t0
        P1 = lat.plaquette()
    out.update({
        "tuned_f32": cfg["f32"], "tuned_f64": cfg["f64"], "tuned_heat_bath_f32": cfg["hb_f32"],
        "anneal_seconds": t_anneal, "anneal_site_updates_per_s": 2000 * V / t_anneal,
        "after_anneal": {"theta": th_a, "F": F_a},
        "fix_seconds": t_fix, "converged": r.converged, "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_fp32,
        "sweeps_fp64": r.sweeps_fp64, "theta": r.theta, "F": r.F,
        "fix_site_updates_per_s": r.sweeps * V / t_fix if t_fix > 0 else None,
        "plaquette_drift": abs(P1 - P0),
    })
    log(f"fullsize: anneal {t_anneal:.1f} s, theta {th_a:.3e}; OR {t_fix:.1f} s, sweeps {r.sweeps} "
        f"({r.sweeps_fp32}/{r.sweeps_fp64}), theta {r.theta:.3e}, converged {r.converged}, |dP| {abs(P1 - P0):.1e}")
    return out


def _time_oracle(oracle, links, dims, omega, mode, budget_s):
    """(sweeps, seconds) of oracle sweeps filling about budget_s, after one untimed sweep."""
    work = links.copy()
    t0 = time.perf_counter()
    oracle.sweep(work, dims, 1, omega, mode)
    first = time.perf_counter() - t0
    n = max(1, min(200, int(budget_s / max(first, 1e-3)) - 1))
    t1 = time.perf_counter()
    oracle.sweep(work, dims, n, omega, mode)
    return n, time.perf_counter() - t1


def cpu_baseline(links, dims, omega, mode, budget_s, budget_1core_s):
    import oracle

    V = links.shape[0]
    cores = oracle.num_threads()
    n, dt = _time_oracle(oracle, links, dims, omega, mode, budget_s)
    out = {
        "value": V * n / dt,
        "unit": "site-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{n} FP64 oracle sweeps of the same {'x'.join(map(str, dims))} lattice (omega={omega}, "
                  f"{'exact' if mode == 0 else 'binomial'} power), after 1 untimed sweep; {dt:.1f} s",
    }
    if budget_1core_s > 0:
        # the same oracle on one core (its results do not depend on the thread count)
        oracle.set_num_threads(1)
        try:
            n1, dt1 = _time_oracle(oracle, links, dims, omega, mode, budget_1core_s)
        finally:
            oracle.set_num_threads(cores)
        out["one_core"] = {"value": V * n1 / dt1, "unit": "site-updates/s", "cores": 1,
                           "sample": f"{n1} sweeps after 1 untimed sweep; {dt1:.1f} s"}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dims", type=str, default="32,32,32,32")
    ap.add_argument("--eps", type=float, default=0.8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--omega", type=float, default=1.7)
    ap.add_argument("--mode", type=int, default=0, help="0 = exact SU(2) power, 1 = binomial form")
    ap.add_argument("--tps", type=int, default=4)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--nt", type=int, default=0,
                    help="cache policy: 0 plain, 1 non-temporal loads and stores, 2 non-temporal stores")
    ap.add_argument("--nt32", type=int, default=0)
    ap.add_argument("--tps32", type=int, default=4)
    ap.add_argument("--block32", type=int, default=256)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--cpu-1core-budget", type=float, default=6.0,
                    help="seconds of single-core oracle work (0: skip the one-core figure)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--chunk", type=int, default=10,
                    help="sweeps per gf_sweep_or call in the timed region (>= 2: replayed hipGraph; 1: direct launches)")
    ap.add_argument("--no-fix", action="store_true", help="skip the run to theta < 1e-12")
    ap.add_argument("--batched", action="store_true", help="also run the 64-lattice batched workload")
    ap.add_argument("--serve", action="store_true", help="(the serving leg runs by default; kept for scripts)")
    ap.add_argument("--no-serve", action="store_true", help="skip the Poisson-arrival serving workload")
    ap.add_argument("--serve-jobs", type=int, default=100)
    ap.add_argument("--serve-closed", action="store_true",
                    help="also run the serving jobs closed loop (all queued at t = 0: peak lattices/s)")
    ap.add_argument("--serve-budget-gb", type=float, default=0.0,
                    help="HBM budget of the serving pool (0: 80 %% of free device memory)")
    ap.add_argument("--pool-tps32", type=int, default=2,
                    help="lanes per site of the pool's float32 sweeps (2: fastest over the batched set on MI355X)")
    ap.add_argument("--pool-tps64", type=int, default=1,
                    help="lanes per site of the pool's float64 sweeps (1: fastest over the batched set on MI355X)")
    ap.add_argument("--fullsize", action="store_true", help="also run the 48^3x96 anneal + mixed-precision workload")
    ap.add_argument("--full-max-sweeps", type=int, default=10000)
    ap.add_argument("--job-max-sweeps", type=int, default=10000)
    ap.add_argument("--fix-max-sweeps", type=int, default=20000)
    ap.add_argument("--fix-eps-smooth", type=float, default=0.6,
                    help="second run to theta < 1e-12 on a smoother input of the same lattice (0: skip)")
    ap.add_argument("--theta-switch", type=float, default=-1.0,
                    help="float32 -> float64 switch of the mixed runs; < 0: chosen by gf_tune_switch")
    ap.add_argument("--no-tune", action="store_true", help="use --tps/--block instead of the autotuner")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (the decomposition of "
              "a lattice over several GPUs is described in the design notes, not implemented)", file=sys.stderr)
        return 2

    import torch

    import gauge_inputs as gi
    from paper_1412_3655_amd import gf

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    dims = tuple(int(x) for x in args.dims.split(","))
    V = gi.volume(dims)
    log(f"generating {dims} eps={args.eps} seed={args.seed}")
    links = gi.gen_links(dims, args.eps, args.seed)
    stream = torch.cuda.Stream()

    if args.copy_probe:
        # one dispatch of a 1 GiB plain copy (1 GiB read, 1 GiB written) to scale HBM counters
        gf.gf_probe_copy(1 << 30, 1, False, 16384)

    result = {}
    tuning = {}
    with gf.Lattice(dims, gf.GF_FP64, stream=stream) as lat:
        lat.set_sweep_config(args.tps, args.block, args.nt)
        lat.set_links(links)
        if not args.no_tune:
            (args.tps, args.block, args.nt), table = lat.autotune(gf.GF_FP64, n_sweeps=5)
            tuning["f64"] = [[t, b, nt, round(us, 1)] for (t, b, nt, us) in table]
            log(f"fp64 autotune: tps={args.tps} block={args.block} cache policy={args.nt}")
        P0 = lat.plaquette()
        log(f"fp64: warmup {args.warmup} sweeps")
        with torch.cuda.stream(stream):
            lat.sweep(args.warmup, args.omega, args.mode)
            lat.sweep(args.chunk, args.omega, args.mode)  # captures the chunk's graph
            total, wall, per_launch = time_run(lat, torch, stream, args.steps, args.omega, args.mode, args.chunk)
            lat.sweep(args.chunk, args.omega, 1 - args.mode)
            total_other, _, _ = time_run(lat, torch, stream, args.steps, args.omega, 1 - args.mode, args.chunk)
        th, F = lat.measure()
        P1 = lat.plaquette()
        log(f"fp64: {args.steps} sweeps in {total * 1e3:.2f} ms (mean half-sweep {per_launch * 1e6:.1f} us); "
            f"theta {th:.3e} F {F:.6f} dP {abs(P1 - P0):.1e}")
        result["f64"] = dict(total=total, wall=wall, per_launch=per_launch, theta=th, F=F, dplaq=abs(P1 - P0),
                             total_other=total_other)

    if not args.no_fp32:
        with gf.Lattice(dims, gf.GF_FP32, stream=stream) as lat:
            lat.set_sweep_config(args.tps32, args.block32, args.nt32)
            lat.set_links(links)
            if not args.no_tune:
                (args.tps32, args.block32, args.nt32), table = lat.autotune(gf.GF_FP32, n_sweeps=5)
                tuning["f32"] = [[t, b, nt, round(us, 1)] for (t, b, nt, us) in table]
                log(f"fp32 autotune: tps={args.tps32} block={args.block32} cache policy={args.nt32}")
            with torch.cuda.stream(stream):
                lat.sweep(args.warmup, args.omega, args.mode)
                lat.sweep(args.chunk, args.omega, args.mode)
                total, wall, per_launch = time_run(lat, torch, stream, args.steps, args.omega, args.mode, args.chunk)
            log(f"fp32: {args.steps} sweeps in {total * 1e3:.2f} ms (mean half-sweep {per_launch * 1e6:.1f} us)")
            result["f32"] = dict(total=total, wall=wall, per_launch=per_launch)

    r64 = result["f64"]
    rate = V * args.steps / r64["total"]
    launch_bytes = (V // 2) * BYTES_PER_SITE["f64"]
    achieved = launch_bytes / r64["per_launch"] / 1e9
    traffic = committed_traffic()
    line = {
        "metric": METRIC,
        "value": rate,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["total"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: exp(i eps H) links + Haar gauge rotation (seeded); no physical ensembles",
        "config": {
            "chunk": args.chunk,
            "workload": f"SU(3) Landau OR sweep, {'x'.join(map(str, dims))} periodic, eps={args.eps}, "
                        f"seed {args.seed}, omega={args.omega}, {'exact' if args.mode == 0 else 'binomial'} "
                        f"power, FP64 12-real links",
            "lattice": list(dims),
            "site_updates_per_step": V,
            "threads_per_site": args.tps,
            "block": args.block,
            "nontemporal": args.nt,
        },
        "hbm_GBps_algorithmic": rate * BYTES_PER_SITE["f64"] / 1e9,
        "pct_hbm_peak": 100.0 * rate * BYTES_PER_SITE["f64"] / 1e9 / HBM_PEAK_GBPS,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "kernel": "k_or_half_sweep<double, TPS=%d, exact, BLOCK=%d, cache policy %d>" % (args.tps, args.block,
                                                                                            args.nt),
            "algorithmic_bytes_per_launch": launch_bytes,
            "mean_launch_us": r64["per_launch"] * 1e6,
        },
        "checks": {"theta_after": r64["theta"], "F_after": r64["F"], "plaquette_drift": r64["dplaq"]},
        "other_or_mode": {
            "mode": "binomial" if args.mode == 0 else "exact",
            "value": V * args.steps / r64["total_other"],
            "unit": "site-updates/s",
        },
    }
    if "f32" in result:
        r32 = result["f32"]
        rate32 = V * args.steps / r32["total"]
        line["fp32"] = {
            "value": rate32,
            "unit": "site-updates/s",
            "hbm_GBps_algorithmic": rate32 * BYTES_PER_SITE["f32"] / 1e9,
            "mean_launch_us": r32["per_launch"] * 1e6,
            "threads_per_site": args.tps32,
            "block": args.block32,
            "nontemporal": args.nt32,
            "note": "201 MB of FP32 links fit in the 256 MB Infinity Cache, so this can exceed HBM peak",
        }
    line["tuning_us_per_sweep"] = tuning or None
    if not args.no_fix:
        line["fix_until_theta_1e-12"] = fix_until_leg(gf, torch, stream, links, dims, args, args.eps)
        if args.fix_eps_smooth > 0:
            log(f"generating {dims} eps={args.fix_eps_smooth} seed={args.seed}")
            smooth = gi.gen_links(dims, args.fix_eps_smooth, args.seed)
            line["fix_until_theta_1e-12_smooth"] = fix_until_leg(gf, torch, stream, smooth, dims, args,
                                                                 args.fix_eps_smooth)
            del smooth
    line["device_copy_GBps"] = copy_bandwidth(gf)
    if args.batched:
        line["batched_64"] = batched_leg(gf, gi, stream, args)
    if not args.no_serve:
        line["serving"] = serving_leg(gf, gi, stream, args)
    if args.fullsize:
        line["fullsize_48x96"] = fullsize_leg(gf, gi, torch, stream, args)
    if not args.no_cpu:
        log("cpu baseline (FP64 oracle)")
        line["cpu_baseline"] = cpu_baseline(links, dims, args.omega, args.mode, args.cpu_budget,
                                            args.cpu_1core_budget)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
