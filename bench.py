"""Benchmark of the checkerboard SU(3) overrelaxation sweep on one MI355X.

Workload (the bandwidth configuration): a 32^4 periodic lattice, links
exp(i eps H) with eps = 0.8 and a Haar gauge rotation (seed 0), overrelaxation
omega = 1.7 (exact SU(2) power), float64 links in the 12-real layout.  One
step = one sweep = the black half-sweep then the white half-sweep = V site
updates; the timed region holds `--steps` sweeps with the links resident in
HBM.  Prints one JSON line.

Extra legs (reported inside the same line; each has a --no-... switch): the
float32 sweep rate; the float64 sweep on the 48^3 x 96 lattice (4.08 GB of
links, far above the 256 MB Infinity Cache: the HBM-only bandwidth point);
the float64 sweeps of both lattices with links stored in 8 reals (the minimal
representation, 1024 B per site update); the float32 sweeps of the 48^3 x 96
lattice with links in 12 and in 8 reals (768 / 512 B per site update); the
32^4 run to theta < 1e-12 in float64 and in mixed precision with float32 links
in 12 and in 8 reals (capped; also on a smoother input of the same generator,
eps = 0.6, which converges, and on the same input after a 2000-sweep
simulated-annealing prelude, which also converges); the
8^4 convergence workload in float64 and mixed precision; the 64-lattice
batched workload (mixed-precision pool, float32 links in 8 reals by default,
vs float64 one lattice at a time); the
serving workload (Poisson arrivals of jobs of mixed volume, continuous-batching
pool in mixed precision under an HBM budget vs float64 one lattice at a time:
converged lattices/s and p50/p99 time to theta < 1e-12); the 48^3 x 96
anneal + mixed-precision workload; and a cpu_baseline of the FP64 CPU oracle
(a bounded number of 32^4 sweeps on all host cores and on one core, and the
8^4 run to theta < 1e-12, against which the GPU's 8^4 results are compared).
The 32^4 input is generated first and alone; the other legs' inputs are
generated on host threads after the 32^4 sweep legs, so that no generator
thread competes with the timed calls.  `--copy-probe` adds a
plain device copy of known size (the library's streaming probe, 1 GiB read +
1 GiB written per dispatch, one warm-up and one timed dispatch) before the
timed region, so that a `rocprofv3 --pmc` run of this script can scale the HBM
counters of the sweep kernel.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published peak
BYTES_PER_SITE = {"f64": 1536, "f32": 768,  # 8 links x 12 reals, read + write
                  "f64_min8": 1024, "f32_min8": 512}  # 8 links x 8 reals (minimal representation), read + write
# Floating-point operations of one overrelaxation site update as the kernel computes it
# (K tracked through the subgroups; exact power; add, sub, mul = 1, FMA = 2, sqrt, div,
# atan2, sin, cos = 1 each): row 2 of 8 links 8 x 42 = 336, K from 8 leaves 7 x 18 = 126,
# 3 subgroups 3 x (8 projection + 14 power) = 66, 2 rotations of K and 2 of G by a
# subgroup element 4 x 84 = 336, rows 0-1 of G U or U G^dag for 8 links 8 x 132 = 1056.
FLOPS_PER_SITE_UPDATE = 336 + 126 + 66 + 336 + 1056
# The paper's 470 GFlops at ~80 % of a GTX 580's 192.4 GB/s with 768-B single-precision site
# updates implies ~2.35e3 flop per site update: its convention, used for a like-for-like figure.
PAPER_FLOPS_PER_SITE_UPDATE = 2350
PAPER_GFLOPS = 470.0
METRIC = "SU(3) OR site-updates/s + HBM GB/s (% peak); converged lattices/s, p99 to θ<1e-12"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "or_sweep_f64_32x4_traffic.md")
TRAFFIC_FILE_48 = os.path.join(ROOT, "profiles", "or_sweep_f64_48x96_traffic.md")
FULL_DIMS = (48, 48, 48, 96)
SWEEP_SOURCES = ["gf_sweep.hip", "gf_sweep_impl.h", "gf_site.h", "gf_device.h"]
# the 8-real sweep also compiles its codec and launcher
MIN8_SOURCES = SWEEP_SOURCES + ["gf_min8.h", "gf_sweep_min8.hip"]
MIN8F_SOURCES = SWEEP_SOURCES + ["gf_min8.h", "gf_sweep_min8f.hip"]
TRAFFIC_FILE_48_F32 = os.path.join(ROOT, "profiles", "or_sweep_f32_48x96_traffic.md")
TRAFFIC_FILE_48_F32_MIN8 = os.path.join(ROOT, "profiles", "or_sweep_f32min8_48x96_traffic.md")
TRAFFIC_FILE_48_MIN8 = os.path.join(ROOT, "profiles", "or_sweep_f64min8_48x96_traffic.md")
TRAFFIC_FILE_32_MIN8 = os.path.join(ROOT, "profiles", "or_sweep_f64min8_32x4_traffic.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sweep_source_hash(sources=SWEEP_SOURCES) -> str:
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_1412_3655_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(path, sources, config):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary, or None when it
    is missing, the sweep kernel changed since, or no counts were taken in the launch
    configuration (tps, block, cache policy) `config`.  The summary holds one line
    `traffic_per_launch: <tps> <block> <policy> <bytes>` per configuration counted."""
    try:
        text = open(path).read()
    except (OSError, TypeError):
        return None
    src = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    if not src or src.group(1) != sweep_source_hash(sources):
        return None
    for m in re.finditer(r"traffic_per_launch:\s*(\d+) (\d+) (\d+) ([0-9.eE+]+)", text):
        if tuple(int(x) for x in m.groups()[:3]) == tuple(config):
            return float(m.group(4))
    return None


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Inputs:
    """The legs' inputs, generated up front several lattices at a time on host threads
    (the generator is deterministic per (dims, eps, seed) whatever thread runs it), so that
    no timed leg waits for the CPU or shares it with generation."""

    def __init__(self, gi, workers):
        self.gi = gi
        self.ex = ThreadPoolExecutor(max(1, workers))
        self.fut = {}

    def want(self, dims, eps, seed):
        key = (tuple(int(d) for d in dims), float(eps), int(seed))
        if key not in self.fut:
            self.fut[key] = self.ex.submit(self.gi.gen_links, *key)
        return key

    def get(self, dims, eps, seed):
        return self.fut[self.want(dims, eps, seed)].result()

    def wait_all(self):
        t0 = time.perf_counter()
        for f in list(self.fut.values()):
            f.result()
        return time.perf_counter() - t0

    def drop(self, dims, eps, seed):
        self.fut.pop((tuple(int(d) for d in dims), float(eps), int(seed)), None)

    def close(self):
        self.ex.shutdown(wait=True)
        self.fut.clear()


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


def fix_until_leg(gf, torch, stream, links, dims, args, eps, adaptive_too=False, anneal=0, max_sweeps=None):
    """The run of one input to theta < 1e-12: plain FP64 and FP32-bulk / FP64-polish (GF_MIXED),
    with exact checks every 10 sweeps, and (adaptive_too) again with adaptive checks (the
    fused estimate decides where the exact measurement runs; same result bitwise).  anneal > 0:
    a simulated-annealing prelude of that many heat-bath sweeps (T 1.25 -> 0.01, Philox key 0)
    first, timed apart, and only the float64 and the 8-real mixed runs."""
    out = {"eps": eps}
    kw = dict(omega=args.omega, mode=args.mode, theta_target=1e-12,
              max_sweeps=max_sweeps or args.fix_max_sweeps, check_every=10, reunit_every=100,
              theta_switch=args.theta_switch)
    if anneal:
        out["anneal_sweeps"] = anneal
    P0 = None
    runs = [("fp64", gf.GF_FP64, False, 12), ("mixed", gf.GF_MIXED, False, 12), ("mixed_min8", gf.GF_MIXED, False, 8)]
    if anneal:
        runs = [runs[0], runs[2]]
    if adaptive_too:
        runs += [("fp64_adaptive", gf.GF_FP64, True, 12), ("mixed_adaptive", gf.GF_MIXED, True, 12)]
    for name, prec, adaptive, storage in runs:
        with gf.Lattice(dims, prec, stream=stream, storage=storage) as lat:
            lat.set_check_policy(adaptive)
            lat.set_sweep_config(args.tps, args.block, args.nt, kernel=gf.GF_FP64, min_waves=args.minw)
            lat.set_links(links)
            if prec == gf.GF_MIXED:
                # the float32 sweeps of a mixed lattice also update g(x): tuned as their own kernel
                key = "mixed_fp32_config" if storage == 12 else "mixed_min8_fp32_config"
                if args.no_tune:
                    lat.set_sweep_config(args.tps32, args.block32, args.nt32, kernel=gf.GF_FP32)
                    out[key] = [args.tps32, args.block32, args.nt32]
                else:
                    out[key] = list(lat.autotune(gf.GF_FP32, n_sweeps=5)[0])
                log(f"fix_until eps={eps}: {name} float32 sweeps with g tracking at {out[key]}")
            if P0 is None:
                P0 = lat.plaquette()  # of the float64 input (a mixed lattice starts on float32 links)
            if prec == gf.GF_MIXED:
                floor, sw = lat.tune_switch(1e-12)
                pre = "" if storage == 12 else "min8_"
                out[pre + "fp32_theta_floor"] = floor
                out[pre + "theta_switch"] = sw if args.theta_switch < 0 else args.theta_switch
            ta = 0.0
            if anneal:
                if prec == gf.GF_MIXED and not args.no_tune:
                    lat.autotune_anneal(gf.GF_FP32, n_sweeps=2)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lat.anneal(anneal, 1.25, 0.01, 0)
                torch.cuda.synchronize()
                ta = time.perf_counter() - t0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = lat.fix_until(**kw)
            dt = time.perf_counter() - t0
            measures, estimates = lat.counters
            P1 = lat.plaquette()
        out[name] = {"seconds": dt, "converged": r.converged, "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_fp32,
                     "sweeps_fp64": r.sweeps_fp64, "theta": r.theta, "F": r.F, "plaquette_drift": abs(P1 - P0),
                     "exact_measurements": measures, "estimates": estimates}
        if anneal:
            out[name]["anneal_seconds"] = ta
            out[name]["total_seconds"] = ta + dt
        log(f"fix_until eps={eps} {name}: {dt:.2f} s, sweeps {r.sweeps} ({r.sweeps_fp32}/{r.sweeps_fp64}), "
            f"theta {r.theta:.3e}, F {r.F:.12f}")
    # the float64 GPU run is the reference here (it is parity-tested against the oracle)
    for name in ("mixed", "mixed_min8"):
        if name not in out:
            continue
        out[name]["dF_vs_fp64"] = out[name]["F"] - out["fp64"]["F"]
        out[name]["dtheta_vs_fp64"] = out[name]["theta"] - out["fp64"]["theta"]
        out["speedup_%s_vs_fp64" % name] = out["fp64"]["seconds"] / out[name]["seconds"]
    if anneal:
        out["note"] = ("the prelude's heat bath takes each input to a different basin than overrelaxation alone; "
                       "on these rough inputs the sweep count to theta < 1e-12 then depends on the precision's "
                       "trajectory, so the two runs' sweep counts differ")
    for name in ("fp64", "mixed"):
        a = out.get(name + "_adaptive")
        if a:
            same = all(a[k] == out[name][k] for k in ("sweeps", "sweeps_fp32", "sweeps_fp64", "theta", "F"))
            a["same_result_as_exact_checks"] = same
            a["speedup_vs_exact_checks"] = out[name]["seconds"] / a["seconds"]
    return out


def batched_leg(gf, inputs, stream, args):
    """64 lattices of uneven volume to theta < 1e-12: mixed-precision pool vs FP64 one at a time
    (and, with --batched-fp64-pool, the float64 pool)."""
    from paper_1412_3655_amd import serving

    jobs = serving.batched_jobs(64, 4)
    links = {j.job_id: inputs.get(j.dims, j.eps, j.seed) for j in jobs}
    fix = dict(omega=args.omega, mode=args.mode, theta_target=1e-12, max_sweeps=args.job_max_sweeps, check_every=10,
               reunit_every=100, theta_switch=args.theta_switch)
    t32, t64 = args.pool_tps32, args.pool_tps64
    out = {"workload": "64 lattices, shapes uniform over {12^4, 16^4, 16^3x32, 24^3x48}, eps uniform in "
                       "[0.4, 1.0] (master seed 4), link seeds 1000+i, to theta < 1e-12",
           "jobs": 64, "sites": sum(serving.volume(j.dims) for j in jobs), "max_sweeps": args.job_max_sweeps,
           "pool_tps32": t32, "pool_tps64": t64}
    tune = not args.no_pool_autotune
    ov = not args.no_overlap
    out["pool_autotune"] = tune
    out["pool_overlap"] = ov
    r32 = args.pool_reals32
    out["pool_float32_reals_per_link"] = r32
    legs = [("pool_mixed", lambda: serving.run_pool(jobs, lambda j: links[j.job_id], gf.GF_MIXED, 10, 64, None,
                                                    fix, False, t32, t64, autotune=tune, overlap=ov, reals32=r32))]
    if args.batched_fp64_pool:
        legs.append(("pool_fp64", lambda: serving.run_pool(jobs, lambda j: links[j.job_id], gf.GF_FP64, 10, 64,
                                                           None, fix, False, t32, t64, autotune=tune, overlap=ov)))
    if not args.no_fifo:
        legs.append(("fifo_fp64", lambda: serving.run_fifo(jobs, lambda j: links[j.job_id], gf.GF_FP64, fix, False,
                                                           args.tps, args.block, args.nt)))
    runs = {}
    for name, fn in legs:
        st = fn()
        runs[name] = st
        out[name] = st.summary()
        log(f"batched {name}: {st.converged}/64 converged in {st.seconds:.2f} s")
    if "fifo_fp64" in runs:
        # final theta and F of every mixed-precision result against the float64 run of the same job
        out["pool_mixed_vs_fifo_fp64_per_result"] = serving.compare_finals(runs["pool_mixed"], runs["fifo_fp64"])
    if "fifo_fp64" in out:
        out["speedup_converged_per_s_pool_mixed_vs_fifo_fp64"] = (
            (out["pool_mixed"]["converged_lattices_per_s"] or 0) / out["fifo_fp64"]["converged_lattices_per_s"]
            if out["fifo_fp64"]["converged_lattices_per_s"] else None)
    return out


def serving_jobs(args):
    from paper_1412_3655_amd import serving

    buckets = (0.4, 0.7, 1.0) if args.serve_eps_buckets else None
    jobs = serving.serving_trace(args.serve_jobs, 20.0, 5, eps_buckets=buckets)
    if buckets:
        # one input per (L, eps), shared by the jobs that draw it
        bank = {}
        for j in jobs:
            bank.setdefault((j.dims, j.eps), 3000 + len(bank))
        return jobs, {j.job_id: bank[(j.dims, j.eps)] for j in jobs}
    return jobs, {j.job_id: j.seed for j in jobs}  # every job its own input, seed 2000 + k


def serving_leg(gf, inputs, stream, args):
    """Poisson arrivals (20/s) of jobs of mixed volume: continuous batching vs FP64 FIFO."""
    from paper_1412_3655_amd import serving

    jobs, seed_of = serving_jobs(args)
    links_of = lambda j: inputs.get(j.dims, j.eps, seed_of[j.job_id])
    if args.serve_eps_buckets:
        eps_text = ("eps drawn uniform in [0.4, 1.0] and rounded to the nearest of {0.4, 0.7, 1.0}, and jobs with "
                    "equal (L, eps) share one input")
    else:
        eps_text = "eps uniform in [0.4, 1.0], every job its own input (link seed 2000 + k)"
    fix = dict(omega=args.omega, mode=args.mode, theta_target=1e-12, max_sweeps=args.job_max_sweeps, check_every=10,
               reunit_every=100, theta_switch=args.theta_switch)
    t32, t64 = args.pool_tps32, args.pool_tps64
    budget = int(args.serve_budget_gb * 1e9) if args.serve_budget_gb > 0 else None
    out = {"workload": f"{len(jobs)} Poisson arrivals at 20/s (master seed 5), L^4 with V log-uniform in "
                       "[8^4, 32^4], 30 % with a 500-sweep anneal (T 1.25 -> 0.01), to theta < 1e-12; " + eps_text,
           "jobs": len(jobs), "rate_per_s": 20.0, "max_sweeps": args.job_max_sweeps,
           "distinct_inputs": len({(j.dims, j.eps, seed_of[j.job_id]) for j in jobs}), "last_arrival_s": jobs[-1].arrival, "pool_tps32": t32, "pool_tps64": t64,
           "hbm_budget_bytes": budget,
           "largest_job_bytes": max(gf.gf_pool_job_bytes(j.dims, gf.GF_MIXED, args.pool_reals32) for j in jobs),
           "pool_overlap": not args.no_overlap}
    ov = not args.no_overlap
    jlog = log if args.serve_verbose else None
    r32 = args.pool_reals32
    out["pool_float32_reals_per_link"] = r32
    st = serving.run_pool(jobs, links_of, gf.GF_MIXED, 10, 256, budget, fix, True, t32, t64, log=jlog, overlap=ov,
                          reals32=r32)
    out["pool_mixed"] = st.summary()
    log(f"serving pool: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s, max queue {st.max_queue}, "
        f"peak {st.peak_bytes / 1e9:.2f} GB")
    if args.no_fifo:
        return out
    st_pool = st
    st = serving.run_fifo(jobs, links_of, gf.GF_FP64, fix, True, args.tps, args.block, args.nt, log=jlog)
    out["fifo_fp64"] = st.summary()
    out["pool_mixed_vs_fifo_fp64_per_result"] = serving.compare_finals(st_pool, st)
    log(f"serving fifo: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s")
    a, b = out["pool_mixed"]["converged_lattices_per_s"], out["fifo_fp64"]["converged_lattices_per_s"]
    out["speedup_converged_per_s_pool_mixed_vs_fifo_fp64"] = a / b if a and b else None
    if args.serve_closed:
        # the same jobs all queued at t = 0: peak throughput, latency counted from t = 0
        closed = {}
        st = serving.run_pool(jobs, links_of, gf.GF_MIXED, 10, 256, budget, fix, False, t32, t64, log=jlog,
                              overlap=ov, reals32=r32)
        closed["pool_mixed"] = st.summary()
        log(f"serving closed loop pool: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s")
        st = serving.run_fifo(jobs, links_of, gf.GF_FP64, fix, False, args.tps, args.block, args.nt, log=jlog)
        closed["fifo_fp64"] = st.summary()
        log(f"serving closed loop fifo: {st.converged}/{len(jobs)} converged, {st.seconds:.1f} s")
        a, b = closed["pool_mixed"]["converged_lattices_per_s"], closed["fifo_fp64"]["converged_lattices_per_s"]
        closed["speedup_converged_per_s_pool_mixed_vs_fifo_fp64"] = a / b if a and b else None
        out["closed_loop"] = closed
    return out


def fullsize_f64_leg(gf, torch, stream, u, args):
    """Float64 overrelaxation sweep on 48^3 x 96 (eps = 1.0, seed 0): 4.08 GB of links against a
    256 MB Infinity Cache, so the half-sweep streams from HBM: the clean bandwidth point."""
    return sweep_leg(gf, torch, stream, u, FULL_DIMS, args, args.full_steps, 12, "eps=1.0, seed 0",
                     TRAFFIC_FILE_48)


def sweep_leg(gf, torch, stream, u, dims, args, steps, storage, input_name, traffic_file=None, prec=None):
    """Tune, warm up and time `steps` overrelaxation sweeps of one float64 (prec GF_FP64) or float32
    (GF_FP32) lattice whose links are stored in `storage` reals (12: two rows; 8: the minimal
    representation)."""
    prec = gf.GF_FP64 if prec is None else prec
    f32 = prec == gf.GF_FP32
    tag = "fp32" if f32 else "fp64"
    V = u.shape[0]
    name = "x".join(map(str, dims))
    with gf.Lattice(dims, prec, stream=stream, storage=storage) as lat:
        lat.set_links(u)
        if args.no_tune:
            (tps, block, nt, minw), table = ((args.tps32, args.block32, args.nt32, 0) if f32 else
                                             (args.tps, args.block, args.nt, args.minw) if storage == 12 else
                                             (args.tps8, args.block8, args.nt8, 0)), []
            lat.set_sweep_config(tps, block, nt, min_waves=minw)
        else:
            (tps, block, nt, minw), table = lat.autotune(prec, n_sweeps=3)
        log(f"{name} {tag}/{storage}: tps={tps} block={block} cache policy={nt} min waves={minw}")
        with torch.cuda.stream(stream):
            lat.sweep(args.warmup, args.omega, args.mode)
            total, wall, per_launch = time_run(lat, torch, stream, steps, args.omega, args.mode, args.chunk)
        th, F = lat.measure()
    rate = V * steps / total
    bps = BYTES_PER_SITE[tag.replace("fp", "f") + ("" if storage == 12 else "_min8")]
    launch_bytes = (V // 2) * bps
    achieved = launch_bytes / per_launch / 1e9
    log(f"{name} {tag}/{storage}: {steps} sweeps in {total * 1e3:.1f} ms (mean half-sweep {per_launch * 1e6:.1f} us, "
        f"{achieved:.0f} GB/s)")
    return {
        "workload": "SU(3) Landau OR sweep, %s periodic, %s, omega=%g, %s power, %s %d-real links" % (
            name, input_name, args.omega, "exact" if args.mode == 0 else "binomial", tag.upper(), storage),
        "steps": steps,
        "value": rate,
        "unit": "site-updates/s",
        "ms_per_step": total * 1e3 / steps,
        "gflops": rate * FLOPS_PER_SITE_UPDATE / 1e9,
        "threads_per_site": tps, "block": block, "nontemporal": nt, "min_waves": minw,
        "tuning_us_per_sweep": [[t, b, c, w, round(us, 1)] for (t, b, c, w, us) in table],
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": committed_traffic(traffic_file, (MIN8F_SOURCES if f32 else MIN8_SOURCES) if storage == 8
                                         else SWEEP_SOURCES, (tps, block, nt)),
            "kernel": "k_or_half_sweep<%s, TPS=%d, exact, BLOCK=%d, cache policy %d%s%s>" % (
                "float" if f32 else "double", tps, block, nt, ", 2 waves/SIMD" if minw == 2 else "",
                ", 8-real links" if storage == 8 else ""),
            "algorithmic_bytes_per_launch": launch_bytes,
            "bytes_per_site_update": bps,
            "mean_launch_us": per_launch * 1e6,
        },
        "checks": {"theta_after": th, "F_after": F},
    }


def min8_legs(gf, torch, stream, links, dims, full, args):
    """Beside the 12-real figures: the same float64 sweeps with links stored in 8 reals (1024 B per
    site update instead of 1536 B), on the bandwidth lattice and on 48^3 x 96."""
    out = {"bytes_per_site_update": BYTES_PER_SITE["f64_min8"]}
    out["bandwidth_lattice"] = sweep_leg(gf, torch, stream, links, dims, args, args.steps, 8,
                                         f"eps={args.eps}, seed {args.seed}",
                                         TRAFFIC_FILE_48_MIN8 if tuple(dims) == FULL_DIMS else
                                         TRAFFIC_FILE_32_MIN8 if tuple(dims) == (32, 32, 32, 32) else None)
    if full is not None:
        out["fullsize_48x96"] = sweep_leg(gf, torch, stream, full, FULL_DIMS, args, args.full_steps, 8,
                                          "eps=1.0, seed 0", TRAFFIC_FILE_48_MIN8)
    # the storage as a tuning axis: both storages timed on each lattice, the faster kept
    for name, u, d in (("bandwidth_lattice", links, dims), ("fullsize_48x96", full, FULL_DIMS)):
        if u is None:
            continue
        with gf.Lattice(d, gf.GF_FP64, stream=stream) as lat:
            lat.set_links(u)
            reals, us12, us8 = lat.autotune_storage(3)
        log(f"{'x'.join(map(str, d))} storage autotune: {reals} reals (12: {us12:.1f} us, 8: {us8:.1f} us per sweep)")
        out.setdefault("storage_autotune", {})[name] = {"chosen_reals_per_link": reals,
                                                        "us_per_sweep_12": us12, "us_per_sweep_8": us8}
    return out


def fullsize_f32_legs(gf, torch, stream, full, args):
    """Float32 overrelaxation sweeps on 48^3 x 96 (HBM-bound: 2.04 GB of 12-real float32 links)
    with links in 12 reals (768 B per site update) and in 8 reals (512 B), and the storage tuner's
    choice between them."""
    out = {}
    for storage, tf in ((12, TRAFFIC_FILE_48_F32), (8, TRAFFIC_FILE_48_F32_MIN8)):
        out["reals_%d" % storage] = sweep_leg(gf, torch, stream, full, FULL_DIMS, args, args.full_steps, storage,
                                              "eps=1.0, seed 0", tf, prec=gf.GF_FP32)
    with gf.Lattice(FULL_DIMS, gf.GF_FP32, stream=stream) as lat:
        lat.set_links(full)
        reals, us12, us8 = lat.autotune_storage(3)
    out["storage_autotune"] = {"chosen_reals_per_link": reals, "us_per_sweep_12": us12, "us_per_sweep_8": us8}
    out["speedup_8_vs_12"] = out["reals_8"]["value"] / out["reals_12"]["value"]
    log(f"48x96 fp32: 8 reals {out['speedup_8_vs_12']:.2f}x the 12-real sweep rate; tuner chose {reals}")
    return out


def fullsize_leg(gf, torch, stream, u, args):
    """The 48^3 x 96 workload (eps = 1.0, seed 0) in mixed precision: 2000 float32 heat-bath sweeps
    on g(x) with T falling linearly from 1.25 to 0.01 (Philox per site), then overrelaxation to
    theta < 1e-13 with float32 bulk, float64 polish and reunitarisation every 100 sweeps."""
    dims = FULL_DIMS
    V = u.shape[0]
    out = {"workload": "48x48x48x96, eps=1.0, seed 0; anneal 2000 (T 1.25 -> 0.01), then OR to theta < 1e-13; "
                       "float32 links in the storage the tuner picks",
           "max_sweeps": args.full_max_sweeps}
    with gf.Lattice(dims, gf.GF_FP64, stream=stream) as lat:
        lat.set_links(u)
        P0 = lat.plaquette()
    with gf.Lattice(dims, gf.GF_MIXED, stream=stream) as lat:
        lat.set_links(u)
        cfg = {}
        # the float32 links' storage (12 or 8 reals) as a tuning axis, then every kernel's shape
        reals, us12, us8 = lat.autotune_storage(3)
        out["float32_storage"] = {"chosen_reals_per_link": reals, "us_per_sweep_12": us12, "us_per_sweep_8": us8}
        log(f"fullsize mixed: float32 links in {reals} reals (12: {us12:.0f} us, 8: {us8:.0f} us per sweep)")
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


def fix_8x4_leg(gf, torch, u, args):
    """The 8^4 convergence workload (eps = 0.6, seed 0, omega 1.7, checked every sweep,
    reunitarised every 100) in float64 and in mixed precision on the GPU; the oracle's run of the
    same input is timed and compared in the cpu_baseline leg."""
    dims = (8, 8, 8, 8)
    out = {}
    for name, prec in (("fp64", gf.GF_FP64), ("mixed", gf.GF_MIXED)):
        with gf.Lattice(dims, prec) as lat:
            lat.set_links(u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = lat.fix_until(omega=1.7, mode=0, theta_target=1e-12, max_sweeps=3000, check_every=1,
                              reunit_every=100, theta_switch=args.theta_switch)
            dt = time.perf_counter() - t0
            links = lat.get_links()
        out[name] = {"seconds": dt, "converged": r.converged, "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_fp32,
                     "sweeps_fp64": r.sweeps_fp64, "theta": r.theta, "F": r.F, "links": links}
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


def cpu_baseline(links, dims, omega, mode, budget_s, budget_1core_s, fix8=None, u8=None):
    import numpy as np

    import oracle

    V = links.shape[0]
    cores = oracle.num_threads()
    n, dt = _time_oracle(oracle, links, dims, omega, mode, budget_s)
    out = {
        "value": V * n / dt,
        "unit": "site-updates/s",
        "cores": cores,
        "cpu_model": host_cpu_model(),
        "kind": "oracle",
        "sample": f"{n} FP64 oracle sweeps of the same {'x'.join(map(str, dims))} lattice (omega={omega}, "
                  f"{'exact' if mode == 0 else 'binomial'} power), after 1 untimed sweep; {dt:.1f} s",
    }
    out["hbm_equivalent_GBps"] = out["value"] * BYTES_PER_SITE["f64"] / 1e9
    if budget_1core_s > 0:
        # the same oracle on one core (its results do not depend on the thread count)
        oracle.set_num_threads(1)
        try:
            n1, dt1 = _time_oracle(oracle, links, dims, omega, mode, budget_1core_s)
        finally:
            oracle.set_num_threads(cores)
        out["one_core"] = {"value": V * n1 / dt1, "unit": "site-updates/s", "cores": 1,
                           "sample": f"{n1} sweeps after 1 untimed sweep; {dt1:.1f} s"}
    if fix8 is not None:
        # the 8^4 convergence workload through the oracle: its time to theta < 1e-12, and the GPU
        # float64 and mixed-precision results' errors against it
        d8 = (8, 8, 8, 8)
        ref = u8.copy()
        t0 = time.perf_counter()
        r = oracle.fix_until(ref, d8, 1.7, 0, 1e-12, 3000, 1, 100)
        t_or = time.perf_counter() - t0
        cmp = {"workload": "8^4, eps=0.6, seed 0, omega 1.7, exact power, checked every sweep, reunitarised "
                           "every 100, to theta < 1e-12 (3000 sweeps at most)",
               "oracle": {"seconds": t_or, "converged": r["converged"], "sweeps": r["sweeps"], "theta": r["theta"],
                          "F": r["F"], "threads": 1}}  # 4096 sites: below the oracle's OpenMP threshold
        for name, g in fix8.items():
            cmp["gpu_" + name] = {
                "seconds": g["seconds"], "converged": g["converged"], "sweeps": g["sweeps"],
                "sweeps_fp32": g["sweeps_fp32"], "sweeps_fp64": g["sweeps_fp64"], "theta": g["theta"], "F": g["F"],
                "theta_minus_oracle": g["theta"] - r["theta"], "F_minus_oracle": g["F"] - r["F"],
                "max_abs_links_minus_oracle": float(np.abs(g["links"] - ref).max()),
            }
        out["fix_8x4"] = cmp
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed regions of --steps sweeps after the headline one (median and spread)")
    ap.add_argument("--dims", type=str, default="32,32,32,32")
    ap.add_argument("--eps", type=float, default=0.8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--omega", type=float, default=1.7)
    ap.add_argument("--mode", type=int, default=0, help="0 = exact SU(2) power, 1 = binomial form")
    ap.add_argument("--tps", type=int, default=4)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--nt", type=int, default=0,
                    help="cache policy: 0 plain, 1 non-temporal loads and stores, 2 non-temporal stores")
    ap.add_argument("--minw", type=int, default=0,
                    help="register limit of the float64 sweep: 0 compiler's allocation, 2 at least 2 waves per SIMD")
    ap.add_argument("--tps8", type=int, default=2, help="with --no-tune: lanes per site of the 8-real sweeps")
    ap.add_argument("--block8", type=int, default=128, help="with --no-tune: block of the 8-real sweeps")
    ap.add_argument("--nt8", type=int, default=1, help="with --no-tune: cache policy of the 8-real sweeps")
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
    ap.add_argument("--no-fix", action="store_true", help="skip the runs to theta < 1e-12 (32^4 and 8^4)")
    ap.add_argument("--no-min8", action="store_true",
                    help="skip the float64 sweeps with links stored in 8 reals (bandwidth lattice and 48^3x96)")
    ap.add_argument("--batched", action="store_true", help="(the batched leg runs by default; kept for scripts)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-lattice batched workload")
    ap.add_argument("--batched-fp64-pool", action="store_true", help="also run the batched jobs in a float64 pool")
    ap.add_argument("--serve", action="store_true", help="(the serving leg runs by default; kept for scripts)")
    ap.add_argument("--no-serve", action="store_true", help="skip the Poisson-arrival serving workload")
    ap.add_argument("--serve-jobs", type=int, default=100)
    ap.add_argument("--serve-eps-buckets", action="store_true",
                    help="serving leg: round eps to the nearest of {0.4, 0.7, 1.0} and share one input per (L, eps) "
                         "(host memory and generation time of long traces)")
    ap.add_argument("--serve-verbose", action="store_true", help="log every finished serving job")
    ap.add_argument("--serve-closed", action="store_true",
                    help="also run the serving jobs closed loop (all queued at t = 0: peak lattices/s)")
    ap.add_argument("--serve-budget-gb", type=float, default=4.0,
                    help="HBM budget of the serving pool in GB (0: 80 %% of free device memory)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="batched and serving pools: step, retire and admit one after another instead of "
                         "retiring and admitting while the next step runs")
    ap.add_argument("--no-fifo", action="store_true",
                    help="batched and serving legs: skip the float64 one-lattice-at-a-time comparison")
    ap.add_argument("--pool-reals32", type=int, default=8, choices=(8, 12),
                    help="batched and serving pools: reals per float32 link (8: the minimal representation)")
    ap.add_argument("--pool-tps32", type=int, default=0,
                    help="lanes per site of the pool's float32 sweeps (0: the library's default, 1 with 8-real "
                         "links and 2 with 12-real links, the fastest over the batched set on MI355X)")
    ap.add_argument("--no-pool-autotune", action="store_true",
                    help="batched leg: keep the pool's default sweep shape instead of gf_pool_autotune")
    ap.add_argument("--pool-tps64", type=int, default=0,
                    help="lanes per site of the pool's float64 sweeps (0: the library's default, 1, the fastest "
                         "over the batched set on MI355X)")
    ap.add_argument("--fullsize", action="store_true", help="(the 48^3x96 legs run by default; kept for scripts)")
    ap.add_argument("--no-fullsize", action="store_true",
                    help="skip the 48^3x96 float64 sweep and the 48^3x96 anneal + mixed-precision workload")
    ap.add_argument("--no-fullsize-pipeline", action="store_true",
                    help="run the 48^3x96 float64 sweep but not the anneal + mixed-precision workload")
    ap.add_argument("--full-steps", type=int, default=40, help="timed float64 sweeps of the 48^3x96 lattice")
    ap.add_argument("--full-max-sweeps", type=int, default=10000)
    ap.add_argument("--job-max-sweeps", type=int, default=10000)
    ap.add_argument("--fix-max-sweeps", type=int, default=20000)
    ap.add_argument("--fix-anneal", type=int, default=2000,
                    help="the 32^4 input again with a simulated-annealing prelude of this many heat-bath sweeps "
                         "before the run to theta < 1e-12 (0: skip)")
    ap.add_argument("--fix-anneal-max-sweeps", type=int, default=200000)
    ap.add_argument("--fix-eps-smooth", type=float, default=0.6,
                    help="second run to theta < 1e-12 on a smoother input of the same lattice (0: skip)")
    ap.add_argument("--theta-switch", type=float, default=-1.0,
                    help="float32 -> float64 switch of the mixed runs; < 0: chosen by gf_tune_switch")
    ap.add_argument("--no-tune", action="store_true",
                    help="use --tps/--block/--nt (12-real) and --tps8/--block8/--nt8 (8-real) instead of the autotuner")
    ap.add_argument("--gen-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads generating the inputs up front")
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

    # the 32^4 input first and alone: its sweep legs are timed with HIP events around calls
    # issued from this thread, and generator threads competing for the interpreter lock
    # would open gaps between those calls; every other leg's input is generated on host
    # threads after those legs, and those legs wait until generation is done
    inputs = Inputs(gi, args.gen_threads)
    links = inputs.get(dims, args.eps, args.seed)

    def want_the_rest():
        if not args.no_fix:
            inputs.want((8, 8, 8, 8), 0.6, 0)
            if args.fix_eps_smooth > 0:
                inputs.want(dims, args.fix_eps_smooth, args.seed)
        if not args.no_fullsize:
            inputs.want(FULL_DIMS, 1.0, 0)
        if not args.no_batched:
            from paper_1412_3655_amd import serving

            for j in serving.batched_jobs(64, 4):
                inputs.want(j.dims, j.eps, j.seed)
        if not args.no_serve:
            sjobs, seed_of = serving_jobs(args)
            for j in sjobs:
                inputs.want(j.dims, j.eps, seed_of[j.job_id])
        log(f"generating {len(inputs.fut)} inputs on {args.gen_threads} threads")
    stream = torch.cuda.Stream()

    if args.copy_probe:
        # one dispatch of a 1 GiB plain copy (1 GiB read, 1 GiB written) to scale HBM counters
        gf.gf_probe_copy(1 << 30, 1, False, 16384)

    result = {}
    tuning = {}
    with gf.Lattice(dims, gf.GF_FP64, stream=stream) as lat:
        lat.set_sweep_config(args.tps, args.block, args.nt, min_waves=args.minw)
        lat.set_links(links)
        if not args.no_tune:
            (args.tps, args.block, args.nt, args.minw), table = lat.autotune(gf.GF_FP64, n_sweeps=5)
            tuning["f64"] = [[t, b, nt, w, round(us, 1)] for (t, b, nt, w, us) in table]
            log(f"fp64 autotune: tps={args.tps} block={args.block} cache policy={args.nt} min waves={args.minw}")
        P0 = lat.plaquette()
        log(f"fp64: warmup {args.warmup} sweeps")
        with torch.cuda.stream(stream):
            lat.sweep(args.warmup, args.omega, args.mode)
            lat.sweep(args.chunk, args.omega, args.mode)  # captures the chunk's graph
            total, wall, per_launch = time_run(lat, torch, stream, args.steps, args.omega, args.mode, args.chunk)
            # further timed regions of the same length, reported beside the headline region
            repeats = [time_run(lat, torch, stream, args.steps, args.omega, args.mode, args.chunk)
                       for _ in range(args.repeats)]
            lat.sweep(args.chunk, args.omega, 1 - args.mode)
            total_other, _, _ = time_run(lat, torch, stream, args.steps, args.omega, 1 - args.mode, args.chunk)
        th, F = lat.measure()
        P1 = lat.plaquette()
        log(f"fp64: {args.steps} sweeps in {total * 1e3:.2f} ms (mean half-sweep {per_launch * 1e6:.1f} us); "
            f"theta {th:.3e} F {F:.6f} dP {abs(P1 - P0):.1e}")
        result["f64"] = dict(total=total, wall=wall, per_launch=per_launch, theta=th, F=F, dplaq=abs(P1 - P0),
                             total_other=total_other, repeats=repeats)

    if not args.no_fp32:
        with gf.Lattice(dims, gf.GF_FP32, stream=stream) as lat:
            lat.set_sweep_config(args.tps32, args.block32, args.nt32)
            lat.set_links(links)
            if not args.no_tune:
                (args.tps32, args.block32, args.nt32, _), table = lat.autotune(gf.GF_FP32, n_sweeps=5)
                tuning["f32"] = [[t, b, nt, round(us, 1)] for (t, b, nt, _, us) in table]
                log(f"fp32 autotune: tps={args.tps32} block={args.block32} cache policy={args.nt32}")
            with torch.cuda.stream(stream):
                lat.sweep(args.warmup, args.omega, args.mode)
                lat.sweep(args.chunk, args.omega, args.mode)
                total, wall, per_launch = time_run(lat, torch, stream, args.steps, args.omega, args.mode, args.chunk)
            log(f"fp32: {args.steps} sweeps in {total * 1e3:.2f} ms (mean half-sweep {per_launch * 1e6:.1f} us)")
            result["f32"] = dict(total=total, wall=wall, per_launch=per_launch)

    t_gen1 = time.perf_counter()
    want_the_rest()
    waited = inputs.wait_all()
    t_gen = time.perf_counter() - t_gen1
    log(f"inputs of the other legs ready {t_gen:.1f} s after the 32^4 sweep legs")

    r64 = result["f64"]
    rate = V * args.steps / r64["total"]
    launch_bytes = (V // 2) * BYTES_PER_SITE["f64"]
    achieved = launch_bytes / r64["per_launch"] / 1e9
    traffic = committed_traffic(TRAFFIC_FILE if tuple(dims) == (32, 32, 32, 32) else
                                TRAFFIC_FILE_48 if tuple(dims) == FULL_DIMS else None, SWEEP_SOURCES,
                                (args.tps, args.block, args.nt))
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
            "min_waves": args.minw,
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
            "kernel": "k_or_half_sweep<double, TPS=%d, exact, BLOCK=%d, cache policy %d%s>" % (
                args.tps, args.block, args.nt, ", 2 waves/SIMD" if args.minw == 2 else ""),
            "algorithmic_bytes_per_launch": launch_bytes,
            "mean_launch_us": r64["per_launch"] * 1e6,
            "note": "the 403 MB float64 field partly fits the 256 MB Infinity Cache, which the reversed white "
                    "half-sweep reuses; fullsize_48x96_f64 is the HBM-only point",
        },
        "gflops": {
            "value": rate * FLOPS_PER_SITE_UPDATE / 1e9,
            "flops_per_site_update": FLOPS_PER_SITE_UPDATE,
            "value_paper_convention": rate * PAPER_FLOPS_PER_SITE_UPDATE / 1e9,
            "paper_flops_per_site_update": PAPER_FLOPS_PER_SITE_UPDATE,
            "paper_gflops_gtx580": PAPER_GFLOPS,
            "note": "the paper's figure: up to 470 GFlops at ~80 % of a GeForce GTX 580's bandwidth (context, "
                    "another machine and precision)",
        },
        "checks": {"theta_after": r64["theta"], "F_after": r64["F"], "plaquette_drift": r64["dplaq"]},
        "other_or_mode": {
            "mode": "binomial" if args.mode == 0 else "exact",
            "value": V * args.steps / r64["total_other"],
            "unit": "site-updates/s",
        },
        "input_generation_s": t_gen,
    }
    if r64["repeats"]:
        reps = sorted(V * args.steps / t for (t, _, _) in r64["repeats"])
        line["repeats"] = {
            "count": len(reps),
            "value_median": reps[len(reps) // 2],
            "value_min": reps[0],
            "value_max": reps[-1],
            "mean_launch_us": [round(p * 1e6, 2) for (_, _, p) in r64["repeats"]],
            "note": "further timed regions of --steps sweeps each, after the headline region",
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
    full = None
    if not args.no_fullsize:
        full = inputs.get(FULL_DIMS, 1.0, 0)
        line["fullsize_48x96_f64"] = fullsize_f64_leg(gf, torch, stream, full, args)
    if not args.no_min8:
        line["f64_min8"] = min8_legs(gf, torch, stream, links, dims, full, args)
    if not args.no_fullsize and not args.no_fp32:
        line["fullsize_48x96_f32"] = fullsize_f32_legs(gf, torch, stream, full, args)
    del full
    fix8 = None
    if not args.no_fix:
        line["fix_until_theta_1e-12"] = fix_until_leg(gf, torch, stream, links, dims, args, args.eps)
        if args.fix_anneal > 0:
            line["fix_until_theta_1e-12_annealed"] = fix_until_leg(gf, torch, stream, links, dims, args, args.eps,
                                                                   anneal=args.fix_anneal,
                                                                   max_sweeps=args.fix_anneal_max_sweeps)
        if args.fix_eps_smooth > 0:
            smooth = inputs.get(dims, args.fix_eps_smooth, args.seed)
            line["fix_until_theta_1e-12_smooth"] = fix_until_leg(gf, torch, stream, smooth, dims, args,
                                                                 args.fix_eps_smooth, adaptive_too=True)
            inputs.drop(dims, args.fix_eps_smooth, args.seed)
            del smooth
        fix8 = fix_8x4_leg(gf, torch, inputs.get((8, 8, 8, 8), 0.6, 0), args)
        line["fix_8x4"] = {k: {kk: vv for kk, vv in v.items() if kk != "links"} for k, v in fix8.items()}
    line["device_copy_GBps"] = copy_bandwidth(gf)
    copy_best = max(line["device_copy_GBps"].values())
    line["roofline"]["frac_of_copy"] = line["roofline"]["achieved"] / copy_best
    for leg in (line.get("fullsize_48x96_f64"), *(line.get("f64_min8", {}).get(k) for k in
                                                  ("bandwidth_lattice", "fullsize_48x96"))):
        if leg:
            leg["roofline"]["frac_of_copy"] = leg["roofline"]["achieved"] / copy_best
    if not args.no_batched:
        line["batched_64"] = batched_leg(gf, inputs, stream, args)
    if not args.no_serve:
        line["serving"] = serving_leg(gf, inputs, stream, args)
    if not args.no_fullsize and not args.no_fullsize_pipeline:
        line["fullsize_48x96"] = fullsize_leg(gf, torch, stream, inputs.get(FULL_DIMS, 1.0, 0), args)
    if not args.no_fullsize:
        inputs.drop(FULL_DIMS, 1.0, 0)
    if not args.no_cpu:
        log("cpu baseline (FP64 oracle)")
        line["cpu_baseline"] = cpu_baseline(links, dims, args.omega, args.mode, args.cpu_budget,
                                            args.cpu_1core_budget, fix8,
                                            inputs.get((8, 8, 8, 8), 0.6, 0) if fix8 else None)
    else:
        line["cpu_baseline"] = None
    inputs.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
