#!/usr/bin/env python3
"""Benchmark of the 2D EM-PIC step on one MI355X.

A step is one pass of the whole hot path over the resident simulation:
interpolate + Boris push + charge-conserving deposit + tile hand-off
(k_push_deposit), current fold, binomial filter, Yee field advance and the
step bookkeeping.  The default workload is the two counter-streaming electron
clouds on a periodic 1024 x 1024 grid (16,777,216 particles, 16 per cell per
species), whose particle arrays (0.4 GB read and written per step) are larger
than the 256 MB Infinity Cache, so the push kernel streams from HBM.

Prints one JSON line: whole-job throughput in particle pushes per second over
K timed steps (inputs resident in HBM), the roofline of the dominant kernel
(k_push_deposit, HBM-bound) from HIP events, step-latency percentiles and the
FP64 CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = ("particle pushes/sec (push+deposit, FP32) vs HBM roofline; "
          "p50/p99 batched step latency")

# algorithmic HBM bytes of k_push_deposit: per particle the state read and
# written once (packed cell int32 + x, y, ux, uy, uz), per cell the six field
# components read once and the three current components written once
BYTES_PER_PARTICLE = {False: 2 * (4 + 5 * 4), True: 2 * (4 + 5 * 8)}
BYTES_PER_CELL = {False: (6 + 3) * 4, True: (6 + 3) * 8}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_push_deposit_clouds_1024x1024_traffic.md")


def measured_traffic():
    """HBM bytes per k_push_deposit launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (calibrated on a plain copy), or None if
    that summary was taken on other kernel sources or build flags than the
    current ones."""
    import hashlib
    try:
        vals = {}
        for line in open(TRAFFIC_PROFILE):
            parts = line.split()
            if len(parts) == 2 and parts[0].endswith(("sha256", "per_launch")):
                vals[parts[0]] = parts[1]
        pkg = os.path.join(ROOT, "paper_2106_12485_amd")
        src = os.path.join(pkg, "csrc")
        kh = hashlib.sha256(open(os.path.join(src, "pic_kernels.hip"), "rb").read()).hexdigest()
        hh = hashlib.sha256(open(os.path.join(src, "pic_dev.h"), "rb").read()).hexdigest()
        # the compiler flags live in build.py
        bh = hashlib.sha256(open(os.path.join(pkg, "build.py"), "rb").read()).hexdigest()
        if (vals.get("kernel_source_sha256") != kh or vals.get("header_source_sha256") != hh
                or vals.get("build_source_sha256") != bh):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="clouds_1024x1024")
    ap.add_argument("--deposit", default="reduction", choices=("reduction", "commutative"),
                    help="how tiles' currents are combined: per-tile blocks summed by a fold "
                         "launch, or four checkerboard colours adding straight into J")
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=5,
                    help="oracle steps timed for the CPU baseline (0 = skip)")
    ap.add_argument("--cpu-coverage", action="store_true",
                    help="only time the oracle over the measurement plan's coverage (the "
                         "64x64 and 2000x256 runs in full, 20 steps of the two clouds, 64 "
                         "steps of the 8000x512 run in the parallel-for mode) and print it")
    ap.add_argument("--clock-warmup-s", type=float, default=0.3,
                    help="untimed, before the measured run: seconds of steps of a throwaway "
                         "copy of the workload, so that the GPU's clocks have left their idle "
                         "state (0 = skip; skipped with --profile-only)")
    ap.add_argument("--phase-step", type=int, default=500,
                    help="first step of the second timed window (0 = skip it)")
    ap.add_argument("--profile-only", action="store_true",
                    help="warm-up and timed steps only (for rocprofv3)")
    ap.add_argument("--direct", action="store_true",
                    help="with --profile-only: launch kernels directly, not from the graph")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the serving leg (0 = skip it)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg and print its JSON")
    ap.add_argument("--budget-gb", type=float, default=32.0,
                    help="HBM budget of the serving loop")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def progress(msg):
    """One line on stderr when a stage of the run ends (stdout keeps the JSON)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def copy_peak_gbs(mib=1024, reps=5):
    """Measured device-copy bandwidth (read + write bytes per second), the
    practical ceiling of a streaming kernel on this GPU, best of reps."""
    import torch
    n = mib * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (best * 1e-3) / 1e9


def clock_warmup(w, fp64, deposit, seconds):
    """Step a throwaway copy of workload w for `seconds` of wall time, then
    free it.  A GPU that was idle runs its first tens of milliseconds of
    work at lower clocks (the two-cloud push took 250-260 us per launch over
    the first steps after a cold start, ~210 us on a warm GPU), so the
    measured run starts after this.  Returns the steps done."""
    import torch
    from paper_2106_12485_amd import Simulation
    tmp = Simulation(w, fp64=fp64, deposit=deposit)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        tmp.step(16)
        torch.cuda.synchronize()
        n += 16
    tmp.close()
    del tmp
    torch.cuda.empty_cache()
    return n


def copy_calibration(mib):
    import torch
    n = mib * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=n * 4, launches=5)))


def serving_leg(nreq, budget_gb, chunk=10, rate_ratio=4, max_particles=1 << 24,
                lone_particles=1 << 22):
    """Stream of independent periodic plasmas (grids 64^2..512^2, 4/16/64 ppc,
    thermal or two-stream, 200 steps each) served within an HBM budget: every
    request present at t = 0, then Poisson arrivals at 0.5, 1 and 2 times the
    one-at-a-time service rate; each load served one at a time, in lockstep
    batches and in multi-rate batches (cheaper requests take up to rate_ratio
    times as many steps per chunk).  The batches admit a request only while
    the running set's initial loads stay within max_particles (the two-cloud
    run's 16.8M particles already fill the GPU), in arrival order, or within
    lone_particles when no other request waits behind it (at light load a
    request that finds the GPU busy then waits instead of slowing a large
    one down).  Request latency p50/p99 and throughput for every mode at
    every load."""
    from inputs import serving_requests
    from paper_2106_12485_amd import serve
    budget = int(budget_gb * 2 ** 30)
    base = serving_requests(n_requests=nreq)
    reqs0 = [(0.0, w, w.steps) for _, w in base]

    def pushes(res):
        return sum(float(r["diag"]["n_particles"].sum()) * n
                   for r, (_, w, n) in zip(res["results"], reqs0))

    def summary(res, reqs):
        rs = res["results"]
        ok = all(r["status"] == 0 for r in rs)
        span = max(r["done_s"] for r in rs) - min(a for a, _, _ in reqs)
        lat = np.array([r["latency_s"] for r in rs]) * 1e3
        sm = res["step_ms"]
        return dict(ok=ok, makespan_s=round(span, 4), requests_per_s=round(len(rs) / span, 3),
                    pushes_per_s=pushes(res) / span,
                    request_latency_ms=dict(p50=round(float(np.percentile(lat, 50)), 3),
                                            p99=round(float(np.percentile(lat, 99)), 3)),
                    chunk_step_ms=dict(p50=round(float(np.percentile(sm, 50)), 4),
                                       p99=round(float(np.percentile(sm, 99)), 4),
                                       n=int(len(sm))))

    def modes(reqs):
        return dict(
            one_at_a_time=summary(serve(reqs, budget, batched=False, chunk_steps=chunk), reqs),
            batched_lockstep=summary(serve(reqs, budget, batched=True, chunk_steps=chunk,
                                           max_particles=max_particles,
                                           lone_particles=lone_particles), reqs),
            batched_multirate=summary(serve(reqs, budget, batched=True, chunk_steps=chunk,
                                            rate_ratio=rate_ratio, max_particles=max_particles,
                                            lone_particles=lone_particles), reqs))

    serve(reqs0[:4], budget, batched=True, chunk_steps=chunk)  # warm-up
    t0 = modes(reqs0)
    progress("serving: all requests at t = 0 done")
    rate = t0["one_at_a_time"]["requests_per_s"]
    out = dict(workload="serving stream: %d periodic plasmas, grids 64..512^2, ppc 4/16/64, "
                        "200 steps each, HBM budget %.0f GB" % (nreq, budget_gb),
               chunk_steps=chunk, rate_ratio=rate_ratio, max_particles=max_particles,
               lone_particles=lone_particles,
               one_at_a_time_rate_per_s=rate,
               all_at_t0=t0)
    rng = np.random.default_rng(0x5EED0003)
    for load in (0.5, 1.0, 2.0):
        arr = np.cumsum(rng.exponential(1.0 / (load * rate), len(reqs0)))
        arr -= arr[0]
        reqsp = [(float(a), w, n) for a, (_, w, n) in zip(arr, reqs0)]
        out["poisson_%gx" % load] = dict(rate_per_s=round(load * rate, 3), **modes(reqsp))
        progress("serving: Poisson arrivals at %g x done" % load)
    return out


def oracle_for(w):
    """The FP64 oracle loaded with workload w (its own loader and laser)."""
    from oracle import OracleSim, Species
    o = OracleSim(w.nx, w.ny, w.lx, w.ly, w.dt, window=w.moving_window,
                  filter_passes=w.filter_passes, filter_compensate=w.filter_compensate,
                  seed=w.seed)
    for s in w.species:
        o.add_species(Species(s.qm, s.density, s.x_lo, s.x_hi, s.ppc, s.uth, s.ufl))
    if w.laser is not None:
        L = w.laser
        o.add_laser(L.a0, L.omega0, L.W0, L.fwhm, L.x_center, L.focus, L.axis, L.pol)
    return o


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)


def cpu_coverage():
    """The oracle over the measurement plan's CPU coverage: particle pushes per
    second (particles at each step summed over the steps, / wall time)."""
    from inputs import WORKLOADS
    plan = (("thermal_64x64", None, 1), ("lwfa_2000x256", None, 1),
            ("clouds_1024x1024", 20, 1), ("clouds_1024x1024", 20, host_threads()),
            ("lwfa_8000x512", 64, host_threads()))
    rows = []
    for name, nsteps, threads in plan:
        w = WORKLOADS[name]()
        o = oracle_for(w)
        o.set_threads(threads)
        k = nsteps or w.steps
        pushes = 0.0
        t0 = time.perf_counter()
        for i in range(k):
            pushes += sum(o.count(j) for j in range(len(w.species)))
            o.step(1)
            if (i + 1) % 20 == 0:
                progress("oracle %s, %d thread(s): step %d of %d" % (name, threads, i + 1, k))
        dt = time.perf_counter() - t0
        rows.append(dict(workload=name, steps=k, threads=threads, seconds=round(dt, 2),
                         pushes=int(pushes), pushes_per_s=pushes / dt))
        print(json.dumps(rows[-1]), flush=True)
        del o
    return rows


def cpu_baseline(w, nsteps):
    """Time the FP64 oracle (single-threaded C) on the same workload: its own
    load, then nsteps full steps."""
    o = oracle_for(w)
    n = sum(o.count(k) for k in range(len(w.species)))
    t0 = time.perf_counter()
    o.step(nsteps)
    dt = time.perf_counter() - t0
    out = dict(value=n * nsteps / dt, unit="particle pushes/s", cores=1, kind="oracle",
               sample="%d full steps of %s from its initial load (%d particles), FP64, "
                      "one thread" % (nsteps, w.name, n),
               seconds=round(dt, 3))
    # the same oracle with the paper's parallel-for particle loop on the host cores
    threads = host_threads()
    o.set_threads(threads)
    t0 = time.perf_counter()
    o.step(nsteps)
    dtp = time.perf_counter() - t0
    out["parallel_for"] = dict(value=n * nsteps / dtp, cores=threads,
                               sample="the next %d steps, particle loop split over %d threads "
                                      "with private current copies" % (nsteps, threads),
                               seconds=round(dtp, 3))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from inputs import WORKLOADS
    from paper_2106_12485_amd import Simulation

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.serve_only:
        print(json.dumps(serving_leg(args.serve_requests, args.budget_gb)))
        return
    if args.cpu_coverage:
        print(json.dumps(dict(cpu_coverage=cpu_coverage(), cores=host_threads())))
        return
    w = WORKLOADS[args.workload]()
    warm_steps = 0
    if args.clock_warmup_s > 0 and not args.profile_only:
        warm_steps = clock_warmup(w, args.fp64, args.deposit, args.clock_warmup_s)
        progress("clock warm-up done (%d steps of a throwaway copy)" % warm_steps)
    sim = Simulation(w, fp64=args.fp64, deposit=args.deposit)
    nparts = sum(sim.count(k) for k in range(len(w.species)))
    stream = sim.stream

    if args.profile_only and args.direct:
        sim.timing(True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    # timed region: K steps replayed from the captured step graph
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if args.profile_only:
        print(json.dumps(dict(steps=args.steps, ms_per_step=(t1 - t0) * 1e3 / args.steps)))
        return
    n_end = sum(sim.count(k) for k in range(len(w.species)))
    status = sim.status()
    elapsed = t1 - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = nparts * args.steps / elapsed
    ncell = w.nx * w.ny

    def kernel_pass(nsteps):
        """Per-kernel split over nsteps direct launches, HIP events recorded
        on the stream the kernels run on; the push's roofline over them."""
        sim.timing(True)
        sim.step(nsteps)
        tk_ = sim.timing_read()
        sim.timing(False)
        ms_push, n_push = tk_["push_deposit"]
        avg_s = ms_push / max(n_push, 1) * 1e-3
        npart = sum(sim.count(k) for k in range(len(w.species)))
        alg = npart * BYTES_PER_PARTICLE[args.fp64] + ncell * BYTES_PER_CELL[args.fp64]
        return tk_, avg_s, alg, alg / avg_s / 1e9

    tk, avg_push_s, alg_bytes, achieved = kernel_pass(args.steps)

    # per-step latency distribution (events around each replayed step)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for k in range(args.steps):
        starts[k].record(stream)
        sim.step(1)
        ends[k].record(stream)
    torch.cuda.synchronize()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])

    progress("timed steps done")
    line = dict(
        metric=METRIC, value=value, unit="particle pushes/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64" if args.fp64 else "f32", data="synthetic",
        config=dict(workload=w.name, cells="%dx%d" % (w.nx, w.ny), particles=int(nparts),
                    species=len(w.species), ppc_per_species=w.species[0].ppc[0] *
                    w.species[0].ppc[1], dt=w.dt, filter_passes=w.filter_passes,
                    moving_window=w.moving_window, deposit=args.deposit),
        clock_warmup=dict(seconds=args.clock_warmup_s if warm_steps else 0.0, steps=warm_steps,
                          what="untimed steps of a throwaway copy of the workload before the "
                               "measured run (GPU clocks out of their idle state)"),
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4),
                      traffic=(None if args.workload != "clouds_1024x1024" or args.fp64
                               or args.deposit != "reduction" else measured_traffic()),
                      kernel="k_push_deposit", avg_launch_ms=round(avg_push_s * 1e3, 4),
                      alg_bytes_per_launch=int(alg_bytes),
                      pushes_per_s_kernel=nparts / avg_push_s),
        kernel_ms_per_step={k: round(v[0] / max(v[1], 1), 4) for k, v in tk.items() if v[1]},
        step_latency_ms=dict(p50=round(float(np.percentile(lat, 50)), 4),
                             p99=round(float(np.percentile(lat, 99)), 4)),
        particles_end=int(n_end), status=int(status),
    )
    # a second window later in the run: for the two clouds, steps 500-600,
    # when the clouds have crossed and the tiles' loads are no longer uniform
    done = args.warmup + 3 * args.steps
    if args.phase_step > 0 and args.phase_step >= done and w.steps >= args.phase_step + 100:
        sim.step(args.phase_step - done)
        tp, avg_p, alg_p, ach_p = kernel_pass(100)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(100)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_p = e0.elapsed_time(e1) / 100
        nph = sum(sim.count(k) for k in range(len(w.species)))
        line["phase"] = dict(
            steps="%d-%d" % (args.phase_step + 100, args.phase_step + 200),
            kernel_steps="%d-%d" % (args.phase_step, args.phase_step + 100),
            ms_per_step=round(ms_p, 4), pushes_per_s=nph / (ms_p * 1e-3),
            roofline=dict(bound="hbm", achieved=round(ach_p, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(ach_p / HBM_PEAK_GBS, 4), traffic=None,
                          kernel="k_push_deposit", avg_launch_ms=round(avg_p * 1e3, 4),
                          alg_bytes_per_launch=int(alg_p)),
            kernel_ms_per_step={k: round(v[0] / max(v[1], 1), 4) for k, v in tp.items() if v[1]},
            status=int(sim.status()))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    progress("step windows done")
    cp = copy_peak_gbs()
    line["roofline"]["copy_peak"] = round(cp, 1)
    line["roofline"]["frac_of_copy_peak"] = round(achieved / cp, 4)
    if "phase" in line:
        line["phase"]["roofline"]["frac_of_copy_peak"] = round(line["phase"]["roofline"]["achieved"] / cp, 4)
    if args.serve_requests > 0:
        sv = serving_leg(args.serve_requests, args.budget_gb)
        line["serving"] = sv
        p1 = sv["poisson_1x"]
        line["latency_ms"] = dict(
            p50=p1["batched_lockstep"]["request_latency_ms"]["p50"],
            p99=p1["batched_lockstep"]["request_latency_ms"]["p99"],
            what="request latency (completion - arrival) of the serving stream, Poisson "
                 "arrivals at the one-at-a-time service rate, continuous batching in "
                 "lockstep chunks",
            one_at_a_time=p1["one_at_a_time"]["request_latency_ms"],
            batched_multirate=p1["batched_multirate"]["request_latency_ms"])
    if args.cpu_steps > 0:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
