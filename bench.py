#!/usr/bin/env python3
"""Benchmark of the RBE Fourier-space step on one MI355X.

One step = the whole Fourier-space hot path on one batch: cell update
(rbe_rescale_box: V, sampler tables, S), batch draw (rbe_sample_k), structure
factors, their fixed-order reduction, virial tensor and energy, and forces
(rbe_forces_pressure).  Inputs are resident in HBM before the timed region.

Beside it (default workload): ns/day of the full NPT step of the 30k-charge
rigid water (Fourier part, real-space pairs, Langevin integrator with the
rigid-molecule constraints), and a served mixed-size stream of NPT systems
(p50/p99 step latency, aggregate (N*P)/s, fused vs one system at a time).

Prints ONE JSON line (metric, value, ..., roofline, cpu_baseline, ns_per_day,
served); progress notes go to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RBE k-space (N·P)/s and ns/day, 30k-charge water NPT; served p50/p99 step ms"

# MI355X: 256 CUs at 2.4 GHz.  FP32 vector peak 157.3 TFLOP/s = 128 FMA lanes
# per CU per clock; v_sin_f32 / v_cos_f32 issue at a quarter of that, 32 per CU
# per clock -> 256 * 2.4e9 * 32 = 1.966e13 transcendental ops/s.
TRANS_PEAK = 256 * 2.4e9 * 32
# sines and cosines the method needs per (particle, frequency) pair: the
# structure factor takes cos and sin of k.r (real and imaginary part of rho);
# the force takes Im(exp(-i k.r) rho) = |rho| sin(arg rho - k.r), one sine
TRANS_PER_PAIR = {"sfac": 2, "force": 1, "step": 3}
TRANS_PER_PAIR_STEP = TRANS_PER_PAIR["sfac"] + TRANS_PER_PAIR["force"]
PER_UNIT = {"sfac": "2 transcendentals (cos, sin of k.r) per (particle, frequency) pair",
            "force": "1 transcendental (sin of arg rho - k.r) per (particle, frequency) pair",
            "step": "3 transcendentals per (particle, frequency) pair: cos, sin of k.r for rho "
                    "and sin of arg rho - k.r for the force"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="water_30k")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--p", type=int, default=None, help="override the batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--large-steps", type=int, default=40,
                    help="timed steps of the 10^6-charge, P = 2000 Fourier step (0: skip)")
    ap.add_argument("--md-steps", type=int, default=300,
                    help="timed full NPT steps for ns/day (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=120,
                    help="requests of the served stream (0: skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--md-variants", type=int, default=1,
                    help="also time the full step with cell lists and with FP32 pairs (0: skip)")
    ap.add_argument("--skin", type=float, default=1.0,
                    help="real-space neighbour-list skin (A) of the full NPT step and the "
                         "served stream (0: cell lists every step)")
    ap.add_argument("--slab-steps", type=int, default=1000,
                    help="timed Fourier steps of the membrane-shaped slab (0: skip)")
    ap.add_argument("--no-fixed-cell", action="store_true",
                    help="skip the fixed-cell sub-record (its launches share the headline "
                         "kernels' names in a profiler's per-kernel averages)")
    ap.add_argument("--issue-rates", action="store_true",
                    help="only measure the device's sine / FMA issue rates and exit")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MB",
                    help="only run a plain device copy of MB megabytes 10 times (for scaling "
                         "the HBM byte counters of a profiler run) and exit")
    return ap.parse_args()


def copy_calibration(mb):
    import torch
    n = int(mb * 1e6) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 10}))


def profiled_traffic(kernel, workload):
    """HBM bytes per dispatch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2110_14362_amd", "csrc", "rbe_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if not line.startswith("traffic: "):
                continue
            kv = dict(tok.split("=", 1) for tok in line.split()[1:])
            if (kv.get("kernel") == kernel and kv.get("workload") == workload
                    and kv.get("source_sha256") == sha):
                return int(kv["read_bytes"]) + int(kv["write_bytes"])
    return None


def npt_box(box, i):
    """The cell of step i as an NPT run moves it: every side scaled by
    1 + 3e-5 sin(i), about the per-step change of the 30k-charge water cell
    at 1 fs, so every step has a new cell (new volume, sampler tables and
    normaliser), as under the barostat."""
    f = 1.0 + 3e-5 * math.sin(float(i))
    return [b * f for b in box]


def make_step(ctx, box, x, y, z, fx, fy, fz, vir, en, fixed_cell=False):
    def step(i):
        ctx.rescale_box(box if fixed_cell else npt_box(box, i))
        ctx.sample_k(i)
        ctx.forces_pressure(x, y, z, fx, fy, fz, accumulate=False, virial6=vir, energy=en)
    return step


def time_steps(step, K, W, torch):
    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        step(i)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(sysd, seconds, first_step):
    """Full oracle steps (tables, draw, rho, virial, forces) for about
    `seconds`, BLAS limited to one thread; returns (steps, elapsed)."""
    from threadpoolctl import threadpool_limits
    from oracle import rbe as orbe
    from oracle import sampler as osamp
    P = sysd["p"]
    reps, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=1):
        while True:
            box = npt_box(sysd["box"], first_step + reps)
            m = osamp.sample_k(sysd["alpha"], box, P, seed=1, system_id=0, step=first_step + reps)
            S = osamp.box_tables(sysd["alpha"], box)["S"]
            orbe.rbe_kspace(sysd["pos"], sysd["q"], box, sysd["alpha"], m, S,
                            coulomb=sysd["coulomb"])
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return reps, el


def _oracle_worker(args):
    sysd, seconds, first = args
    return _oracle_steps(sysd, seconds, first)


def cpu_baseline(sysd, seconds):
    """The FP64 oracle, as it stands, timed on this host's cores: one process
    with BLAS on one thread, and one such process per core (independent steps
    in parallel: the throughput of all cores)."""
    import multiprocessing as mp
    N, P = len(sysd["q"]), sysd["p"]
    reps, el = _oracle_steps(sysd, seconds, 0)
    one = N * P * reps / el
    # the host's share of cores (at most 16 worker processes)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, [(sysd, seconds, 100000 * (w + 1)) for w in range(cores)])
        wall = time.perf_counter() - t0
    all_steps = sum(r[0] for r in res)
    return {"value": one, "unit": "(N*P)/s", "cores": 1, "kind": "oracle",
            "sample": "%d full steps of %s (N=%d, P=%d) under a changing cell: tables, draw, "
                      "rho, virial, forces in FP64 numpy, BLAS limited to 1 thread"
                      % (reps, sysd["config"], N, P),
            "seconds": el, "cpu_model": cpu_model(),
            "all_cores": {"value": N * P * all_steps / wall, "unit": "(N*P)/s", "cores": cores,
                          "steps": all_steps, "seconds": wall,
                          "how": "one oracle process per core, each running its own steps "
                                 "(BLAS on one thread each)"}}


def note(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def large_roofline(steps, precision, torch):
    """The Fourier step where the GPU is saturated: 10^6-charge water (333,333
    molecules, L = 215.24 A, g = 0.3/A), P = 2000; per-kernel HIP-event times."""
    from paper_2110_14362_amd import workloads
    from paper_2110_14362_amd.rbe import RBE
    dev = torch.device("cuda:0")
    s = workloads.make("water_1m")
    P = 2000
    N = len(s["q"])
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    x, y, z, q = t(s["pos"][:, 0]), t(s["pos"][:, 1]), t(s["pos"][:, 2]), t(s["q"])
    f = [torch.zeros(N, dtype=torch.float64, device=dev) for _ in range(3)]
    vir = torch.zeros(6, dtype=torch.float64, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    box = [float(b) for b in s["box"]]
    ctx = RBE(q, box, P, s["alpha"], coulomb=s["coulomb"], precision=precision, box_mode="iso",
              seed=2110143620, system_id=0)
    step = make_step(ctx, box, x, y, z, *f, vir, en)       # the cell changes every step
    el = time_steps(step, steps, 5, torch)
    ctx.timing_enable(steps)
    time_steps(step, steps, 0, torch)
    kt = ctx.timing_read()
    ctx.timing_enable(0)
    ctx.check()
    plan = ctx.plan()
    ctx.close()
    kern = {k: (v[0] / v[1] * 1e3) if v[1] else None for k, v in kt.items()}
    out = {"workload": "water_1m: N = %d, P = %d, %s" % (N, P, precision),
           "ms_per_step": el / steps * 1e3, "value": N * P / (el / steps), "unit": "(N*P)/s",
           "kernels_us": kern}
    for k in ("sfac", "force"):
        if kern.get(k):
            a = TRANS_PER_PAIR[k] * N * P / (kern[k] * 1e-6)
            out["roofline_" + k] = {"bound": "alu", "achieved": a / 1e12, "peak": TRANS_PEAK / 1e12,
                                    "unit": "Ttrans/s", "frac": a / TRANS_PEAK}
    out["plan"] = plan
    return out


def md_ns_per_day(steps, precision, torch, skin=0.0, real_precision="fp64"):
    """Full NPT step of the 30k-charge rigid water (10,000 molecules at 1 g/cm^3,
    L = 66.88 A, g = 0.3/A, r_c = 10 A, P = 100, 1 fs, 300 K, 1 atm): every
    kernel of the step, one system, per-system launches; skin > 0: real-space
    neighbour lists (rebuilds counted)."""
    from paper_2110_14362_amd import workloads
    from paper_2110_14362_amd.rbe import Batch, system_desc
    c = workloads.CONFIGS["water_30k"]
    s = workloads.rigid_water(c["n_mol"], seed=c["seed"])
    g, rc = c["g"], c["rc"]
    md = workloads.npt_real(s["box"], rc=rc)
    md["rigid"] = s["rigid"]
    if skin > 0.0:
        md["skin"] = skin
    n = len(s["q"])
    desc = system_desc(n, c["p"], g * g, workloads.COULOMB_REAL, rc, md, ntypes=3, seed=1,
                       system_id=1)
    b = Batch(1 << 32, max_systems=1, precision=precision, real_precision=real_precision)
    slot = b.admit(desc, s["pos"], s["q"], s["mass"], s["box"], types=s["types"], lj=s["lj"])
    for _ in range(20):
        b.step(fused=False)
    b.sync()
    ev0, bu0 = b.list_stats(slot)
    t0 = time.perf_counter()
    for _ in range(steps):
        b.step(fused=False)
    b.sync()
    el = time.perf_counter() - t0
    b.check(slot)
    ev1, bu1 = b.list_stats(slot)
    st = b.read(slot)
    b.close()
    t_step = el / steps
    return {"value": md["dt"] * 1e-6 * 86400.0 / t_step, "unit": "ns/day",
            "ms_per_step": t_step * 1e3, "steps": steps, "dt_fs": md["dt"],
            "workload": "rigid 3-site water, %d molecules, N = %d, box %.2f A, g = %.2f/A, "
                        "r_c = %.0f A, P = %d, NPT 300 K / 1 atm" % (c["n_mol"], n, s["box"][0],
                                                                   g, rc, c["p"]),
            "step": "integrator first half | Fourier part (%s) | real-space pairs (%s, %s) | "
                    "integrator second half" % (precision, real_precision.upper(),
                                                "neighbour lists, skin %.1f A" % skin
                                                if skin > 0 else "cell lists"),
            "list_builds_per_step": (bu1 - bu0) / max(ev1 - ev0, 1),
            "final_box_A": float(st["box"][0])}


def _serve_legs(b, reqs, fourier_only, tag):
    """Serial capacity, then Poisson arrivals at 0.8 of it served one system at
    a time and with continuous batching, then everything at once (fused)."""
    from paper_2110_14362_amd import serve
    nreq = len(reqs)
    ser = serve.serve_serial(b, reqs, fourier_only=fourier_only)
    note("served %s: serial %.2f s" % (tag, ser["wall_s"]))
    rate = 0.8 * nreq / ser["wall_s"]
    arrivals = serve.poisson_arrivals(nreq, rate)
    for r, t in zip(reqs, arrivals):
        r.arrival, r.lat, r.done = float(t), [], 0
    fifo = serve.serve(b, reqs, fused=False, max_active=1, fourier_only=fourier_only)
    note("served %s: one at a time, Poisson %.2f s" % (tag, fifo["wall_s"]))
    for r, t in zip(reqs, arrivals):
        r.arrival, r.lat, r.done = float(t), [], 0
    fused = serve.serve(b, reqs, fused=True, fourier_only=fourier_only)
    note("served %s: fused Poisson %.2f s" % (tag, fused["wall_s"]))
    for r in reqs:
        r.arrival, r.lat, r.done = 0.0, [], 0
    b.timing_enable(4 * reqs[0].steps)
    sat = serve.serve(b, reqs, fused=True, fourier_only=fourier_only)
    kt = b.timing_read()
    b.timing_enable(0)
    note("served %s: fused saturated %.2f s" % (tag, sat["wall_s"]))
    fourier = {}
    for k in ("sfac", "force"):
        if kt[k] > 0:
            a = TRANS_PER_PAIR[k] * kt["np"] / (kt[k] * 1e-3)
            fourier["roofline_" + k] = {"bound": "alu", "achieved": a / 1e12,
                                        "peak": TRANS_PEAK / 1e12, "unit": "Ttrans/s",
                                        "frac": a / TRANS_PEAK}
    fourier["device_ms_per_step"] = {k: kt[k] / max(kt["steps"], 1) for k in b.BATCH_KINDS}
    fourier["timed_steps"] = kt["steps"]
    keep = ("wall_s", "np_per_s", "p50_ms", "p99_ms")
    return {"steps_per_request": reqs[0].steps, "arrival_rate_per_s": rate,
            "serial_capacity": {k: ser[k] for k in keep},
            "one_at_a_time_poisson": {k: fifo[k] for k in keep},
            "fused_poisson": {k: fused[k] for k in keep + ("max_active", "ticks")},
            "fused_saturated": {k: sat[k] for k in keep + ("max_active", "ticks")},
            "throughput_gain_saturated": sat["np_per_s"] / ser["np_per_s"],
            "throughput_gain_poisson": fused["np_per_s"] / fifo["np_per_s"],
            "saturated_kernels": fourier}


def served_stream(nreq, budget_gib, precision, skin=0.0, fourier_steps=400):
    """Served mixed-size stream: requests of N log-uniform in [1e3, 2e5] (half
    ions, half rigid water), cubic or 1:1:1.25 cells at 0.100284 charges/A^3,
    P = 100, real-space neighbour lists with up to `skin` (as the box allows).
    Two streams of the same systems: 20 full NPT steps per request, and
    `fourier_steps` Fourier-space steps per request (the k-space step alone,
    rbe_batch_step_fourier).  Each: one system at a time back to back (the
    serial capacity), Poisson arrivals at 0.8 of it served one at a time and
    with continuous batching (fused launches), all requests at once (fused)."""
    from paper_2110_14362_amd import serve
    from paper_2110_14362_amd.rbe import Batch
    budget = int(budget_gib * (1 << 30))
    b = Batch(budget, max_systems=1024, precision=precision)
    warm = serve.make_requests(3, seed=77, kinds=("ions", "water"), nmin=2000, nmax=20000,
                               steps=3, skin=skin)
    serve.serve_serial(b, warm)
    reqs = serve.make_requests(nreq, kinds=("ions", "water"), skin=skin)
    npt = _serve_legs(b, reqs, False, "NPT")
    reqs_f = serve.make_requests(nreq, kinds=("ions", "water"), skin=skin, steps=fourier_steps)
    four = _serve_legs(b, reqs_f, True, "Fourier")
    b.close()
    return {"requests": nreq, "mean_n": float(np.mean([r.n for r in reqs])), "budget_bytes": budget,
            "npt_step": npt, "fourier_step": four,
            "note": "latency = time between a request's consecutive step completions, the "
                    "first from its arrival (queueing included); (N*P)/s counts the "
                    "Fourier-space pairs of all steps over the wall time, admission included"}


def issue_rates():
    """The device's own issue rates behind the peaks (rbe_measure_issue_rates)."""
    from paper_2110_14362_amd.rbe import measure_issue_rates
    r = measure_issue_rates()
    r["sin32_frac_of_peak_used"] = r["sin32"] / TRANS_PEAK
    return r


def slab_step(steps, precision, torch):
    """The membrane-shaped slab (80 x 80 x 100 A, two sheets of 1,024
    zwitterion dipoles, 3-site water in |z| > 25 A, 36,187 charges, g = 0.3/A,
    P = 200), semi-isotropic: every step scales lx = ly and lz by different
    small factors (a new cell, tables and normaliser per step)."""
    from paper_2110_14362_amd import workloads
    from paper_2110_14362_amd.rbe import RBE
    dev = torch.device("cuda:0")
    s = workloads.make("slab_36k")
    N, P = len(s["q"]), s["p"]
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    x, y, z, q = t(s["pos"][:, 0]), t(s["pos"][:, 1]), t(s["pos"][:, 2]), t(s["q"])
    f = [torch.zeros(N, dtype=torch.float64, device=dev) for _ in range(3)]
    vir = torch.zeros(6, dtype=torch.float64, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    box = [float(b) for b in s["box"]]
    ctx = RBE(q, box, P, s["alpha"], coulomb=s["coulomb"], precision=precision,
              box_mode="semiiso", seed=2110143620, system_id=3)

    def step(i):
        fa = 1.0 + 3e-5 * math.sin(float(i))
        fz = 1.0 - 2e-5 * math.cos(float(i))
        ctx.rescale_box([box[0] * fa, box[1] * fa, box[2] * fz])
        ctx.sample_k(i)
        ctx.forces_pressure(x, y, z, *f, accumulate=False, virial6=vir, energy=en)
    el = time_steps(step, steps, 50, torch)
    ctx.timing_enable(steps)
    time_steps(step, steps, 0, torch)
    kt = ctx.timing_read()
    ctx.timing_enable(0)
    ctx.check()
    plan = ctx.plan()
    ctx.close()
    kern = {k: (v[0] / v[1] * 1e3) if v[1] else None for k, v in kt.items()}
    out = {"workload": "slab_36k: %s, N = %d, P = %d, semi-isotropic, %s"
                       % (s["name"], N, P, precision),
           "ms_per_step": el / steps * 1e3, "value": N * P / (el / steps), "unit": "(N*P)/s",
           "steps": steps, "kernels_us": kern, "plan": plan}
    for k in ("sfac", "force"):
        if kern.get(k):
            a = TRANS_PER_PAIR[k] * N * P / (kern[k] * 1e-6)
            out["roofline_" + k] = {"bound": "alu", "achieved": a / 1e12, "peak": TRANS_PEAK / 1e12,
                                    "unit": "Ttrans/s", "frac": a / TRANS_PEAK}
    return out


def main():
    args = parse()
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.issue_rates:
        print(json.dumps(issue_rates()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (--gpus 1); sharding the "
              "Fourier-space step over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2110_14362_amd import workloads
    from paper_2110_14362_amd.rbe import RBE

    dev = torch.device("cuda:0")
    s = workloads.make(args.workload)
    if args.p:
        s["p"] = args.p
    N, P = len(s["q"]), s["p"]
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    x, y, z = t(s["pos"][:, 0]), t(s["pos"][:, 1]), t(s["pos"][:, 2])
    q = t(s["q"])
    fx, fy, fz = (torch.zeros(N, dtype=torch.float64, device=dev) for _ in range(3))
    vir = torch.zeros(6, dtype=torch.float64, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    box = [float(b) for b in s["box"]]
    mode = "semiiso" if args.workload.startswith("slab") else "iso"

    results = {}
    for prec in ([args.precision] + [p for p in ("fp32", "fp64") if p != args.precision]):
        ctx = RBE(q, box, P, s["alpha"], coulomb=s["coulomb"], precision=prec, box_mode=mode,
                  seed=2110143620, system_id=0)
        step = make_step(ctx, box, x, y, z, fx, fy, fz, vir, en)
        K = args.steps if prec == args.precision else max(1, args.steps // 4)
        el = time_steps(step, K, args.warmup, torch)
        # per-kernel device time, HIP events on the library's stream, same steps again
        ctx.timing_enable(K)
        time_steps(step, K, 0, torch)
        kt = ctx.timing_read()
        ctx.timing_enable(0)
        ctx.check()
        results[prec] = dict(seconds=el, steps=K, kernels=kt, plan=ctx.plan())
        if prec == args.precision and not args.no_fixed_cell:
            # the same steps as one launch each (rbe_set_fused), where the plan
            # allows it: a sub-record (the two-launch form is the default)
            ctx.set_fused(True)
            if ctx.plan()["fused"]:
                el1 = time_steps(step, K, args.warmup, torch)
                ctx.timing_enable(K)
                time_steps(step, K, 0, torch)
                kt1 = ctx.timing_read()
                ctx.timing_enable(0)
                ctx.check()
                results["single_launch"] = dict(seconds=el1, steps=K, kernels=kt1)
            ctx.set_fused(False)
            # the same step at a fixed cell (the batch drawn ahead by the
            # previous step is then used): a sub-record, not the headline
            fstep = make_step(ctx, box, x, y, z, fx, fy, fz, vir, en, fixed_cell=True)
            elf = time_steps(fstep, K, args.warmup, torch)
            results["fixed_cell"] = dict(seconds=elf, steps=K)
        ctx.close()

    main_r = results[args.precision]
    ms = main_r["seconds"] / main_r["steps"] * 1e3
    value = N * P / (ms * 1e-3)
    kern = {k: {"avg_us": (v[0] / v[1] * 1e3) if v[1] else None, "launches": v[1]}
            for k, v in main_r["kernels"].items()}
    dom = max(("sfac", "force", "step"), key=lambda k: kern[k]["avg_us"] or 0.0)
    t_dom = kern[dom]["avg_us"] * 1e-6
    achieved = TRANS_PER_PAIR[dom] * N * P / t_dom
    step_dev = sum((v["avg_us"] or 0.0) for v in kern.values()) * 1e-6
    plan = main_r["plan"]
    f64 = args.precision == "fp64"
    tf = "true" if f64 else "false"
    kname = {"sfac": "k_sfac<%s,%d,false>" % (tf, 1 if f64 else plan["R"]),
             "force": "k_force<%s,%d,%d>" % (tf, 1 if f64 else 2, plan["k2reduce"]),
             "step": "k_step<%s,%d,false>" % (tf, 1 if f64 else plan["R"])}[dom]
    roof = {"bound": "alu", "kernel": kname,
            "achieved": achieved / 1e12, "peak": TRANS_PEAK / 1e12, "unit": "Ttrans/s",
            "frac": achieved / TRANS_PEAK, "traffic": profiled_traffic(kname, args.workload + (
                "_p%d" % args.p if args.p else "")),
            "per_unit": PER_UNIT[dom] + "; %d x %d pairs per launch" % (N, P),
            "timing": "HIP events that each launch records itself (hipExtLaunchKernel) on the "
                      "library stream, over %d steps" % main_r["steps"]}
    out = {
        "metric": METRIC, "value": value, "unit": "(N*P)/s", "n_gpus": 1,
        "steps": main_r["steps"], "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": "%s: %s" % (s["config"], s["name"]), "n": N, "p": P,
                   "alpha": s["alpha"], "box": box, "precision": args.precision,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "roofline_step": {"bound": "alu",
                          "achieved": TRANS_PER_PAIR_STEP * N * P / step_dev / 1e12,
                          "peak": TRANS_PEAK / 1e12, "unit": "Ttrans/s",
                          "frac": TRANS_PER_PAIR_STEP * N * P / step_dev / TRANS_PEAK,
                          "note": "three transcendentals per pair (cos, sin for rho; one sine "
                                  "for the force) over the summed device time of all kernels "
                                  "of a step"},
        "kernels_us": kern,
        "plan": plan,
    }
    fc = results.pop("fixed_cell", None)
    if fc is not None:
        out["fixed_cell"] = {"value": N * P / (fc["seconds"] / fc["steps"]),
                             "ms_per_step": fc["seconds"] / fc["steps"] * 1e3, "steps": fc["steps"],
                             "note": "the same step with the cell left unchanged between steps "
                                     "(no table rebuild; the batch drawn ahead is used); the "
                                     "headline value changes the cell every step, as NPT does"}
    sl = results.pop("single_launch", None)
    if sl is not None:
        out["single_launch"] = {
            "value": N * P / (sl["seconds"] / sl["steps"]),
            "ms_per_step": sl["seconds"] / sl["steps"] * 1e3, "steps": sl["steps"],
            "kernels_us": {k: (v[0] / v[1] * 1e3) if v[1] else None
                           for k, v in sl["kernels"].items()},
            "note": "the same steps (changing cell) as one launch each (rbe_set_fused); "
                    "identical results; the two-launch form is the default"}
    for prec, r in results.items():
        if prec != args.precision:
            ms2 = r["seconds"] / r["steps"] * 1e3
            out[prec] = {"value": N * P / (ms2 * 1e-3), "ms_per_step": ms2, "steps": r["steps"],
                         "kernels_us": {k: (v[0] / v[1] * 1e3) if v[1] else None
                                        for k, v in r["kernels"].items()}}
    if not args.no_cpu_baseline:
        note("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
    note("issue rates")
    out["issue_rates"] = issue_rates()
    if args.workload == "water_30k" and args.slab_steps > 0:
        note("membrane-shaped slab")
        out["slab_36k"] = slab_step(args.slab_steps, args.precision, torch)
    if args.workload == "water_30k" and args.large_steps > 0:
        note("10^6-charge Fourier step")
        out["saturated_1m_p2000"] = large_roofline(args.large_steps, args.precision, torch)
    if args.workload == "water_30k" and args.md_steps > 0:
        note("full NPT step")
        out["ns_per_day"] = md_ns_per_day(args.md_steps, args.precision, torch, skin=args.skin)
        if args.md_variants:
            out["ns_per_day_variants"] = {
                "cell_lists_fp64": md_ns_per_day(args.md_steps, args.precision, torch, skin=0.0),
                "fp32_pairs": md_ns_per_day(args.md_steps, args.precision, torch, skin=args.skin,
                                            real_precision="fp32")}
    if args.workload == "water_30k" and args.serve_requests > 0:
        note("served stream")
        out["served"] = served_stream(args.serve_requests, args.serve_budget_gib, args.precision,
                                      skin=args.skin)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
