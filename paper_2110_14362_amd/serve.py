"""Served stream of independent NPT systems on one GPU (continuous batching).

Requests arrive over time (Poisson arrivals); each is one system that runs a
fixed number of NPT steps with its state kept on the device.  The server
admits an arrived request as soon as a slot and the device-memory budget
allow (first come, first served), advances every admitted system by one step
per tick (one fused launch per kernel for all of them), and retires a system
when its steps are done.  Host-side scheduling only: every step of every
system runs in the library's kernels (rbe_batch_*).

Latency of a step is the time between a request's consecutive step
completions; the first is measured from its arrival, so queueing counts.
"""

import collections
import math
import time

import numpy as np

from . import workloads
from .rbe import Batch, system_desc


class Request:
    __slots__ = ("rid", "arrival", "sysd", "md", "desc", "steps", "slot", "t_last", "done",
                 "lat", "bytes", "result")

    def __init__(self, rid, arrival, sysd, md, steps):
        self.rid = rid
        self.arrival = arrival
        self.sysd = sysd
        self.md = md
        self.steps = steps
        ntypes = 0 if sysd.get("lj") is None else int(np.asarray(sysd["lj"]).shape[0])
        self.desc = system_desc(len(sysd["q"]), sysd["p"], sysd["alpha"], sysd["coulomb"],
                                sysd["rc"], md, ntypes=ntypes, seed=sysd.get("seed", rid),
                                system_id=rid)
        self.bytes = Batch.footprint(self.desc, sysd["box"])
        self.slot = None
        self.t_last = None
        self.done = 0
        self.lat = []
        self.result = None

    @property
    def n(self):
        return int(self.desc.n)

    @property
    def work(self):
        """(particle, frequency) pairs of one Fourier-space step."""
        return int(self.desc.n) * int(self.desc.p)


def make_requests(count, seed=2110143625, kinds=("ions",), nmin=1000, nmax=200000, p=100,
                  steps=20, skin=0.0, sampler="exact"):
    """The served stream's systems (arrival times are set by the caller);
    skin > 0: real-space neighbour lists with at most that skin; sampler:
    'exact' or 'mh' (the online Metropolis-Hastings chains)."""
    reqs = []
    for i in range(count):
        s = workloads.serving_request(i, seed=seed, nmin=nmin, nmax=nmax, p=p, steps=steps,
                                      kinds=kinds)
        md = workloads.npt_real(s["box"], rc=s["rc"])
        if skin > 0.0:
            md["skin"] = workloads.list_skin(s["box"], s["rc"], skin)
        if sampler != "exact":
            md["sampler"] = sampler
        if s.get("rigid"):
            md["rigid"] = s["rigid"]
        reqs.append(Request(i, 0.0, s, md, steps))
    return reqs


def poisson_arrivals(count, rate, seed=2110143626):
    """Arrival times (s) of a Poisson process of the given rate (1/s)."""
    g = np.random.default_rng(np.random.PCG64(seed))
    return np.cumsum(g.exponential(1.0 / rate, count))


def _admit(batch, r):
    s = r.sysd
    return batch.admit(r.desc, s["pos"], s["q"], s["mass"], s["box"], types=s.get("types"),
                       lj=s.get("lj"))


def serve(batch, reqs, fused=True, max_active=None, keep_results=False, check=True,
          clock=time.perf_counter, fourier_only=False):
    """Run the stream; reqs carry arrival times (s from the start).  Returns
    summary statistics; per-request latencies stay in r.lat.  max_active = 1
    with fused = False is the one-system-at-a-time server (first come, first
    served, each system's kernels launched on their own).  fourier_only: each
    step is the Fourier-space step alone (rbe_batch_step_fourier)."""
    pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
    active = {}
    t0 = clock()
    ticks = 0
    peak_active = 0
    busy = 0.0
    while pending or active:
        now = clock() - t0
        while pending and pending[0].arrival <= now and (max_active is None
                                                          or len(active) < max_active):
            r = pending[0]
            slot = _admit(batch, r)
            if slot is None:
                if not active:
                    raise RuntimeError("request %d (%d bytes) does not fit the empty batch"
                                       % (r.rid, r.bytes))
                break
            pending.popleft()
            r.slot = slot
            r.t_last = r.arrival
            active[slot] = r
        if not active:
            wait = pending[0].arrival - (clock() - t0)
            if wait > 0:
                time.sleep(wait)
            continue
        peak_active = max(peak_active, len(active))
        ts = clock()
        batch.step(fused=fused, fourier_only=fourier_only)
        batch.sync()
        t = clock()
        busy += t - ts
        t -= t0
        ticks += 1
        for slot in list(active):
            r = active[slot]
            r.lat.append(t - r.t_last)
            r.t_last = t
            r.done += 1
            if r.done == r.steps:
                if check:
                    batch.check(slot)
                if keep_results:
                    r.result = batch.read(slot)
                batch.release(slot)
                del active[slot]
    wall = clock() - t0
    return summarize(reqs, wall, ticks=ticks, max_active=peak_active, busy=busy)


def serve_serial(batch, reqs, keep_results=False, check=True, clock=time.perf_counter,
                 fourier_only=False):
    """The same requests one system at a time, each with its own per-kernel
    launches, back to back (all taken as arrived at t = 0)."""
    t0 = clock()
    for r in reqs:
        r.lat = []
        slot = _admit(batch, r)
        if slot is None:
            raise RuntimeError("request %d does not fit the empty batch" % r.rid)
        r.slot = slot
        r.t_last = clock() - t0
        for _ in range(r.steps):
            batch.step(fused=False, fourier_only=fourier_only)
            batch.sync()
            t = clock() - t0
            r.lat.append(t - r.t_last)
            r.t_last = t
        if check:
            batch.check(slot)
        if keep_results:
            r.result = batch.read(slot)
        batch.release(slot)
    wall = clock() - t0
    return summarize(reqs, wall)


def summarize(reqs, wall, **extra):
    lat = np.concatenate([np.asarray(r.lat) for r in reqs]) * 1e3
    work = sum(r.work * r.steps for r in reqs)
    out = dict(requests=len(reqs), steps=int(sum(r.steps for r in reqs)), wall_s=wall,
               np_per_s=work / wall if wall > 0 else math.nan,
               p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
               mean_n=float(np.mean([r.n for r in reqs])))
    out.update(extra)
    return out
