"""Trace driver of the serving form and its FIFO baseline.

``run_server`` replays a Poisson request trace against ``sr.Server``:
requests are submitted when their arrival time comes (wall clock), the
server ticks continuously (each tick advances every admitted request by one
stream-kick-stream step in one batched pass), and a request's latency runs
from its arrival to the moment its results are in host memory.

``run_fifo`` is the baseline: the same requests, one at a time in arrival
order, each stepped by plain single-box calls (sr_force on global float32
coordinates plus elementwise stream and kick updates).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import sr
from . import workloads


class BoxCache:
    """Zel'dovich initial conditions per lattice size (float64 positions,
    zero velocities, unit masses), generated once and shared by requests."""

    def __init__(self, seed: int = 5):
        self.seed = seed
        self.cache = {}

    def get(self, ngrid: int):
        if ngrid not in self.cache:
            pos = workloads.zeldovich_pos64(ngrid, float(ngrid), self.seed * 1000 + ngrid)
            n = pos.shape[0]
            self.cache[ngrid] = (pos, np.zeros((n, 3), np.float32), np.ones(n, np.float32))
        return self.cache[ngrid]


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def run_server(server: "sr.Server", trace, boxes: BoxCache, dt: float = 0.05,
               time_scale: float = 1.0, keep_results: bool = False, log=None) -> dict:
    """Replays ``trace`` (workloads.Request list) against ``server``."""
    n = len(trace)
    outs = {}
    arrival = {}
    done = {}
    rid_of = {}
    t0 = time.perf_counter()
    nxt = 0
    last_log = t0
    ticks = 0
    busy = 0
    while len(done) < n:
        now = time.perf_counter()
        while nxt < n and t0 + trace[nxt].arrival * time_scale <= now:
            rq = trace[nxt]
            pos, vel, mass = boxes.get(rq.ngrid)
            m = mass.shape[0]
            op = tuple(sr.pinned_empty(m, np.float64) for _ in range(3))
            ov = tuple(sr.pinned_empty(m, np.float32) for _ in range(3))
            rid = server.submit(float(rq.ngrid), rq.steps, dt, pos, vel, mass, op, ov)
            rid_of[rid] = rq.rid
            arrival[rq.rid] = t0 + rq.arrival * time_scale
            outs[rq.rid] = (op, ov)
            nxt += 1
        active = server.tick()
        ticks += 1
        busy += active > 0
        for rid in server.poll():
            k = rid_of.pop(rid)
            done[k] = time.perf_counter()
            if not keep_results:
                for a in outs[k][0] + outs[k][1]:
                    sr.pinned_release(a)
                outs.pop(k)
        if active == 0 and nxt < n and not rid_of:
            wait = t0 + trace[nxt].arrival * time_scale - time.perf_counter()
            if wait > 0:
                time.sleep(min(wait, 0.01))
        if log and time.perf_counter() - last_log > 5.0:
            last_log = time.perf_counter()
            log("serving: %d/%d done, %d submitted, %d ticks" % (len(done), n, nxt, ticks))
    t1 = time.perf_counter()
    lat = [done[k] - arrival[k] for k in done]
    parts = sum(r.ngrid ** 3 * r.steps for r in trace)
    return {"latency_p50_s": _pct(lat, 50), "latency_p99_s": _pct(lat, 99),
            "latency_mean_s": float(np.mean(lat)), "makespan_s": t1 - t0,
            "requests_per_s": n / (t1 - t0), "particle_steps_per_s": parts / (t1 - t0),
            "ticks": ticks, "results": outs if keep_results else None}


def _stream(x, v, half_dt, L):
    x.add_(v, alpha=half_dt)
    torch.remainder(x, L, out=x)
    x.masked_fill_(x >= L, 0.0)


def run_fifo(ctx: "sr.Context", trace, boxes: BoxCache, r_max: float, eps: float, poly,
             cell: float, dt: float = 0.05, time_scale: float = 1.0, log=None) -> dict:
    """FIFO baseline: one request at a time with plain single-box calls."""
    dev = torch.device("cuda:0")
    n = len(trace)
    lat = []
    t0 = time.perf_counter()
    last_log = t0
    for k, rq in enumerate(trace):
        arr = t0 + rq.arrival * time_scale
        wait = arr - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        pos, vel, mass = boxes.get(rq.ngrid)
        L = float(rq.ngrid)
        x = [torch.from_numpy(np.ascontiguousarray(pos[:, d], dtype=np.float32)).to(dev)
             for d in range(3)]
        v = [torch.from_numpy(np.ascontiguousarray(vel[:, d])).to(dev) for d in range(3)]
        m = torch.from_numpy(mass).to(dev)
        for xd in x:
            xd.masked_fill_(xd >= L, 0.0)
        box = sr.Box.make(L)
        out = tuple(torch.empty_like(m) for _ in range(3))
        for _ in range(rq.steps):
            for d in range(3):
                _stream(x[d], v[d], 0.5 * dt, L)
            a = sr.sr_force(ctx, x[0], x[1], x[2], m, box, cell, r_max, eps, poly, out=out)
            for d in range(3):
                v[d].add_(a[d], alpha=dt)
                _stream(x[d], v[d], 0.5 * dt, L)
        res = [xd.double().cpu() for xd in x] + [vd.cpu() for vd in v]  # waits
        del res
        lat.append(time.perf_counter() - arr)
        if log and time.perf_counter() - last_log > 5.0:
            last_log = time.perf_counter()
            log("fifo: %d/%d done" % (k + 1, n))
    t1 = time.perf_counter()
    parts = sum(r.ngrid ** 3 * r.steps for r in trace)
    return {"latency_p50_s": _pct(lat, 50), "latency_p99_s": _pct(lat, 99),
            "latency_mean_s": float(np.mean(lat)), "makespan_s": t1 - t0,
            "requests_per_s": n / (t1 - t0), "particle_steps_per_s": parts / (t1 - t0)}
