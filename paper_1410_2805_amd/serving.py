"""Trace driver of the serving form and its FIFO baseline.

``run_server`` replays a Poisson request trace against ``sr.Server``:
requests are submitted when their arrival time comes (wall clock), the
server ticks continuously (each tick advances every admitted request by one
stream-kick-stream step in one batched pass), and a request's latency runs
from its arrival to the moment its results are in host memory.

``run_fifo`` is the baseline: the same requests, one at a time in arrival
order, each stepped by plain single-box calls (sr_sks_split: the serving
maps and the split-coordinate pair loop of one box per call).  It runs the
same arithmetic as the server, so both return the same results (bitwise, at
the same tuning): the comparison is at equal accuracy.

``time_scale`` stretches the arrival times; 0 puts every arrival at t = 0,
which measures each path's saturation throughput.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import sr
from . import workloads


class BoxCache:
    """Zel'dovich initial conditions per lattice size (float64 positions,
    zero velocities, unit masses), generated once and shared by requests.
    get() gives (n, 3) arrays; soa() gives the same data as page-locked
    structure-of-arrays, host numpy views and the torch tensors behind them,
    so that uploads do not wait for the device."""

    def __init__(self, seed: int = 5):
        self.seed = seed
        self.cache = {}
        self.pinned = {}

    def get(self, ngrid: int):
        if ngrid not in self.cache:
            pos = workloads.zeldovich_pos64(ngrid, float(ngrid), self.seed * 1000 + ngrid)
            n = pos.shape[0]
            self.cache[ngrid] = (pos, np.zeros((n, 3), np.float32), np.ones(n, np.float32))
        return self.cache[ngrid]

    def soa(self, ngrid: int):
        """((x, y, z), (vx, vy, vz), m) pinned numpy arrays, and the pinned
        torch tensors [x, y, z, vx, vy, vz, m]."""
        if ngrid not in self.pinned:
            pos, vel, mass = self.get(ngrid)
            n = mass.shape[0]
            ts = [torch.empty(n, dtype=torch.float64, pin_memory=True) for _ in range(3)]
            ts += [torch.empty(n, dtype=torch.float32, pin_memory=True) for _ in range(4)]
            arrs = [x.numpy() for x in ts]
            for d in range(3):
                arrs[d][:] = pos[:, d]
                arrs[3 + d][:] = vel[:, d]
            arrs[6][:] = mass
            self.pinned[ngrid] = ((tuple(arrs[:3]), tuple(arrs[3:6]), arrs[6]), ts)
        return self.pinned[ngrid]


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def _keeps(keep_results, rid) -> bool:
    return keep_results is True or (bool(keep_results) and rid in keep_results)


def run_server(server: "sr.Server", trace, boxes: BoxCache, dt: float = 0.05,
               time_scale: float = 1.0, keep_results=False, log=None) -> dict:
    """Replays ``trace`` (workloads.Request list) against ``server``.
    keep_results: True, or a set of request ids whose results to return."""
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
            (pos, vel, mass), _ = boxes.soa(rq.ngrid)
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
            if not _keeps(keep_results, k):
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


def run_fifo(ctx: "sr.Context", trace, boxes: BoxCache, r_max: float, eps: float, poly,
             cell: float, dt: float = 0.05, time_scale: float = 1.0, keep_results=False,
             log=None) -> dict:
    """FIFO baseline: one request at a time with plain single-box calls on
    split coordinates (the context's tuning: give it the server's x
    sub-cells for bitwise equal results)."""
    dev = torch.device("cuda:0")
    n = len(trace)
    lat = []
    outs = {}
    t0 = time.perf_counter()
    last_log = t0
    for k, rq in enumerate(trace):
        arr = t0 + rq.arrival * time_scale
        wait = arr - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        _, ts = boxes.soa(rq.ngrid)
        box = sr.Box.make(float(rq.ngrid))
        x64 = [a.to(dev, non_blocking=True) for a in ts[:3]]
        c3, ox, oy, oz = sr.sr_split_from_f64(ctx, x64[0], x64[1], x64[2], box, cell)
        st = {"cell3": c3, "ox": ox, "oy": oy, "oz": oz, "m": ts[6].to(dev, non_blocking=True)}
        for d, key in enumerate(("vx", "vy", "vz")):
            st[key] = ts[3 + d].to(dev, non_blocking=True)
        acc = tuple(torch.empty_like(st["m"]) for _ in range(3))
        for _ in range(rq.steps):
            sr.sr_sks_split(ctx, st, box, cell, r_max, eps, poly, dt, out=acc)
        p64 = sr.sr_split_to_f64(ctx, c3, ox, oy, oz, box, cell)
        res = ([a.cpu().numpy() for a in p64],
               [st[key].cpu().numpy() for key in ("vx", "vy", "vz")])  # waits
        if _keeps(keep_results, rq.rid):
            outs[rq.rid] = res
        del res, x64, st, p64
        lat.append(time.perf_counter() - arr)
        if log and time.perf_counter() - last_log > 5.0:
            last_log = time.perf_counter()
            log("fifo: %d/%d done" % (k + 1, n))
    t1 = time.perf_counter()
    parts = sum(r.ngrid ** 3 * r.steps for r in trace)
    return {"latency_p50_s": _pct(lat, 50), "latency_p99_s": _pct(lat, 99),
            "latency_mean_s": float(np.mean(lat)), "makespan_s": t1 - t0,
            "requests_per_s": n / (t1 - t0), "particle_steps_per_s": parts / (t1 - t0),
            "results": outs if keep_results else None}
