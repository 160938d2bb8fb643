"""Benchmark of the short-range particle-particle force on one MI355X.

One step = one sr_force call on a resident synthetic box: binning into the
chaining mesh (cell ids, histogram, scan, scatter, per-cell sort, gather),
work-item construction, the pair loop over the 27-cell stencil, the
scatter of accelerations back to the caller's order, and the FP64 momentum
reduction.  Inputs are in HBM before the timed region starts.

Prints ONE JSON line on stdout (progress goes to stderr):
  value     useful directed pair interactions per second of whole steps
  roofline  the pair-loop kernel against the FP32 vector peak, counting 30
            FLOP per evaluated (candidate) pair, its average duration taken
            from HIP events recorded on the library's stream
  cpu_baseline  the FP64 brute-force oracle on a bounded sample of targets
            of the same box, on this host's cores
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32 (256 CU x 2.4 GHz x 256 FLOP/clk)
FLOP_PER_PAIR = 30           # per evaluated pair; FMA = 2, rsqrt = 1
R_MAX, EPS = 3.0, 0.1

WORKLOADS = {
    "zeldovich128": "128^3 Zel'dovich-displaced lattice (P(k) ~ k^-2 to Nyquist, rms 0.5), "
                    "periodic L=128, r_max=3, eps=0.1, cell 3 (42^3 cells)",
    "uniform32": "32^3 uniform random, periodic L=32, r_max=3, eps=0.1, cell 3 (10^3 cells)",
    "nfw256": "256^3 clustered open share (70% NFW halos, 30% uniform), L=256, skin 3, "
              "r_max=3, eps=0.1, cell 3 (85^3 cells)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(p, poly, seconds: float):
    """Times the oracle on a seeded target sample sized for ~`seconds`."""
    import numpy as np

    from oracle import oracle as O
    rng = np.random.default_rng(2024)
    threads = O.max_threads()
    k = 64
    t_used = 0.0
    total_pairs = 0
    total_targets = 0
    while True:
        tg = np.sort(rng.choice(p.n, k, replace=False))
        t0 = time.perf_counter()
        r = O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64),
                    periodic=p.periodic, skin=p.skin, targets=tg)
        dt = time.perf_counter() - t0
        t_used += dt
        total_pairs += int(r["npair"].sum())
        total_targets += k
        log("cpu_baseline: %d targets in %.2fs" % (k, dt))
        if t_used >= seconds or k >= p.n:
            break
        k = int(min(p.n, max(k * 2, k * (seconds - t_used) / max(dt, 1e-3))))
        k = max(64, min(k, p.n))
    return {
        "value": total_pairs / t_used,
        "unit": "useful pair interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d seeded targets x all %d sources (FP64 brute force, OpenMP over targets), "
                  "%.1f s; %.3g pair evaluations/s" % (total_targets, p.n, t_used,
                                                       total_targets * p.n / t_used),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="zeldovich128", choices=sorted(WORKLOADS))
    ap.add_argument("--cell", type=float, default=3.0)
    ap.add_argument("--xsplit", type=int, default=0, help="pair-loop x sub-cells (0: library default)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 256 MiB device-to-device copy (a known-size kernel "
                         "for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1410_2805_amd import gridfit, sr, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calib_copy:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log("generating %s" % args.workload)
    p = workloads.config(args.workload)
    poly = gridfit.poly_coeffs()
    t = {k: torch.from_numpy(getattr(p, k)).to(dev) for k in "xyzm"}
    box = sr.Box.make(p.L, periodic=p.periodic, skin=p.skin)
    arena = sr.sr_scratch_bytes(box, args.cell, p.n, True)
    ctx = sr.Context(0, arena_bytes=arena)
    if args.xsplit:
        ctx.set_tuning(args.xsplit)
    xsplit = ctx.get_tuning()["xsplit"]
    out = tuple(torch.empty(p.n, dtype=torch.float32, device=dev) for _ in range(3))
    mom = torch.zeros(3, dtype=torch.float64, device=dev)

    useful, cand, _ = sr.sr_pair_stats(ctx, t["x"], t["y"], t["z"], box, args.cell, R_MAX)
    log("pairs: useful %d candidates %d (waste %.2fx)" % (useful, cand, cand / max(useful, 1)))

    def step():
        sr.sr_force(ctx, t["x"], t["y"], t["z"], t["m"], box, args.cell, R_MAX, EPS, poly,
                    out=out, momentum=mom)

    for _ in range(args.warmup):
        step()
    ctx.sync()
    ctx.timing_enable(True)
    ctx.timing_collect()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ctx.sync()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    prep_ms, force_ms, calls = ctx.timing_collect()
    ctx.timing_enable(False)
    force_avg = force_ms / max(calls, 1)
    prep_avg = prep_ms / max(calls, 1)
    log("step %.4f ms (prep %.4f ms, pair loop %.4f ms over %d calls)" % (ms_step, prep_avg,
                                                                        force_avg, calls))
    achieved = FLOP_PER_PAIR * cand / (force_avg * 1e-3) / 1e12
    value = useful / (ms_step * 1e-3)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, poly, args.cpu_seconds)

    res = {
        "metric": "short-range pair interactions/s",
        "value": value,
        "unit": "useful directed pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload],
            "name": args.workload,
            "n": p.n,
            "cell": args.cell,
            "xsplit": xsplit,
            "useful_pairs": useful,
            "candidate_pairs": cand,
            "waste": cand / max(useful, 1),
            "prep_ms": prep_avg,
            "pair_loop_ms": force_avg,
            "pair_loop_useful_per_s": useful / (force_avg * 1e-3),
            "pct_fp32_peak": 100.0 * achieved / FP32_PEAK_TFLOPS,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_force",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": None,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
