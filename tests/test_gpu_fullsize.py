"""Full-size parity of the batched and serving forms.

Batched: the 64-box workload (particle counts log-uniform in [16^3, 96^3],
half uniform, half NFW-clustered, 14.6 M particles) in one plan at the
autotuned tuning, in global and in split (cell + offset) coordinates: every
box bitwise equal to its single-box call, and min(N_b, 512) sampled targets
per box within tolerance of the FP64 oracle.

Serving: 16 requests of the serving trace (Poisson arrivals at 200/s, boxes
of 24^3..128^3 particles, 10 stream-kick-stream steps each) admitted
together into 64 slots: each result bitwise equal to the same request
stepped alone by single-box calls; full FP64 trajectories for boxes of at
most 32^3 particles; the kicks of steps 1 and 10 of every request against the
oracle on 512 sampled particles."""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1410_2805_amd import gridfit, serving
from paper_1410_2805_amd import workloads as W
from tests.parity import (accel_np, check_accel, check_accel_slack, kick_accel_ref,
                          position_slack, to_dev)

pytestmark = pytest.mark.gpu

R_MAX, EPS, CELL, DT = 3.0, 0.1, 3.0, 0.05


@pytest.fixture(scope="module")
def sr():
    from paper_1410_2805_amd import sr as S
    return S


@pytest.fixture(scope="module")
def ctx(sr):
    c = sr.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def poly():
    return gridfit.poly_coeffs()


@pytest.fixture(scope="module")
def batch64():
    specs = W.batch_specs(64, seed=4)
    return [W.make_box(s) for s in specs]


def _sample(n, k, seed):
    if n <= k:
        return np.arange(n)
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def _with_tuning(ctx, tuning, fn):
    before = ctx.get_tuning()
    ctx.set_tuning(xsplit=tuning["xsplit"], order=tuning["order"], persistent=tuning["persistent"])
    try:
        return fn()
    finally:
        ctx.set_tuning(**before)


def test_batch64_global_full_size(sr, ctx, poly, batch64):
    dev = []
    for p in batch64:
        t = to_dev(p)
        t.update({k: torch.empty(p.n, dtype=torch.float32, device="cuda:0") for k in ("ax", "ay", "az")})
        t["box"] = sr.Box.make(p.L)
        t["cell"] = CELL
        dev.append(t)
    mom = torch.zeros(3 * len(dev), dtype=torch.float64, device="cuda:0")
    plan = sr.Plan(ctx, dev, R_MAX, EPS, poly, momentum=mom)
    try:
        best, _ = plan.autotune(reps=1)
        print("autotuned", best)
        plan.launch()
        ctx.sync()
        for b, (p, t) in enumerate(zip(batch64, dev)):
            a = accel_np(t["ax"], t["ay"], t["az"])

            def single():
                r = sr.sr_force(ctx, t["x"], t["y"], t["z"], t["m"], t["box"],
                                CELL * best["cell_scale"], R_MAX, EPS, poly)
                ctx.sync()
                return accel_np(*r[:3])

            assert np.array_equal(a, _with_tuning(ctx, best, single)), "box %d" % b
            tg = _sample(p.n, 512, b)
            ref = O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64),
                          targets=tg)
            check_accel(a[tg], ref, "batch64 box %d (n=%d)" % (b, p.n))
            want = (p.m.astype(np.float64)[:, None] * a).sum(0)
            got = mom.cpu().numpy()[3 * b: 3 * b + 3]
            assert np.allclose(got, want, rtol=0, atol=1e-9 * (np.abs(a).sum() + 1))
    finally:
        plan.close()


def test_batch64_split_full_size(sr, ctx, poly, batch64):
    """The batched form in split coordinates from FP64 master positions."""
    dev = []
    for p in batch64:
        box = sr.Box.make(p.L)
        x, y, z = [torch.from_numpy(np.ascontiguousarray(c)).to("cuda:0")
                   for c in p.pos64().T]
        c3, ox, oy, oz = sr.sr_split_from_f64(ctx, x, y, z, box, CELL)
        t = {"x": ox, "y": oy, "z": oz, "cell3": c3,
             "m": torch.from_numpy(p.m).to("cuda:0"), "box": box, "cell": CELL}
        t.update({k: torch.empty(p.n, dtype=torch.float32, device="cuda:0") for k in ("ax", "ay", "az")})
        dev.append(t)
    mom = torch.zeros(3 * len(dev), dtype=torch.float64, device="cuda:0")
    plan = sr.Plan(ctx, dev, R_MAX, EPS, poly, momentum=mom)
    try:
        best, _ = plan.autotune(reps=1)
        assert best["cell_scale"] == 1.0
        plan.launch()
        ctx.sync()
        for b, (p, t) in enumerate(zip(batch64, dev)):
            a = accel_np(t["ax"], t["ay"], t["az"])

            def single():
                r = sr.sr_force_split(ctx, t["cell3"], t["x"], t["y"], t["z"], t["m"], t["box"],
                                      CELL, R_MAX, EPS, poly)
                ctx.sync()
                return accel_np(*r[:3])

            assert np.array_equal(a, _with_tuning(ctx, best, single)), "split box %d" % b
            tg = _sample(p.n, 512, 100 + b)
            ref = O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64),
                          targets=tg)
            h = p.L / np.floor(p.L / CELL)
            check_accel_slack(a[tg], ref, position_slack(ref["npair"], 1.0, h, EPS),
                              "batch64 split box %d (n=%d)" % (b, p.n))
    finally:
        plan.close()


def _trace_requests(k=16):
    trace = W.serving_trace(2000, rate=200.0, seed=5)
    by_size = sorted(trace, key=lambda r: (r.ngrid, r.rid))
    idx = np.unique(np.linspace(0, len(by_size) - 1, k).round().astype(int))
    return [by_size[i] for i in idx]


def test_serving_trace_requests_full_size(sr, ctx, poly):
    reqs = _trace_requests(16)
    assert len(reqs) == 16 and reqs[-1].ngrid == 128 and reqs[0].ngrid == 24
    boxes = serving.BoxCache(seed=5)
    # all 16 admitted at once (64 slots): they share every tick
    srv = sr.Server(ctx, 16 << 30, 64, R_MAX, EPS, poly, CELL, xsplit=2)
    try:
        mixed = {}
        ids = {}
        for rq in reqs:
            (pos, vel, mass), _ = boxes.soa(rq.ngrid)
            n = mass.shape[0]
            op = tuple(sr.pinned_empty(n, np.float64) for _ in range(3))
            ov = tuple(sr.pinned_empty(n, np.float32) for _ in range(3))
            ids[srv.submit(float(rq.ngrid), rq.steps, DT, pos, vel, mass, op, ov)] = rq.rid
            mixed[rq.rid] = (op, ov)
        got = set()
        stepped = []
        t_end = time.monotonic() + 120.0  # ticks only enqueue: bound by time
        while time.monotonic() < t_end:
            stepped.append(srv.tick())
            got.update(srv.poll())
            if got >= set(ids):
                break
            if stepped[-1] == 0:
                time.sleep(0.001)
        assert got >= set(ids), "requests did not complete"
        # admitted together: all 16 stepped on each of the first 10 ticks
        assert stepped[:10] == [16] * 10 and sum(stepped) == 160
    finally:
        srv.close()
    before = ctx.get_tuning()
    ctx.set_tuning(xsplit=2)
    try:
        for rq in reqs:
            pos, vel, mass = boxes.get(rq.ngrid)
            n = mass.shape[0]
            L = float(rq.ngrid)
            box = sr.Box.make(L)
            x64 = [torch.from_numpy(np.ascontiguousarray(pos[:, d])).to("cuda:0") for d in range(3)]
            c3, ox, oy, oz = sr.sr_split_from_f64(ctx, *x64, box, CELL)
            st = {"cell3": c3, "ox": ox, "oy": oy, "oz": oz,
                  "m": torch.from_numpy(mass).to("cuda:0")}
            for d, key in enumerate(("vx", "vy", "vz")):
                st[key] = torch.from_numpy(np.ascontiguousarray(vel[:, d])).to("cuda:0")
            acc = tuple(torch.empty(n, dtype=torch.float32, device="cuda:0") for _ in range(3))
            snaps = {}
            for s in range(1, rq.steps + 1):
                if s == rq.steps:
                    p9 = sr.sr_split_to_f64(ctx, c3, ox, oy, oz, box, CELL)
                    snaps["pos9"] = torch.stack(p9, 1).cpu().numpy()
                    snaps["vel9"] = torch.stack([st["vx"], st["vy"], st["vz"]], 1).cpu().numpy()
                sr.sr_sks_split(ctx, st, box, CELL, R_MAX, EPS, poly, DT, out=acc)
                if s in (1, rq.steps):
                    snaps["acc%d" % s] = accel_np(*acc)
            pf = torch.stack(sr.sr_split_to_f64(ctx, c3, ox, oy, oz, box, CELL), 1).cpu().numpy()
            vf = torch.stack([st["vx"], st["vy"], st["vz"]], 1).cpu().numpy()
            ctx.sync()
            op, ov = mixed[rq.rid]
            # alone (single-box calls) equals the mix, bitwise
            assert np.array_equal(np.stack(op, 1), pf), "request %d positions" % rq.rid
            assert np.array_equal(np.stack(ov, 1), vf), "request %d velocities" % rq.rid
            h = L / np.floor(L / CELL)
            tg = _sample(n, 512, rq.rid)
            # step 1 kicks with the force at the initial positions (v = 0)
            r1 = kick_accel_ref(pos, vel, mass, L, tg, R_MAX, EPS, poly, DT)
            check_accel_slack(snaps["acc1"][tg], r1, position_slack(r1["npair"], 1.0, h, EPS),
                              "request %d (ngrid %d) step 1" % (rq.rid, rq.ngrid))
            r10 = kick_accel_ref(snaps["pos9"], snaps["vel9"], mass, L, tg, R_MAX, EPS, poly, DT)
            check_accel_slack(snaps["acc%d" % rq.steps][tg], r10,
                              position_slack(r10["npair"], 1.0, h, EPS),
                              "request %d (ngrid %d) step 10" % (rq.rid, rq.ngrid))
            if rq.ngrid <= 32:
                P, V = pos.copy(), vel.astype(np.float64)
                for _ in range(rq.steps):
                    P, V, _ = O.sks(P, V, mass, L, R_MAX, EPS, poly.astype(np.float64), DT)
                d = pf - P
                d -= L * np.round(d / L)
                assert np.max(np.abs(d)) < 2e-5, "request %d trajectory" % rq.rid
                assert np.max(np.abs(vf - V)) < 2e-5 * max(1.0, np.abs(V).max())
    finally:
        ctx.set_tuning(**before)
