"""Batched form (sr_plan_*): many boxes per pass, graph replay, autotuner.

Every box of a plan must give bitwise the accelerations of sr_force on that
box alone with the same tuning, and the oracle's within tolerance."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1410_2805_amd import gridfit
from paper_1410_2805_amd import workloads as W
from tests.parity import accel_np, check_accel, to_dev

pytestmark = pytest.mark.gpu

R_MAX, EPS = 3.0, 0.1


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


def _boxes(tiny=True):
    out = []
    u = W.uniform(4096, 16.0, 1)
    out.append((u, 3.0))
    c = W.nfw_share(8000, 20.0, 2, periodic=True, halo_cap=2000)
    out.append((c, 3.0))
    o = W.nfw_share(9000, 21.0, 3, skin=3.0)
    out.append((o, 3.0))
    if tiny:  # only 3 cells per axis: invalid at a coarser cell scale
        t = W.uniform(857, 9.5, 4)
        out.append((t, 3.0))
    e = W.Particles(*(np.zeros(0, np.float32) for _ in range(4)), 12.0)
    out.append((e, 3.0))
    m = W.uniform(2197, 13.0, 5)
    m.m = np.random.default_rng(5).uniform(0.5, 2.0, m.n).astype(np.float32)
    out.append((m, 3.25))
    return out


def _plan_inputs(sr, boxes):
    dev = []
    for p, cell in boxes:
        t = to_dev(p)
        n = p.n
        t.update({k: torch.zeros(max(n, 1), dtype=torch.float32, device="cuda:0")[:n]
                  for k in ("ax", "ay", "az")})
        t["box"] = sr.Box.make(p.L, periodic=p.periodic, skin=p.skin)
        t["cell"] = cell
        dev.append(t)
    return dev


def _single(sr, ctx, p, cell, poly, tuning):
    t = to_dev(p)
    before = ctx.get_tuning()
    ctx.set_tuning(xsplit=tuning["xsplit"], order=tuning["order"],
                   persistent=tuning["persistent"])
    try:
        ax, ay, az, _ = sr.sr_force(ctx, t["x"], t["y"], t["z"], t["m"],
                                    sr.Box.make(p.L, periodic=p.periodic, skin=p.skin),
                                    cell * tuning["cell_scale"], R_MAX, EPS, poly)
        ctx.sync()
    finally:
        ctx.set_tuning(**before)
    return accel_np(ax, ay, az)


def _ref(p, poly):
    return O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64),
                   periodic=p.periodic, skin=p.skin)


@pytest.mark.parametrize("tuning", [dict(xsplit=2, order=1, persistent=0, cell_scale=1.0),
                                    dict(xsplit=1, order=0, persistent=1, cell_scale=1.0),
                                    dict(xsplit=3, order=1, persistent=1, cell_scale=1.0),
                                    dict(xsplit=2, order=0, persistent=0, cell_scale=1.25)])
def test_batch_matches_single_boxes(sr, ctx, poly, tuning):
    boxes = _boxes(tiny=tuning["cell_scale"] == 1.0)
    dev = _plan_inputs(sr, boxes)
    mom = torch.zeros(3 * len(boxes), dtype=torch.float64, device="cuda:0")
    plan = sr.Plan(ctx, dev, R_MAX, EPS, poly, momentum=mom)
    try:
        plan.set_tuning(**tuning)
        plan.run()
        ctx.sync()
        for b, ((p, cell), t) in enumerate(zip(boxes, dev)):
            a = accel_np(t["ax"], t["ay"], t["az"])
            single = _single(sr, ctx, p, cell, poly, tuning)
            assert np.array_equal(a, single), "box %d differs from its single-box call" % b
            if p.n:
                check_accel(a, _ref(p, poly), "batch box %d" % b)
            want = (p.m.astype(np.float64)[:, None] * a).sum(0) if p.n else np.zeros(3)
            got = mom.cpu().numpy()[3 * b: 3 * b + 3]
            assert np.allclose(got, want, rtol=0, atol=1e-9 * (np.abs(a).sum() + 1))
    finally:
        plan.close()


def test_invalid_tuning_and_box(sr, ctx, poly):
    boxes = _boxes()
    dev = _plan_inputs(sr, boxes)
    plan = sr.Plan(ctx, dev, R_MAX, EPS, poly)
    try:
        with pytest.raises(sr.SRError):
            plan.set_tuning(xsplit=2, order=0, persistent=0, cell_scale=2.0)  # 9.5 box: < 3 cells
        with pytest.raises(sr.SRError):
            plan.set_tuning(xsplit=9, order=0, persistent=0)
    finally:
        plan.close()
    bad = dict(dev[0])
    bad["cell"] = 2.0  # cell narrower than r_max
    with pytest.raises(sr.SRError):
        sr.Plan(ctx, [dev[1], bad], R_MAX, EPS, poly)


def test_graph_replay(sr, ctx, poly):
    """A captured pass replayed several times, with eager work and syncs in
    between, equals the eager pass bitwise each time, and follows updates of
    the input buffers."""
    boxes = _boxes()
    dev = _plan_inputs(sr, boxes)
    mom = torch.zeros(3 * len(boxes), dtype=torch.float64, device="cuda:0")
    plan = sr.Plan(ctx, dev, R_MAX, EPS, poly, momentum=mom)
    try:
        plan.run()
        ctx.sync()
        eager = [accel_np(t["ax"], t["ay"], t["az"]) for t in dev]
        eager_mom = mom.cpu().numpy().copy()
        plan.capture()
        for rep in range(3):
            for t in dev:
                for k in ("ax", "ay", "az"):
                    t[k].fill_(float("nan"))
            mom.zero_()
            junk = torch.randn(1 << 20, device="cuda:0").sum()  # eager work between replays
            torch.cuda.synchronize()
            plan.launch()
            ctx.sync()
            for b, t in enumerate(dev):
                assert np.array_equal(accel_np(t["ax"], t["ay"], t["az"]), eager[b]), (rep, b)
            assert np.array_equal(mom.cpu().numpy(), eager_mom)
            del junk
        # move box 0's particles by a whole period image: same forces expected
        p0 = boxes[0][0]
        shifted = np.mod(p0.pos64() + 4.0, p0.L).astype(np.float32)
        for d, k in enumerate("xyz"):
            dev[0][k].copy_(torch.from_numpy(shifted[:, d].copy()))
        plan.launch()
        ctx.sync()
        q = W.Particles(shifted[:, 0].copy(), shifted[:, 1].copy(), shifted[:, 2].copy(),
                        p0.m.copy(), p0.L)
        a0 = accel_np(dev[0]["ax"], dev[0]["ay"], dev[0]["az"])
        check_accel(a0, _ref(q, poly), "replay after input update")
    finally:
        plan.close()


def test_autotune_picks_a_valid_tuning(sr, ctx, poly):
    boxes = _boxes()
    dev = _plan_inputs(sr, boxes)
    plan = sr.Plan(ctx, dev, R_MAX, EPS, poly)
    try:
        best, ms = plan.autotune(reps=1)
        assert 1 <= best["xsplit"] <= 3 and best["cell_scale"] >= 1.0 and ms > 0
        assert plan.get_tuning() == best
        plan.launch()
        ctx.sync()
        for b, ((p, cell), t) in enumerate(zip(boxes, dev)):
            if p.n:
                check_accel(accel_np(t["ax"], t["ay"], t["az"]), _ref(p, poly), "tuned %d" % b)
    finally:
        plan.close()
