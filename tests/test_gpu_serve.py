"""Serving form: continuous batching with resident split-coordinate state.

A request's result must be bitwise the same alone and in a mix, follow the
FP64 oracle's stream-kick-stream trajectory, and admission must respect the
HBM budget; cancelling one request leaves the others unchanged."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1410_2805_amd import gridfit
from paper_1410_2805_amd import workloads as W

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


def _box(ngrid, seed, vscale=0.3):
    pos = W.zeldovich_pos64(ngrid, float(ngrid), seed)
    rng = np.random.default_rng(seed)
    vel = rng.normal(0.0, vscale, pos.shape).astype(np.float32)
    mass = np.ones(pos.shape[0], np.float32)
    return pos, vel, mass


def _submit(sr, srv, ngrid, steps, box, kinetic=None):
    pos, vel, mass = box
    n = mass.shape[0]
    op = tuple(sr.pinned_empty(n, np.float64) for _ in range(3))
    ov = tuple(sr.pinned_empty(n, np.float32) for _ in range(3))
    rid = srv.submit(float(ngrid), steps, DT, pos, vel, mass, op, ov, out_kinetic=kinetic)
    return rid, op, ov


def _drain(srv, want, max_ticks=10000):
    got = set()
    for _ in range(max_ticks):
        srv.tick()
        got.update(srv.poll())
        if want <= got:
            return got
    raise AssertionError("requests did not complete: %s" % (want - got))


def _server(sr, ctx, poly, budget=1 << 30, slots=8):
    return sr.Server(ctx, budget, slots, R_MAX, EPS, poly, CELL)


def test_result_follows_fp64_oracle(sr, ctx, poly):
    ng, steps = 14, 4
    box = _box(ng, 3)
    srv = _server(sr, ctx, poly)
    kin = np.full(1, np.nan)
    try:
        rid, op, ov = _submit(sr, srv, ng, steps, box, kinetic=kin)
        _drain(srv, {rid})
    finally:
        srv.close()
    # FP64 kinetic energy of the returned velocities (Sec. 2.6 units, m = 1)
    v = np.stack(ov, 1).astype(np.float64)
    k_ref = 0.5 * (box[2].astype(np.float64) * (v * v).sum(1)).sum()
    assert abs(kin[0] - k_ref) <= 1e-12 * k_ref
    pos, vel = box[0].copy(), box[1].astype(np.float64)
    for _ in range(steps):
        pos, vel, _ = O.sks(pos, vel, box[2], float(ng), R_MAX, EPS, poly.astype(np.float64), DT)
    got = np.stack(op, 1)
    d = got - pos
    d -= ng * np.round(d / ng)
    assert np.max(np.abs(d)) < 2e-5
    dv = np.stack(ov, 1).astype(np.float64) - vel
    assert np.max(np.abs(dv)) < 2e-5 * max(1.0, np.abs(vel).max())


def test_alone_equals_mix_bitwise(sr, ctx, poly):
    a_box = _box(18, 11)
    srv = _server(sr, ctx, poly)
    try:
        rid, op, ov = _submit(sr, srv, 18, 5, a_box)
        _drain(srv, {rid})
        alone = [a.copy() for a in op + ov]
    finally:
        srv.close()
    srv = _server(sr, ctx, poly)
    try:
        others = []
        for ng, seed in ((24, 12), (12, 13)):
            others.append(_submit(sr, srv, ng, 7, _box(ng, seed))[0])
        srv.tick()
        srv.tick()
        rid, op, ov = _submit(sr, srv, 18, 5, a_box)  # joins mid-flight
        srv.tick()
        others.append(_submit(sr, srv, 20, 3, _box(20, 14))[0])
        _drain(srv, set(others) | {rid})
        mix = [a.copy() for a in op + ov]
    finally:
        srv.close()
    for a, b in zip(alone, mix):
        assert np.array_equal(a, b)


def test_admission_budget_and_queueing(sr, ctx, poly):
    # 128 MiB: 64 MiB of state and 64 MiB of pass scratch; a 64^3 request
    # (68 B/particle of state, 17 MiB; about 210 B/particle of scratch with
    # sub-item sums, 52 MiB) fits, two at once do not; a 96^3 one never fits.
    srv = sr.Server(ctx, 128 << 20, 8, R_MAX, EPS, poly, CELL)
    try:
        with pytest.raises(sr.SRError) as e:
            _submit(sr, srv, 96, 2, _box(96, 1))
        assert e.value.code == sr.SR_EBUSY
        ids = [_submit(sr, srv, 64, 2, _box(64, 20 + k))[0] for k in range(3)]
        srv.tick()
        info = srv.info()
        assert info["active"] == 1 and info["queued"] == 2
        assert info["state_bytes_in_use"] <= info["state_bytes_capacity"]
        _drain(srv, set(ids))
        info = srv.info()
        assert info["completed"] == 3 and info["state_bytes_in_use"] == 0
        assert info["state_bytes_high_water"] <= info["state_bytes_capacity"]
    finally:
        srv.close()


def test_cancel_leaves_others_unchanged(sr, ctx, poly):
    b_box = _box(16, 31)
    srv = _server(sr, ctx, poly)
    try:
        rid, op, ov = _submit(sr, srv, 16, 4, b_box)
        _drain(srv, {rid})
        alone = [a.copy() for a in op + ov]
    finally:
        srv.close()
    srv = _server(sr, ctx, poly)
    try:
        victim = _submit(sr, srv, 22, 6, _box(22, 32))[0]
        queued = _submit(sr, srv, 30, 6, _box(30, 33))[0]
        rid, op, ov = _submit(sr, srv, 16, 4, b_box)
        srv.tick()
        srv.cancel(victim)   # active
        srv.cancel(queued)   # may be active or queued: both are allowed
        with pytest.raises(sr.SRError):
            srv.cancel(123456)
        _drain(srv, {rid})
        for _ in range(5):
            srv.tick()
            srv.poll()
        assert srv.info()["state_bytes_in_use"] == 0
        for a, b in zip(alone, [a.copy() for a in op + ov]):
            assert np.array_equal(a, b)
    finally:
        srv.close()
