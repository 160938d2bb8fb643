"""Multilevel subcycles (Sec. 3.1, Eq. (kicks)) inside the full step: the
HIP path against the FP64 oracle, and against the plain step where the two
must coincide."""
import numpy as np
import pytest
import torch

from oracle import pm as PMO
from paper_1410_2805_amd import gridfit
from paper_1410_2805_amd import workloads as W

pytestmark = pytest.mark.gpu

R_MAX, EPS, CELL = 3.0, 0.1, 3.0


@pytest.fixture(scope="module")
def sr():
    from paper_1410_2805_amd import sr as S
    return S


@pytest.fixture(scope="module")
def ctx(sr):
    c = sr.Context(0)
    yield c
    c.close()


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype)


def _clustered(L=16.0, n=5000, seed=4):
    """Halo particles on a periodic box, kept 1e-5 away from chaining-cell
    faces so that float32 offsets and FP64 positions agree on every cell."""
    c = W.nfw_share(n, L, seed, periodic=True, halo_cap=n // 3)
    pos = np.stack([c.x, c.y, c.z], 1).astype(np.float64)
    h = L / int(L // CELL)
    fr = pos / h - np.floor(pos / h)
    pos = np.where(fr < 1e-5, pos + 2e-5, np.where(fr > 1 - 1e-5, pos - 2e-5, pos))
    pos = np.mod(pos, L)
    vel = np.random.default_rng(seed).normal(scale=0.1, size=pos.shape).astype(np.float32)
    return L, pos, vel, np.ones(pos.shape[0], np.float32)


def _state(sr, ctx, L, pos, vel, m):
    box = sr.Box.make(L)
    x, y, z = [_dev(pos[:, d], torch.float64) for d in range(3)]
    c3, ox, oy, oz = sr.sr_split_from_f64(ctx, x, y, z, box, CELL)
    st = {"cell3": c3, "ox": ox, "oy": oy, "oz": oz, "vx": _dev(vel[:, 0]), "vy": _dev(vel[:, 1]),
          "vz": _dev(vel[:, 2]), "m": _dev(m)}
    return box, st


def _run(sr, ctx, pmh, box, st, prm, steps=1):
    n = st["m"].shape[0]
    lr = tuple(torch.zeros(n, dtype=torch.float32, device="cuda:0") for _ in range(3))
    so = tuple(torch.zeros(n, dtype=torch.float32, device="cuda:0") for _ in range(3))
    for k in range(steps):
        sr.sr_ksk_step(ctx, pmh, st, box, prm, lr, k > 0, so)
    gx, gy, gz = sr.sr_split_to_f64(ctx, st["cell3"], st["ox"], st["oy"], st["oz"], box, CELL)
    ctx.sync()
    return (torch.stack([gx, gy, gz], 1).cpu().numpy(),
            torch.stack([st["vx"], st["vy"], st["vz"]], 1).double().cpu().numpy())


def test_uniform_level_equals_plain_subcycles(sr, ctx):
    """Every particle at level 2 with one subcycle is the plain step with two
    subcycles, operation for operation: bitwise equal."""
    L, pos, vel, m = _clustered()
    poly = gridfit.poly_coeffs()
    pmh = sr.PM(ctx, 16, L)
    try:
        box, st = _state(sr, ctx, L, pos, vel, m)
        a = _run(sr, ctx, pmh, box, st, sr.StepParams.make(R_MAX, EPS, poly, CELL, 0.02, 1,
                                                            ml=(10 ** 6, 2, 2)), steps=2)
        box, st = _state(sr, ctx, L, pos, vel, m)
        b = _run(sr, ctx, pmh, box, st, sr.StepParams.make(R_MAX, EPS, poly, CELL, 0.02, 2),
                 steps=2)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    finally:
        pmh.close()


@pytest.mark.parametrize("d,lmin,lmax", [(4, 1, 3), (2, 1, 4), (8, 2, 3)])
def test_multilevel_step_matches_oracle(sr, ctx, d, lmin, lmax):
    L, pos, vel, m = _clustered()
    poly = gridfit.poly_coeffs()
    dt = 0.02
    pmh = sr.PM(ctx, 16, L)
    try:
        box, st = _state(sr, ctx, L, pos, vel, m)
        gp, gv = _run(sr, ctx, pmh, box, st,
                      sr.StepParams.make(R_MAX, EPS, poly, CELL, dt, 1, ml=(d, lmin, lmax)))
    finally:
        pmh.close()
    P, V, alr, _ = PMO.ksk_step(pos, vel.astype(np.float64), m.astype(np.float64), L, 16, R_MAX,
                                EPS, poly.astype(np.float64), dt, 1, ml=(d, lmin, lmax, CELL))
    from oracle import ml as ML
    lev = ML.levels(pos, L, CELL, d, lmin, lmax)
    assert len(np.unique(lev)) > 1
    dx = gp - P
    dx -= L * np.round(dx / L)
    vs = np.sqrt((V ** 2).sum(1).mean())
    dv = np.abs(gv - V).max()
    print("levels %s: max|dv| %.3e (rms v %.3e) max|dx| %.3e" % (np.bincount(lev), dv, vs,
                                                                 np.abs(dx).max()))
    # float32 velocities and kicks, float32 offsets: the bounds of the plain
    # step's parity test (velocity error over a step, then carried by streams)
    assert dv <= 2e-5 * vs + 1e-5
    assert np.abs(dx).max() <= 2e-5 * dt * vs + 1e-6


@pytest.mark.parametrize("xsplit", [2, 3])
def test_multilevel_x_subcells_match_oracle(sr, ctx, xsplit):
    """Masked passes on x sub-cells: a stencil spans +-xsplit sub-cells in x,
    so the cells binned around each active one (and the targets' stencils)
    span that far too; the step still follows the FP64 oracle."""
    L, pos, vel, m = _clustered(L=21.0, n=9000, seed=11)
    poly = gridfit.poly_coeffs()
    dt = 0.02
    before = ctx.get_tuning()
    pmh = sr.PM(ctx, 16, L)
    try:
        ctx.set_tuning(xsplit=xsplit)
        box, st = _state(sr, ctx, L, pos, vel, m)
        gp, gv = _run(sr, ctx, pmh, box, st,
                      sr.StepParams.make(R_MAX, EPS, poly, CELL, dt, 1, ml=(4, 1, 3)))
    finally:
        ctx.set_tuning(**before)
        pmh.close()
    P, V, _, _ = PMO.ksk_step(pos, vel.astype(np.float64), m.astype(np.float64), L, 16, R_MAX,
                              EPS, poly.astype(np.float64), dt, 1, ml=(4, 1, 3, CELL))
    dx = gp - P
    dx -= L * np.round(dx / L)
    vs = np.sqrt((V ** 2).sum(1).mean())
    dv = np.abs(gv - V).max()
    print("xsplit %d: max|dv| %.3e (rms v %.3e) max|dx| %.3e" % (xsplit, dv, vs, np.abs(dx).max()))
    assert dv <= 2e-5 * vs + 1e-5
    assert np.abs(dx).max() <= 2e-5 * dt * vs + 1e-6


@pytest.mark.parametrize("n,seed", [(20000, 7), (60000, 8)])
def test_multilevel_dense_cells_match_oracle(sr, ctx, n, seed):
    """Dense cells whose stencils hold 4,096..19,329 sources: the multilevel
    passes cut them into finer items whose stencil sources are split over up
    to five sub-items, summed afterwards in order; the step still follows the
    FP64 oracle."""
    L, pos, vel, m = _clustered(n=n, seed=seed)
    poly = gridfit.poly_coeffs()
    dt = 0.02
    pmh = sr.PM(ctx, 16, L)
    try:
        box, st = _state(sr, ctx, L, pos, vel, m)
        gp, gv = _run(sr, ctx, pmh, box, st,
                      sr.StepParams.make(R_MAX, EPS, poly, CELL, dt, 1, ml=(4, 1, 3)))
        # the same step again from the same state: bitwise reproducible
        box, st = _state(sr, ctx, L, pos, vel, m)
        gp2, gv2 = _run(sr, ctx, pmh, box, st,
                        sr.StepParams.make(R_MAX, EPS, poly, CELL, dt, 1, ml=(4, 1, 3)))
    finally:
        pmh.close()
    assert np.array_equal(gp, gp2) and np.array_equal(gv, gv2)
    P, V, _, _ = PMO.ksk_step(pos, vel.astype(np.float64), m.astype(np.float64), L, 16, R_MAX,
                              EPS, poly.astype(np.float64), dt, 1, ml=(4, 1, 3, CELL))
    dx = gp - P
    dx -= L * np.round(dx / L)
    vs = np.sqrt((V ** 2).sum(1).mean())
    dv = np.abs(gv - V).max()
    print("n=%d: max|dv| %.3e (rms v %.3e) max|dx| %.3e" % (n, dv, vs, np.abs(dx).max()))
    assert dv <= 2e-5 * vs + 1e-5
    assert np.abs(dx).max() <= 2e-5 * dt * vs + 1e-6


def test_multilevel_parameters_rejected(sr, ctx):
    L, pos, vel, m = _clustered(n=500)
    pmh = sr.PM(ctx, 16, L)
    try:
        box, st = _state(sr, ctx, L, pos, vel, m)
        n = pos.shape[0]
        z = lambda: torch.zeros(n, dtype=torch.float32, device="cuda:0")
        for ml in ((4, 0, 2), (4, 3, 2), (4, 1, 5), (-1, 1, 2)):
            prm = sr.StepParams.make(R_MAX, EPS, gridfit.poly_coeffs(), CELL, 0.01, 1, ml=ml)
            with pytest.raises(sr.SRError):
                sr.sr_ksk_step(ctx, pmh, st, box, prm, (z(), z(), z()), 0, (z(), z(), z()))
    finally:
        pmh.close()


def test_multilevel_two_subcycles_matches_oracle(sr, ctx):
    """Levels are reassigned at the start of every subcycle: two subcycles
    per step, two steps, against the FP64 oracle step."""
    L, pos, vel, m = _clustered(seed=6)
    poly = gridfit.poly_coeffs()
    dt = 0.02
    pmh = sr.PM(ctx, 16, L)
    try:
        box, st = _state(sr, ctx, L, pos, vel, m)
        gp, gv = _run(sr, ctx, pmh, box, st,
                      sr.StepParams.make(R_MAX, EPS, poly, CELL, dt, 2, ml=(4, 1, 3)), steps=2)
    finally:
        pmh.close()
    P, V, alr = pos, vel.astype(np.float64), None
    for _ in range(2):
        P, V, alr, _ = PMO.ksk_step(P, V, m.astype(np.float64), L, 16, R_MAX, EPS,
                                    poly.astype(np.float64), dt, 2, a_lr=alr,
                                    ml=(4, 1, 3, CELL))
    dx = gp - P
    dx -= L * np.round(dx / L)
    vs = np.sqrt((V ** 2).sum(1).mean())
    dv = np.abs(gv - V).max()
    print("two subcycles x two steps: max|dv| %.3e (rms v %.3e) max|dx| %.3e"
          % (dv, vs, np.abs(dx).max()))
    assert dv <= 4e-5 * vs + 2e-5
    assert np.abs(dx).max() <= 4e-5 * 2 * dt * vs + 2e-6
