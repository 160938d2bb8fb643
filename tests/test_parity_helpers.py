"""CPU checks of the test helpers that compose oracle calls."""
import numpy as np

from oracle import oracle as O
from paper_1410_2805_amd import gridfit
from paper_1410_2805_amd import workloads as W
from tests.parity import kick_accel_ref, position_slack


def test_kick_accel_ref_is_the_oracle_sks_kick():
    """The sampled kick acceleration equals the one oracle_sks applies."""
    c = gridfit.poly_coeffs().astype(np.float64)
    p = W.uniform(600, 10.0, 4)
    pos = p.pos64()
    vel = np.random.default_rng(1).normal(0, 0.4, pos.shape)
    dt = 0.05
    _, _, acc = O.sks(pos, vel, np.ones(p.n), 10.0, 3.0, 0.1, c, dt)
    tg = np.array([0, 17, 299, 599])
    ref = kick_accel_ref(pos, vel, np.ones(p.n), 10.0, tg, 3.0, 0.1, c, dt)
    assert np.allclose(ref["a"], acc[tg], rtol=0, atol=1e-13 * np.abs(acc).max())


def test_position_slack_bounds_a_perturbation():
    """Moving every coordinate by at most u changes each acceleration by no
    more than the slack (random perturbations of a clustered box)."""
    c = gridfit.poly_coeffs().astype(np.float64)
    p = W.nfw_share(3000, 14.0, 2, periodic=True, halo_cap=800)
    pos = p.pos64()
    h = 14.0 / 4
    u = 0.5 * float(np.spacing(np.float32(h)))
    base = O.force(pos[:, 0], pos[:, 1], pos[:, 2], p.m, 14.0, 3.0, 0.1, c)
    for seed in range(3):
        q = pos + np.random.default_rng(seed).uniform(-u, u, pos.shape)
        q -= 14.0 * np.floor(q / 14.0)
        moved = O.force(q[:, 0], q[:, 1], q[:, 2], p.m, 14.0, 3.0, 0.1, c)
        err = np.linalg.norm(moved["a"] - base["a"], axis=1)
        # pairs that cross the cutoff lie in the tie band (A): s moves by < 2^-18 r_max^2
        ok = err <= position_slack(np.maximum(base["npair"], moved["npair"]), 1.0, h, 0.1) \
            + base["A"] + moved["A"] + 1e-12
        assert ok.all()
