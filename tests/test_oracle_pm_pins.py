"""Pins of the FP64 long-range (PM) oracle and of the subcycled step.

Each check uses a fact the oracle does not compute itself: the Taylor
expansions of the influence function (Eq. (greenf)) and of the Super-Lanczos
derivative (Eq. (sldiff)), the paper's printed fit of the filtered grid force
(Eq. (fitform)) for the test-pair experiment of Sec. 2.3, exact CIC
identities (mass conservation, linear fields, the deposit/interpolation
adjoint), Newton's third law on the grid, and the time symmetry and
second-order accuracy of the step of Eq. (tstep).
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pm
from paper_1410_2805_amd import gridfit

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fitform(r):
    """Eq. (fitform) from the printed constants."""
    with open(os.path.join(GOLD, "fitform_constants.json")) as f:
        c = json.load(f)
    b, r2 = c["b"], r * r
    return (np.tanh(b * r) / r2 - (b / r) / np.cosh(b * r) ** 2
            + c["c"] * r * (1 + c["d"] * r2) * np.exp(-c["d"] * r2)
            + c["e"] * (1 + c["f"] * r2 + c["g"] * r2 ** 2 + c["l"] * r2 ** 3) * np.exp(-c["h"] * r2))


def test_green6_sixth_order_along_an_axis():
    """Along one axis G6 (-k^2) = 1 / (1 - h^6 / 315) + O(h^8), h = k Delta:
    the h^2 term fixes the 45/128 normalisation, and the vanishing h^4 and h^6
    terms fix the 5/64, 1/1024 and 2835/1024 weights."""
    ng, L = 64, 96.0
    g = pm.green6(ng, L)
    d = L / ng
    for n in (1, 2, 3):
        k = 2 * np.pi * n / L
        h = k * d
        for idx in ((n, 0, 0), (0, n, 0), (0, 0, n)):
            got = g[idx] * (-k * k) - 1.0
            assert got == pytest.approx(h ** 6 / 315.0, rel=0.05, abs=1e-15), (n, idx)
    assert g[0, 0, 0] == 0.0
    # off-axis: -1/k^2 to sixth order as well
    kx, ky = 2 * np.pi * 2 / L, 2 * np.pi * 1 / L
    assert g[2, 1, 0] * -(kx * kx + ky * ky) == pytest.approx(1.0, abs=2e-6)


def test_super_lanczos_fourth_order():
    """D(k) / (i k) = 1 - h^4 / 30 + O(h^6); odd in k; zero at Nyquist."""
    ng, L = 32, 40.0
    d = L / ng
    for axis in range(3):
        D = np.squeeze(pm.sl_derivative(ng, L, axis))
        assert np.all(D.real == 0)
        for n in (1, 2, 3):
            k = 2 * np.pi * n / L
            h = k * d
            assert D[n].imag / k - 1.0 == pytest.approx(-h ** 4 / 30.0, rel=0.05)
        if axis < 2:
            assert D[-1] == pytest.approx(-D[1])
            assert abs(D[ng // 2]) < 1e-12


def test_filter_limits():
    """S(0) = 1; along an axis S = exp(-k^2 sigma^2 / 4) sinc(k Delta / 2)^n_s."""
    ng, L = 32, 32.0
    s = pm.sinc_gauss(ng, L, 0.8, 3)
    assert s[0, 0, 0] == 1.0
    k = 2 * np.pi * 5 / L
    x = k / 2
    assert s[5, 0, 0] == pytest.approx(np.exp(-k * k * 0.16) * (np.sin(x) / x) ** 3, rel=1e-14)
    assert s[0, 0, 5] == pytest.approx(s[5, 0, 0], rel=1e-14)


def test_grid_unit_scaling():
    """Lengths in grid spacings: doubling L and every position at fixed N_g
    (and fixed masses) divides every acceleration by exactly 4."""
    ng = 16
    rng = np.random.default_rng(5)
    pos = rng.random((40, 3)) * 20.0
    m = rng.uniform(0.5, 2.0, 40)
    a1 = pm.pm_accel(pos, m, ng, 20.0)
    a2 = pm.pm_accel(2.0 * pos, m, ng, 40.0)
    assert np.allclose(a2 * 4.0, a1, rtol=1e-10, atol=1e-13 * np.abs(a1).max())


def test_cic_identities():
    ng, L = 12, 30.0
    d = L / ng
    rng = np.random.default_rng(3)
    pos = rng.random((500, 3)) * L
    m = rng.uniform(0.5, 2.0, 500)
    rho = pm.cic_deposit(pos, m, ng, L)
    assert rho.sum() * d ** 3 == pytest.approx(m.sum(), rel=1e-13)
    # a particle on a grid point lands on that point only; at a cell centre on 8
    one = pm.cic_deposit(np.array([[3 * d, 5 * d, 11 * d]]), np.array([2.0]), ng, L)
    assert one[3, 5, 11] * d ** 3 == pytest.approx(2.0) and np.count_nonzero(one) == 1
    mid = pm.cic_deposit(np.array([[3.5 * d, 5.5 * d, 11.5 * d]]), np.array([8.0]), ng, L)
    assert np.count_nonzero(mid) == 8 and mid[4, 6, 0] * d ** 3 == pytest.approx(1.0)
    # interpolation reproduces a linear field inside the periodic cell range
    gx = np.arange(ng)[:, None, None] * d + 0 * np.zeros((1, ng, ng))
    inner = rng.random((200, 3)) * (L - 2 * d) + 0.5 * d
    assert np.allclose(pm.cic_interp(gx, inner, ng, L), inner[:, 0], atol=1e-12)
    # adjoint: sum_grid rho g Delta^3 = sum_p m interp(g)(p)
    g = rng.normal(size=(ng, ng, ng))
    assert (rho * g).sum() * d ** 3 == pytest.approx((m * pm.cic_interp(g, pos, ng, L)).sum(),
                                                     rel=1e-12)


def test_newton_third_law_and_no_self_force():
    ng, L = 16, 20.0
    rng = np.random.default_rng(7)
    pos = rng.random((300, 3)) * L
    m = rng.uniform(0.5, 2.0, 300)
    a = pm.pm_accel(pos, m, ng, L)
    tot = (m[:, None] * a).sum(0)
    assert np.abs(tot).max() <= 1e-12 * (m[:, None] * np.abs(a)).sum()
    lone = pm.pm_accel(np.array([[3.3, 7.1, 19.9]]), np.array([5.0]), ng, L)
    assert np.abs(lone).max() < 1e-14


@pytest.mark.parametrize("r", [1.0, 2.0, 3.0, 4.0, 5.0])
def test_test_pair_reproduces_fitform(r):
    """The paper's experiment (Sec. 2.3, figure of the pair force): random
    orientations of a source / massless test pair at separation r grid cells;
    the mean radial force follows the fitted Eq. (fitform) to within the
    anisotropy scatter (standard error) plus 2.5 %."""
    ng = L = 64
    rng = np.random.default_rng(int(r * 10))
    vals = []
    for _ in range(48):
        c = rng.random(3) * L
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pos = np.stack([c, np.mod(c + r * u, L)])
        a = pm.pm_accel(pos, np.array([1.0, 0.0]), ng, L)
        vals.append(-np.dot(a[1], u))
    vals = np.asarray(vals)
    want = _fitform(r)
    sem = vals.std() / np.sqrt(vals.size)
    assert abs(vals.mean() - want) <= 3 * sem + 0.025 * want, (vals.mean(), want, sem)


def _total_force(pos, m, L, ng, poly):
    sr = O.force(pos[:, 0], pos[:, 1], pos[:, 2], m, L, 3.0, 0.1, poly)["a"]
    return sr + pm.pm_accel(pos, m, ng, L)


def _system():
    rng = np.random.default_rng(11)
    L, ng, n = 16.0, 16, 48
    pos = rng.random((n, 3)) * L
    vel = rng.normal(scale=0.3, size=(n, 3))
    m = rng.uniform(0.5, 1.5, n)
    return L, ng, pos, vel, m, gridfit.poly_coeffs().astype(np.float64)


def _wrapdiff(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


def test_ksk_free_particle_and_reversibility():
    L, ng, pos, vel, m, poly = _system()
    p1, v1, _, _ = pm.ksk_step(pos[:1], vel[:1], m[:1], L, ng, 3.0, 0.1, poly, 0.7, 3)
    assert np.allclose(_wrapdiff(p1, pos[:1] + 0.7 * vel[:1], L), 0, atol=1e-13)
    assert np.allclose(v1, vel[:1], atol=1e-14)
    p1, v1, _, _ = pm.ksk_step(pos, vel, m, L, ng, 3.0, 0.1, poly, 0.05, 3)
    p0, v0, _, _ = pm.ksk_step(p1, v1, m, L, ng, 3.0, 0.1, poly, -0.05, 3)
    assert np.abs(_wrapdiff(p0, pos, L)).max() < 1e-11
    assert np.abs(v0 - vel).max() < 1e-11


def test_ksk_second_order_against_fine_leapfrog():
    """Over a fixed time the step's error against a fine leapfrog of the total
    force shrinks about fourfold per halving of dt, and the step's own
    a_lr output equals the PM force at the returned positions."""
    L, ng, pos, vel, m, poly = _system()
    T = 0.4
    p, v = pos.copy(), vel.copy()
    nf = 256
    h = T / nf
    a = _total_force(p, m, L, ng, poly)
    for _ in range(nf):
        v = v + 0.5 * h * a
        p = np.mod(p + h * v, L)
        a = _total_force(p, m, L, ng, poly)
        v = v + 0.5 * h * a
    errs = []
    for nstep in (2, 4):
        q, w, alr = pos.copy(), vel.copy(), None
        for _ in range(nstep):
            q, w, alr, _ = pm.ksk_step(q, w, m, L, ng, 3.0, 0.1, poly, T / nstep, 3, a_lr=alr)
        assert np.allclose(alr, pm.pm_accel(q, m, ng, L), rtol=0, atol=1e-13)
        errs.append(np.abs(_wrapdiff(q, p, L)).max())
    assert errs[1] < errs[0]
    assert 2.5 < errs[0] / errs[1] < 6.0, errs


def test_polynomial_regenerated_from_pm_matches_fitform():
    """The polynomial refitted from FP64 PM test pairs (Sec. 2.4 recipe)
    reproduces the paper's printed fit of the grid force to a few percent
    over the whole short-range interval, and its residual is the
    orientation (anisotropy) scatter, not a bias."""
    from oracle import pmfit
    from paper_1410_2805_amd import workloads as W
    sets = W.pm_test_pairs(16, 2048, 64.0, 3.0, 17)
    r, f = pmfit.radial_samples(sets, 64)
    c = pmfit.fit(r, f)
    rr = np.linspace(0.1, 2.9, 57)
    got = rr * pmfit.p_of_s(c, rr * rr)
    want = _fitform(rr)
    assert np.all(np.abs(got - want) <= 0.04 * want), np.max(np.abs(got / want - 1))
    res = r * pmfit.p_of_s(c, r * r) - f
    for lo in (0.5, 1.5, 2.5):
        sel = (r >= lo) & (r < lo + 0.5)
        assert abs(res[sel].mean()) <= 4 * res[sel].std() / np.sqrt(sel.sum()) + 1e-3
