"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something it does not itself compute:
textbook closed forms (Newton, the Plummer potential), the paper's printed
grid-force fit, lattice symmetry and shell counts, a library neighbour search,
physical invariants (Newton's third law, translation invariance), a library
stable sort, and the time symmetry of the stream-kick-stream map.  A dropped
term, wrong sign, wrong index or transposed operand in the oracle fails at
least one of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1410_2805_amd import gridfit
from paper_1410_2805_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ZERO = np.zeros(6)


def _two(r, direction, mj=1.0, L=64.0, eps=1e-12, poly=ZERO, periodic=True):
    """Target at the box centre, one source at distance r along direction."""
    u = np.asarray(direction, float)
    u = u / np.linalg.norm(u)
    c = np.array([L / 2] * 3)
    p = np.stack([c, c + r * u])
    res = O.force(p[:, 0], p[:, 1], p[:, 2], np.array([1.0, mj]), L, 3.0, eps, poly,
                  periodic=periodic, targets=[0])
    return res["a"][0], u, res


@pytest.mark.parametrize("r", [1e-3, 1e-2, 0.1, 1.0, 2.5])
@pytest.mark.parametrize("direction", [(1, 0, 0), (0, -1, 0), (0.3, -0.4, 0.866)])
def test_newtonian_limit(r, direction):
    """p = 0, eps -> 0: Newton's inverse-square attraction, G = 1 (Sec. 2.6)."""
    a, u, _ = _two(r, direction, mj=2.5, eps=1e-22)
    mag = np.linalg.norm(a)
    assert mag * r * r / 2.5 == pytest.approx(1.0, rel=1e-8)
    # attractive: points from the target towards the source, along the line
    assert np.dot(a, u) > 0
    # positions near 32 carry ~1e-14 absolute rounding, so the direction is
    # exact to about 1e-14 / r
    assert np.linalg.norm(np.cross(a / mag, u)) < 2e-14 / r


@pytest.mark.parametrize("r", [0.05, 0.3, 1.0, 2.9])
def test_plummer_term_is_gradient_of_plummer_potential(r):
    """p = 0: the force is minus the gradient of the Plummer potential
    -m / sqrt(r^2 + eps) (eps added to r^2 as in Eq. (force)); checked by a
    central difference of the potential, not by the force formula."""
    eps = 0.1
    a, u, _ = _two(r, (1, 2, 2), mj=1.0, eps=eps)

    def phi(rr):
        return -1.0 / np.sqrt(rr * rr + eps)

    h = 1e-5
    grad = (phi(r + h) - phi(r - h)) / (2 * h)
    assert np.linalg.norm(a) == pytest.approx(grad, rel=1e-7)
    assert np.dot(a, u) > 0


def _fitform_from_paper(r):
    k = json.load(open(os.path.join(GOLD, "fitform_constants.json")))
    b, c, d, e, f, g, h, l = (k[n] for n in "bcdefghl")
    r2 = r * r
    return (np.tanh(b * r) / r2 - (b / r) / np.cosh(b * r) ** 2
            + c * r * (1 + d * r2) * np.exp(-d * r2)
            + e * (1 + f * r2 + g * r2 ** 2 + l * r2 ** 3) * np.exp(-h * r2))


@pytest.mark.parametrize("r", [0.2, 0.5, 1.0, 1.5, 2.0, 2.5, 2.95])
def test_short_range_is_newton_minus_paper_grid_force(r):
    """With the fitted polynomial, the pair force is the Newtonian force minus
    the paper's fitted grid force (Sec. 2.4: short range = Newton - grid;
    Eq. (fitform) with its printed constants) to within the fit error."""
    c = gridfit.poly_coeffs().astype(np.float64)
    a, u, _ = _two(r, (2, -1, 3), eps=1e-14, poly=c)
    want = 1.0 / (r * r) - _fitform_from_paper(r)
    assert abs(np.dot(a, u) - want) < 1.2e-3
    assert np.linalg.norm(a - np.dot(a, u) * u) < 1e-12


def test_fit_constants_match_paper():
    k = json.load(open(os.path.join(GOLD, "fitform_constants.json")))
    got = dict(b=gridfit.FIT_B, c=gridfit.FIT_C, d=gridfit.FIT_D, e=gridfit.FIT_E,
               f=gridfit.FIT_F, g=gridfit.FIT_G, h=gridfit.FIT_H, l=gridfit.FIT_L)
    for n, v in got.items():
        assert v == k[n]


def test_fit_quality_against_paper_form():
    """The committed float32 coefficients reproduce f_grid(r)/r within the
    stated fit error on (0, 3]."""
    c = gridfit.poly_coeffs().astype(np.float64)
    r = np.linspace(1e-3, 3.0, 20001)
    err = np.abs(r * np.polyval(c[::-1], r * r) - _fitform_from_paper(r))
    assert err.max() < 1.1e-3
    assert (err * r * r)[r > 0.1].max() < 7e-4
    # and the committed values are what the recipe gives
    assert np.allclose(gridfit.fit_poly(), c, rtol=2e-6, atol=0)


def test_cutoff_strict_and_zero_beyond():
    c = gridfit.poly_coeffs().astype(np.float64)
    a_in, _, r_in = _two(3.0 - 1e-4, (1, 0, 0), eps=0.1, poly=c)
    a_out, _, r_out = _two(3.0 + 1e-4, (1, 0, 0), eps=0.1, poly=c)
    assert r_in["npair"][0] == 1 and np.linalg.norm(a_in) > 0
    assert r_out["npair"][0] == 0 and np.all(a_out == 0.0)
    # a pair exactly at s = r_max^2 does not interact but is a tie
    a_eq, _, r_eq = _two(3.0, (0, 0, 1), eps=0.1, poly=c)
    assert r_eq["npair"][0] == 0 and np.all(a_eq == 0.0) and r_eq["A"][0] > 0


def test_minimum_image():
    """Interaction through a periodic face uses the nearest image."""
    L = 16.0
    x = np.array([0.5, L - 2.0]); y = np.array([8.0, 8.0]); z = np.array([8.0, 8.0])
    r = O.force(x, y, z, np.ones(2), L, 3.0, 1e-14, ZERO, targets=[0])
    # image separation 2.5 in -x
    assert r["npair"][0] == 1
    assert r["a"][0][0] == pytest.approx(-1.0 / 2.5 ** 2, rel=1e-10)
    x2 = np.array([0.5, L - 2.7])  # image distance 3.2: out of range
    r2 = O.force(x2, y, z, np.ones(2), L, 3.0, 1e-14, ZERO, targets=[0])
    assert r2["npair"][0] == 0 and np.all(r2["a"] == 0)
    rn = O.force(x, y, z, np.ones(2), L, 3.0, 1e-14, ZERO, periodic=False, targets=[0])
    assert rn["npair"][0] == 0  # no wrap in a non-periodic box


def test_lattice_symmetry_and_shell_counts():
    """A periodic unit cubic lattice: every particle feels zero net force and
    has exactly the shell-count number of partners with s < 9."""
    shells = json.load(open(os.path.join(GOLD, "lattice_shells.json")))["counts"]
    want = sum(v for k, v in shells.items() if int(k) < 9)
    L = 8
    g = np.arange(L, dtype=np.float64) + 0.25
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    c = gridfit.poly_coeffs().astype(np.float64)
    r = O.force(X.ravel(), Y.ravel(), Z.ravel(), np.ones(L ** 3), float(L), 3.0, 0.1, c)
    assert np.all(r["npair"] == want)
    assert np.all(np.linalg.norm(r["a"], axis=1) <= 1e-13 * r["S"])
    assert np.all(r["A"] > 0)  # the s = 9 shell is a tie shell


def test_neighbour_set_against_kdtree():
    """Pair counts and accelerations from a library periodic neighbour search
    (scipy cKDTree with boxsize) agree with the brute force."""
    spatial = pytest.importorskip("scipy.spatial")
    p = W.uniform(1500, 11.0, 7)
    pos = p.pos64()
    c = gridfit.poly_coeffs().astype(np.float64)
    eps = 0.1
    tree = spatial.cKDTree(pos, boxsize=11.0)
    pairs = tree.query_pairs(3.0, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    d = pos[j] - pos[i]
    d -= 11.0 * np.round(d / 11.0)
    s = np.einsum("ij,ij->i", d, d)
    keep = s < 9.0
    i, j, d, s = i[keep], j[keep], d[keep], s[keep]
    f = (s + eps) ** -1.5 - np.polyval(c[::-1], s)
    a = np.zeros_like(pos)
    np.add.at(a, i, f[:, None] * d)
    np.add.at(a, j, -f[:, None] * d)
    cnt = np.bincount(i, minlength=p.n) + np.bincount(j, minlength=p.n)
    r = O.force(p.x, p.y, p.z, p.m, 11.0, 3.0, eps, c)
    assert np.array_equal(r["npair"], cnt)
    assert np.max(np.linalg.norm(r["a"] - a, axis=1) / np.maximum(r["S"], 1e-30)) < 1e-12


def test_newton_third_law_and_translation():
    p = W.uniform(3000, 14.0, 11)
    p.m = np.random.default_rng(3).uniform(0.5, 2.0, p.n).astype(np.float32)
    c = gridfit.poly_coeffs().astype(np.float64)
    r = O.force(p.x, p.y, p.z, p.m, 14.0, 3.0, 0.1, c)
    m = p.m.astype(np.float64)
    mom = (m[:, None] * r["a"]).sum(axis=0)
    assert np.linalg.norm(mom) <= 1e-13 * np.sum(m * r["S"])
    shift = np.array([1.25, -3.5, 7.75])
    q = np.mod(p.pos64() + shift, 14.0)
    r2 = O.force(q[:, 0], q[:, 1], q[:, 2], p.m, 14.0, 3.0, 0.1, c)
    assert np.array_equal(r2["npair"], r["npair"])
    assert np.max(np.linalg.norm(r2["a"] - r["a"], axis=1) - 1e-13 * r["S"]) <= 0


def test_passive_skin_rule():
    """Non-periodic domain: particles closer to a face than the skin get no
    short-range force (Sec. 2.2); at exactly the skin width they are active."""
    L, skin = 20.0, 3.0
    x = np.array([2.999, 3.0, 10.0, 10.0, 17.0, 17.001])
    y = np.array([10.0, 10.0, 10.0, 10.5, 10.0, 10.0])
    z = np.full(6, 10.0)
    r = O.force(x, y, z, np.ones(6), L, 3.0, 0.1, ZERO, periodic=False, skin=skin)
    assert list(r["passive"]) == [True, False, False, False, False, True]
    assert np.all(r["a"][0] == 0) and r["npair"][0] == 0
    assert r["npair"][2] == 1  # 2 and 3 are 0.5 apart, far from the faces
    # the passive particle 0 still acts as a source on the active particle 1
    assert r["npair"][1] == 1


def test_bin_matches_library_stable_sort():
    p = W.uniform(20000, 30.0, 5)
    off, perm, cid = O.bin(p.x, p.y, p.z, 30.0, 3.0)
    nc = 10
    assert off.shape == (nc ** 3 + 1,)
    # the library's stable argsort of the cell ids is the permutation
    assert np.array_equal(perm, np.argsort(cid, kind="stable"))
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(np.bincount(cid, minlength=nc ** 3))]))
    assert off[0] == 0 and off[-1] == p.n and np.all(np.diff(off) >= 0)
    # cell coordinates bracket the positions
    cx = cid % nc
    cy = (cid // nc) % nc
    cz = cid // (nc * nc)
    for comp, cc in ((p.x, cx), (p.y, cy), (p.z, cz)):
        assert np.all(cc * 3.0 <= comp.astype(np.float64) + 1e-9)
        assert np.all(comp.astype(np.float64) < (cc + 1) * 3.0 + 1e-9)


def test_bin_exact_cell_edges():
    """Dyadic geometry (L = 32, 8 cells of 4): a coordinate exactly on an edge
    belongs to the upper cell; one float32 ulp below belongs to the lower one;
    the largest float32 below L belongs to the last cell."""
    f32 = np.float32
    xs = []
    for k in range(1, 8):
        xs += [f32(4 * k), np.nextafter(f32(4 * k), f32(0))]
    xs += [f32(0.0), np.nextafter(f32(32.0), f32(0))]
    x = np.array(xs, dtype=np.float32)
    y = np.zeros_like(x)
    off, perm, cid = O.bin(x, y, y, 32.0, 4.0)
    want = []
    for k in range(1, 8):
        want += [k, k - 1]
    want += [0, 7]
    assert list(cid) == want


def test_bin_rejects_out_of_range():
    x = np.array([1.0, 32.0], dtype=np.float32)
    with pytest.raises(ValueError):
        O.bin(x, np.zeros(2), np.zeros(2), 32.0, 4.0)
    with pytest.raises(ValueError):
        O.bin(np.array([-1e-7]), np.zeros(1), np.zeros(1), 32.0, 4.0)
    with pytest.raises(ValueError):
        O.bin(np.array([np.nan]), np.zeros(1), np.zeros(1), 32.0, 4.0)


def test_bin_empty_and_single():
    off, perm, cid = O.bin(np.zeros(0), np.zeros(0), np.zeros(0), 9.0, 3.0)
    assert off.shape == (28,) and np.all(off == 0) and perm.shape == (0,)
    off, perm, cid = O.bin(np.array([8.9]), np.array([0.0]), np.array([4.5]), 9.0, 3.0)
    assert list(perm) == [0] and cid[0] == 2 + 3 * (0 + 3 * 1)


def test_sks_free_streaming_and_reversibility():
    """Stream-kick-stream (Sec. 2.5): with no partner inside r_max a particle
    moves by v dt; the map run with -dt undoes a step (time symmetry of the
    symmetric split); momentum is conserved."""
    c = gridfit.poly_coeffs().astype(np.float64)
    L = 12.0
    pos = np.array([[1.0, 1.0, 1.0], [7.0, 7.0, 7.0]])
    vel = np.array([[0.5, -0.25, 0.125], [-1.0, 0.0, 2.0]])
    p1, v1, a1 = O.sks(pos, vel, np.ones(2), L, 3.0, 0.1, c, 0.1)
    assert np.all(a1 == 0)
    assert np.allclose(p1, np.mod(pos + 0.1 * vel, L), rtol=0, atol=1e-14)
    p = W.uniform(400, 9.0, 21)
    pos = p.pos64()
    vel = np.random.default_rng(2).normal(0, 0.3, pos.shape)
    m = np.ones(p.n)
    q, w, _ = O.sks(pos, vel, m, 9.0, 3.0, 0.1, c, 0.02)
    back, vb, _ = O.sks(q, w, m, 9.0, 3.0, 0.1, c, -0.02)
    dpos = back - pos
    dpos -= 9.0 * np.round(dpos / 9.0)
    assert np.max(np.abs(dpos)) < 1e-10 and np.max(np.abs(vb - vel)) < 1e-10
    assert np.allclose((m[:, None] * w).sum(0), (m[:, None] * vel).sum(0), atol=1e-10)


def test_sks_one_step_closed_form():
    """Two particles at rest, p = 0, eps -> 0: one stream-kick-stream step
    leaves the first half stream idle, kicks each by dt m / r^2 towards the
    other (Newton) and streams it by half the new velocity."""
    L, r, dt = 20.0, 1.25, 0.01
    pos = np.array([[5.0, 7.0, 9.0], [5.0 + r, 7.0, 9.0]])
    vel = np.zeros((2, 3))
    m = np.array([1.0, 3.0])
    p1, v1, a1 = O.sks(pos, vel, m, L, 3.0, 1e-22, ZERO, dt)
    assert a1[0, 0] == pytest.approx(3.0 / r ** 2, rel=1e-12)
    assert a1[1, 0] == pytest.approx(-1.0 / r ** 2, rel=1e-12)
    assert v1[0, 0] == pytest.approx(dt * 3.0 / r ** 2, rel=1e-12)
    assert p1[0, 0] == pytest.approx(5.0 + 0.5 * dt * dt * 3.0 / r ** 2, rel=1e-14)
    assert np.all(v1[:, 1:] == 0) and np.all(p1[:, 1:] == pos[:, 1:])


def _on_axis(sources, L=64.0, eps=1e-22, poly=ZERO):
    """Target at the box centre, sources at signed distances along x with the
    given masses: [(distance, mass), ...].  Returns the oracle's result for
    the target."""
    c = L / 2
    x = np.array([c] + [c + d for d, _ in sources])
    y = np.full(x.shape, c)
    m = np.array([1.0] + [mj for _, mj in sources])
    return O.force(x, y, y, m, L, 3.0, eps, poly, targets=[0])


@pytest.mark.parametrize("r,mj", [(0.05, 1.0), (0.5, 2.0), (1.7, 0.25), (2.9, 4.0)])
def test_abs_sum_two_particles_closed_form(r, mj):
    """S_i, the per-target sum of absolute pair terms, for one source: with
    p = 0 and eps -> 0 it is Newton's m / r^2 (Sec. 2.6, G = 1), and with
    eps = 0.1 the Plummer magnitude m r / (r^2 + eps)^(3/2).  One pair has
    S_i = |a_i|."""
    res = _on_axis([(r, mj)])
    assert res["S"][0] == pytest.approx(mj / r ** 2, rel=1e-12)
    assert res["S"][0] == pytest.approx(np.linalg.norm(res["a"][0]), rel=1e-14)
    res = _on_axis([(-r, mj)], eps=0.1)
    assert res["S"][0] == pytest.approx(mj * r / (r * r + 0.1) ** 1.5, rel=1e-12)


def test_abs_sum_three_particles_closed_form():
    """Two sources on opposite sides: the accelerations cancel or partly
    cancel, S_i still adds both magnitudes; a source beyond r_max adds to
    neither."""
    res = _on_axis([(1.5, 2.0), (-1.5, 2.0)])
    assert np.all(np.abs(res["a"][0]) < 1e-14)
    assert res["S"][0] == pytest.approx(2 * 2.0 / 1.5 ** 2, rel=1e-12)
    res = _on_axis([(0.8, 1.0), (-2.2, 3.0), (3.3, 5.0)])
    want_s = 1.0 / 0.8 ** 2 + 3.0 / 2.2 ** 2
    want_a = 1.0 / 0.8 ** 2 - 3.0 / 2.2 ** 2
    assert res["npair"][0] == 2
    assert res["S"][0] == pytest.approx(want_s, rel=1e-12)
    assert res["a"][0][0] == pytest.approx(want_a, rel=1e-12)
    # a fitted polynomial changes the terms, not the rule: S_i = sum of the
    # two one-source magnitudes
    c = gridfit.poly_coeffs().astype(np.float64)
    both = _on_axis([(0.8, 1.0), (-2.2, 3.0)], eps=0.1, poly=c)
    one = _on_axis([(0.8, 1.0)], eps=0.1, poly=c)
    two = _on_axis([(-2.2, 3.0)], eps=0.1, poly=c)
    assert both["S"][0] == pytest.approx(np.linalg.norm(one["a"][0]) + np.linalg.norm(two["a"][0]),
                                         rel=1e-13)


@pytest.mark.parametrize("sign", [-1.0, 1.0])
def test_tie_band_membership(sign):
    """A_i collects the pairs whose exact s lies within 2^-18 r_max^2 of the
    cutoff on either side (pairs a float32 s may classify the other way):
    s = r_max^2 (1 +- 2^-19) is in the band, s = r_max^2 (1 +- 2^-17) is not.
    Its value is the pair's magnitude, m / r^2 for p = 0, eps -> 0."""
    rin = 3.0 * np.sqrt(1.0 + sign * 2.0 ** -19)
    rout = 3.0 * np.sqrt(1.0 + sign * 2.0 ** -17)
    res = _on_axis([(rin, 2.0)])
    assert res["A"][0] == pytest.approx(2.0 / rin ** 2, rel=1e-10)
    assert res["npair"][0] == (1 if sign < 0 else 0)
    if sign > 0:
        assert np.all(res["a"][0] == 0.0) and res["S"][0] == 0.0
    else:
        assert res["S"][0] == pytest.approx(res["A"][0], rel=1e-14)
    res = _on_axis([(-rout, 2.0)])
    assert res["A"][0] == 0.0
    assert res["npair"][0] == (1 if sign < 0 else 0)
    # only the tie pair contributes to A_i when a near pair is present too
    res = _on_axis([(rin, 2.0), (-0.5, 1.0), (1.0, 1.0)])
    assert res["A"][0] == pytest.approx(2.0 / rin ** 2, rel=1e-10)
