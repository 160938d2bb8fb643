"""Pins of the multilevel stepping oracle (Sec. 3.1, Eq. (kicks)).

Checks against facts outside the oracle: with one level the subcycle is the
plain stream-kick-stream map, with every particle at level n it is n SKS
steps of tau / n (the definition of n kicks with 2n streams), cell counts
against a library histogram, time synchronisation of free particles, and
that dense particles given more kicks follow a fine reference more closely.
Planted mistakes in a copy of the oracle must each fail a pin."""
import importlib.util

import numpy as np
import pytest

from oracle import ml
from oracle import oracle as O
from paper_1410_2805_amd import gridfit

POLY = gridfit.poly_coeffs().astype(np.float64)
R_MAX, EPS = 3.0, 0.1


def _box(seed=1, n=400, L=12.0):
    rng = np.random.default_rng(seed)
    return L, rng.random((n, 3)) * L, rng.normal(size=(n, 3)) * 0.1, rng.uniform(0.5, 1.5, n)


def _clumped(seed=2):
    """A dense clump (about 300 particles in one 3-cell region) in a sparse
    periodic box of side 15 (5^3 chaining cells)."""
    rng = np.random.default_rng(seed)
    L = 15.0
    sparse = rng.random((250, 3)) * L
    clump = 6.0 + rng.random((300, 3)) * 3.0
    pos = np.vstack([sparse, clump])
    vel = rng.normal(size=pos.shape) * 0.05
    return L, pos, vel, np.ones(pos.shape[0])


def test_pieces_and_kick_times():
    assert ml.pieces(1, 1) == 2 and ml.pieces(1, 3) == 12 and ml.pieces(2, 4) == 24
    M = 12
    for lev in (1, 2, 3):
        times = [k for k in range(1, M + 1) if ml.kicks_at(lev, k, M)]
        # n kicks at the midpoints of n equal parts of the subcycle
        assert times == [int((2 * j + 1) * M / (2 * lev)) for j in range(lev)]


def test_single_level_is_sks(mod=ml):
    L, pos, vel, m = _box()
    p1, v1, lev = mod.subcycle(pos, vel, m, L, 3.0, R_MAX, EPS, POLY, 0.05, 10 ** 6, 1, 1)
    p2, v2, _ = O.sks(pos, vel, m, L, R_MAX, EPS, POLY, 0.05)
    assert np.all(lev == 1)
    assert np.allclose(p1, p2, rtol=0, atol=1e-13) and np.allclose(v1, v2, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3])
def test_uniform_level_is_n_sks_steps(n, mod=ml):
    L, pos, vel, m = _box(seed=3)
    p1, v1, _ = mod.subcycle(pos, vel, m, L, 3.0, R_MAX, EPS, POLY, 0.06, 10 ** 6, n, n)
    q, w = pos, vel
    for _ in range(n):
        q, w, _ = O.sks(q, w, m, L, R_MAX, EPS, POLY, 0.06 / n)
    assert np.allclose(p1, q, rtol=0, atol=1e-13) and np.allclose(v1, w, rtol=0, atol=1e-13)


def test_levels_follow_cell_counts(mod=ml):
    for L, pos, cases in ((_clumped()[0], _clumped()[1], ((4, 1, 3), (10, 1, 4), (2, 2, 3))),
                          (12.0, _box(seed=5)[1], ((1, 1, 4), (1, 1, 2)))):
        nc = int(L // 3.0)
        edges = np.linspace(0.0, L, nc + 1)
        counts, _ = np.histogramdd(pos, bins=(edges, edges, edges))
        idx = np.minimum((pos // (L / nc)).astype(int), nc - 1)
        per = counts[idx[:, 0], idx[:, 1], idx[:, 2]]
        rho = np.floor(per * nc ** 3 / pos.shape[0]).astype(int)
        for d, lmin, lmax in cases:
            want = np.clip(rho // d + 1, lmin, lmax)
            got = mod.levels(pos, L, 3.0, d, lmin, lmax)
            assert np.array_equal(got, want)
            assert len(np.unique(got)) > 1


def test_free_particles_stay_synchronous(mod=ml):
    """Zero masses: no forces; every level streams exactly v tau."""
    L, pos, vel, _ = _clumped()
    m = np.zeros(pos.shape[0])
    p, v, lev = mod.subcycle(pos, vel, np.ones(pos.shape[0]) * 0, L, 3.0, R_MAX, EPS, POLY, 0.3,
                             4, 1, 3)
    d = p - np.mod(pos + 0.3 * vel, L)
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-12 and np.array_equal(v, vel)


def test_more_kicks_for_dense_particles_help(mod=ml):
    """Against a fine reference (24 SKS steps), the multilevel subcycle
    (clump at the top level) is closer for the clump's particles than one
    plain SKS step, and no worse elsewhere."""
    L, pos, vel, m = _clumped()
    tau = 0.1
    ref_p, ref_v = pos, vel
    for _ in range(24):
        ref_p, ref_v, _ = O.sks(ref_p, ref_v, m, L, R_MAX, EPS, POLY, tau / 24)
    p_ml, v_ml, lev = mod.subcycle(pos, vel, m, L, 3.0, R_MAX, EPS, POLY, tau, 4, 1, 3)
    p_1, v_1, _ = O.sks(pos, vel, m, L, R_MAX, EPS, POLY, tau)
    dense = lev == 3
    assert dense.sum() > 100 and (lev == 1).sum() > 100
    e_ml = np.linalg.norm(v_ml - ref_v, axis=1)
    e_1 = np.linalg.norm(v_1 - ref_v, axis=1)
    assert e_ml[dense].mean() < 0.5 * e_1[dense].mean()
    assert e_ml.mean() < e_1.mean()


MUTANTS = [
    ("kick length tau", "vel[act] += a * (tau / lev[act])[:, None]", "vel[act] += a * tau"),
    ("M without the factor 2", "    return 2 * v\n", "    return v\n"),
    ("kicks at even multiples", "((t // M) % 2 == 1)", "((t // M) % 2 == 0)"),
    ("density rounded up", "ratio = np.floor(", "ratio = np.ceil("),
    ("mean density inverted", "counts[cid].astype(np.float64) * ncell / n",
     "counts[cid].astype(np.float64) * n / ncell"),
    ("levels not capped", "return np.clip(ratio // d + 1, lmin, lmax)",
     "return np.maximum(ratio // d + 1, lmin)"),
    ("last stream missing", "        if k < M:\n            pos = _stream(pos, vel, h, L)",
     "        if k < M - 1:\n            pos = _stream(pos, vel, h, L)"),
]

PINS = [test_single_level_is_sks, lambda mod: test_uniform_level_is_n_sks_steps(2, mod),
        lambda mod: test_uniform_level_is_n_sks_steps(3, mod), test_levels_follow_cell_counts,
        test_free_particles_stay_synchronous, test_more_kicks_for_dense_particles_help]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    src = open(ml.__file__).read()
    assert old in src, name
    spec = importlib.util.spec_from_loader("ml_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src.replace(old, new, 1), ml.__file__, "exec"), mod.__dict__)
    caught = False
    for pin in PINS:
        try:
            pin(mod=mod)
        except (AssertionError, ValueError, IndexError, ZeroDivisionError):
            caught = True
            break
    assert caught, name
