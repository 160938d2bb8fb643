"""FP64 reference of multilevel (density-adaptive) short-range stepping.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the CPU baseline of
bench.py may use it; the product never does).

Sec. 3.1 gives each particle a number of short-range kicks per subcycle
from the density of its leaf at the start of the subcycle, Eq. (kicks):
    l = floor(rho / rho_0) / d + 1   (integer division by d),
capped by user limits.  A particle with n kicks takes 2n streams of
tau / 2n; to keep all particles synchronous every stream is cut into the
same M pieces of tau / M, with M = 2 lcm(l_min..l_max), and a particle of
level l kicks (by tau / l, with the short-range force of all particles at
that moment) after the stream pieces m with 2 m l / M odd.

Readings: the leaf is the chaining cell (width >= cell) and rho / rho_0 its
particle count over the mean count per cell; l counts kicks directly.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O


def pieces(lmin: int, lmax: int) -> int:
    """M = 2 lcm(lmin, ..., lmax)."""
    v = 1
    for k in range(lmin, lmax + 1):
        v = v * k // math.gcd(v, k)
    return 2 * v


def kicks_at(level, m: int, M: int):
    """True where a particle of this level kicks after stream piece m."""
    level = np.asarray(level)
    t = 2 * m * level
    return (t % M == 0) & ((t // M) % 2 == 1)


def levels(pos, L: float, cell: float, d: int, lmin: int, lmax: int):
    """Kick counts per particle from the chaining-cell counts (Eq. (kicks))."""
    pos = np.asarray(pos, dtype=np.float64)
    offsets, perm, cid = O.bin(pos[:, 0], pos[:, 1], pos[:, 2], L, cell)
    counts = np.diff(offsets)
    ncell = counts.size
    n = pos.shape[0]
    ratio = np.floor(counts[cid].astype(np.float64) * ncell / n).astype(np.int64)
    return np.clip(ratio // d + 1, lmin, lmax)


def _stream(pos, vel, h, L):
    u = pos + h * vel
    u -= L * np.floor(u / L)
    u[u >= L] -= L
    return u


def subcycle(pos, vel, m, L: float, cell: float, r_max: float, eps: float, poly, tau: float,
             d: int, lmin: int, lmax: int):
    """One multilevel subcycle of length tau; returns (pos, vel, level)."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    lev = levels(pos, L, cell, d, lmin, lmax)
    M = pieces(lmin, lmax)
    h = tau / M
    pos = _stream(pos, vel, h, L)
    for k in range(1, M + 1):
        act = np.nonzero(kicks_at(lev, k, M))[0]
        if act.size:
            a = O.force(pos[:, 0], pos[:, 1], pos[:, 2], m, L, r_max, eps, poly,
                        targets=act)["a"]
            vel[act] += a * (tau / lev[act])[:, None]
        if k < M:
            pos = _stream(pos, vel, h, L)
    return pos, vel, lev
