"""FP64 reference of regenerating the grid-force polynomial from the PM.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the CPU baseline of
bench.py may use it; the product never does).

Sec. 2.4 obtains the filtered grid force numerically: pairs of test
particles at many separations and random orientations, the PM force between
them averaged, and a fit.  Here the measured radial forces f_i at
separations r_i (one unit source, massless probes) come from the FP64 PM
oracle, and the polynomial of Eq. (force) is fitted to them directly:
minimise sum_i r_i^2 (r_i p(r_i^2) - f_i)^2 over the six coefficients of
p(s) = sum_k c_k s^k (p stands for f_grid(r) / r; the weight r^2 is the
density of pair separations in 3-D).
"""
from __future__ import annotations

import numpy as np

from oracle import pm


def radial_samples(sets, ng: int, sigma: float = 0.8, ns: int = 3):
    """(r, f): separations and the radial PM force on each probe, pointing
    from the probe toward the source, FP64."""
    rs, fs = [], []
    for s in sets:
        tg = np.arange(1, s.m.shape[0])
        a = pm.pm_accel(s.pos.astype(np.float64), s.m.astype(np.float64), ng, s.L, sigma, ns,
                        targets=tg)
        fs.append(-(a * s.u).sum(axis=1))
        rs.append(s.r)
    return np.concatenate(rs), np.concatenate(fs)


def fit(r, f) -> np.ndarray:
    """c_0..c_5 of the weighted least-squares problem above (FP64)."""
    r = np.asarray(r, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    design = np.empty((r.size, 6))
    for k in range(6):
        design[:, k] = r ** (2 * k + 1) * r
    coef, *_ = np.linalg.lstsq(design, f * r, rcond=None)
    return coef


def p_of_s(c, s):
    """p(s) = sum_k c_k s^k, FP64."""
    s = np.asarray(s, dtype=np.float64)
    return sum(c[k] * s ** k for k in range(6))
