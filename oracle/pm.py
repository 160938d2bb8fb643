"""FP64 reference of the long-range particle-mesh (PM) force (numpy).

TEST INFRASTRUCTURE ONLY (the test suite, the smoke check and the CPU
baseline of bench.py may use it; the product never does).  It follows the
long-range solver of Sec. 2.3 step by step, in float64:

  1. Cloud-in-cell deposit of the particle masses on a periodic N_g^3 grid of
     spacing Delta = L / N_g (grid point j sits at j Delta).
  2. Forward FFT of the density.
  3. Multiply by the sinc-Gaussian filter of Eq. (filter),
        S(k) = exp(-|k|^2 sigma^2 / 4) * prod_i [ (2 / (k_i Delta)) sin(k_i Delta / 2) ]^n_s,
     by the sixth-order influence function G_6 of Eq. (greenf), which
     approximates -1/k^2, and by 4 pi (G = 1 in code units, Sec. 2.6), giving
     the potential phi(k) = 4 pi G_6 S rho(k).
  4. For each axis, the fourth-order Super-Lanczos derivative of Eq. (sldiff),
        D_i(k) = (i / Delta) [ (4/3) sin(k_i Delta) - (1/6) sin(2 k_i Delta) ],
     and the acceleration a_i(k) = -D_i(k) phi(k); one inverse FFT per axis.
  5. Cloud-in-cell interpolation of the three acceleration grids back to the
     particles (same weights as the deposit).

ksk_step composes these with the short-range stream-kick-stream map of the
C oracle into the subcycled step of Eq. (tstep) (Sec. 2.5).

Readings (also listed in the design notes): the filter's sinc factor is
taken per axis (separable, the form of a TSC-like window), sigma is measured
in grid spacings (the matching scale and the fit of Eq. (fitform) are in grid
units), k_i = 2 pi n_i / L
with n_i the signed integer frequency, and the derivative formula is read
with the exponent e^{i 2 pi j x / L} (the printed formula drops the i).
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as _sr


def _freqs(ng: int, L: float):
    n = np.fft.fftfreq(ng, d=1.0 / ng)           # signed integer frequencies
    nr = np.fft.rfftfreq(ng, d=1.0 / ng)
    k = 2.0 * np.pi * n / L
    kr = 2.0 * np.pi * nr / L
    return k[:, None, None], k[None, :, None], kr[None, None, :]


def green6(ng: int, L: float) -> np.ndarray:
    """G_6(k) of Eq. (greenf) on the rfft grid; G_6(0) = 0 (mean removed)."""
    d = L / ng
    kx, ky, kz = _freqs(ng, L)
    s = 0.0
    for kc in (kx, ky, kz):
        s = s + np.cos(kc * d) - (5.0 / 64.0) * np.cos(2 * kc * d) + (1.0 / 1024.0) * np.cos(4 * kc * d)
    s = s - 2835.0 / 1024.0
    with np.errstate(divide="ignore"):
        g = (45.0 / 128.0) * d * d / s
    g[0, 0, 0] = 0.0
    return g


def sinc_gauss(ng: int, L: float, sigma: float = 0.8, ns: int = 3) -> np.ndarray:
    """S(k) of Eq. (filter), sinc factor per axis; sigma in grid spacings."""
    d = L / ng
    kx, ky, kz = _freqs(ng, L)
    k2 = kx * kx + ky * ky + kz * kz
    sd = sigma * d
    out = np.exp(-k2 * sd * sd / 4.0)
    for kc in (kx, ky, kz):
        x = kc * d / 2.0
        with np.errstate(invalid="ignore", divide="ignore"):
            sc = np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))
        out = out * sc ** ns
    return out


def sl_derivative(ng: int, L: float, axis: int) -> np.ndarray:
    """D_axis(k) of Eq. (sldiff) (imaginary unit included)."""
    d = L / ng
    kc = _freqs(ng, L)[axis]
    return 1j * ((4.0 / 3.0) * np.sin(kc * d) - (1.0 / 6.0) * np.sin(2.0 * kc * d)) / d


def _cic(pos: np.ndarray, ng: int, L: float):
    d = L / ng
    u = pos / d
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    return i0 % ng, (i0 + 1) % ng, f


def cic_deposit(pos: np.ndarray, m: np.ndarray, ng: int, L: float) -> np.ndarray:
    """Mass density on the grid (mass / Delta^3)."""
    i0, i1, f = _cic(pos, ng, L)
    rho = np.zeros((ng, ng, ng))
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = i1[:, 0] if cx else i0[:, 0]
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = i1[:, 1] if cy else i0[:, 1]
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = i1[:, 2] if cz else i0[:, 2]
                np.add.at(rho, (ix, iy, iz), m * wx * wy * wz)
    d = L / ng
    return rho / d ** 3


def cic_interp(grid: np.ndarray, pos: np.ndarray, ng: int, L: float) -> np.ndarray:
    i0, i1, f = _cic(pos, ng, L)
    out = np.zeros(pos.shape[0])
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = i1[:, 0] if cx else i0[:, 0]
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = i1[:, 1] if cy else i0[:, 1]
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = i1[:, 2] if cz else i0[:, 2]
                out += grid[ix, iy, iz] * wx * wy * wz
    return out


def pm_accel(pos, m, ng: int, L: float, sigma: float = 0.8, ns: int = 3,
             targets=None) -> np.ndarray:
    """(n, 3) long-range accelerations (float64) of all particles, or of the
    particles listed in targets (every particle still sources the field)."""
    pos = np.asarray(pos, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    rho_k = np.fft.rfftn(cic_deposit(pos, m, ng, L))
    phi_k = 4.0 * np.pi * green6(ng, L) * sinc_gauss(ng, L, sigma, ns) * rho_k
    at = pos if targets is None else pos[np.asarray(targets)]
    acc = np.zeros_like(at)
    for ax in range(3):
        a_grid = np.fft.irfftn(-sl_derivative(ng, L, ax) * phi_k, s=(ng, ng, ng), axes=(0, 1, 2))
        acc[:, ax] = cic_interp(a_grid, at, ng, L)
    return acc


def ksk_step(pos, vel, m, L: float, ng: int, r_max: float, eps: float, poly, dt: float,
             nsub: int, a_lr=None, sigma: float = 0.8, ns: int = 3, ml=None):
    """One full step of Eq. (tstep): a long-range half kick, nsub short-range
    stream-kick-stream subcycles of length dt / nsub (Sec. 2.5), then the
    long-range force at the new positions and the second half kick.

    a_lr, if given, is the PM acceleration at the incoming positions (the
    previous step's final one); ml = (d, l_min, l_max, cell) replaces each
    subcycle by the multilevel one of oracle.ml (then a_sr_last is None).
    Returns (pos, vel, a_lr_new, a_sr_last)."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    if a_lr is None:
        a_lr = pm_accel(pos, m, ng, L, sigma, ns)
    vel = vel + 0.5 * dt * a_lr
    tau = dt / nsub
    a_sr = np.zeros_like(pos)
    for _ in range(nsub):
        if ml is None:
            pos, vel, a_sr = _sr.sks(pos, vel, m, L, r_max, eps, poly, tau)
        else:
            from oracle import ml as _ml
            d, lmin, lmax, cell = ml
            pos, vel, _ = _ml.subcycle(pos, vel, m, L, cell, r_max, eps, poly, tau, d, lmin,
                                       lmax)
            a_sr = None
    a_lr = pm_accel(pos, m, ng, L, sigma, ns)
    vel = vel + 0.5 * dt * a_lr
    return pos, vel, a_lr, a_sr
