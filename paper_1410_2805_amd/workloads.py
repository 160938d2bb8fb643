"""Seeded synthetic particle inputs.

This module only draws random numbers and lays particles out; it holds none
of the force method's arithmetic.  Both the HIP path and the FP64 oracle take
its arrays as inputs, so the two sides see the same particles.

Lengths are in grid units (the code units of Sec. 2.6, Eq. (scaling): one
unit is one long-range PM grid cell) and every workload has mean number
density 1 per unit volume.  All positions are returned as float32 structure-
of-arrays (x, y, z) with 0 <= x < L; masses are float32 ones.

The paper's own runs use cosmological initial conditions and the public
code-comparison data of Sec. 4, which are not available here.  The recipes
below stand in for them with the same shapes and distributions:

* ``uniform``     -- Poisson (uniform random) particles in a periodic cube.
* ``zeldovich``   -- a cubic lattice displaced by a Gaussian random field
                     with power spectrum P(k) ~ k^-2 cut at the grid Nyquist
                     frequency (the Zel'dovich approximation).
* ``nfw_share``   -- one node's share of a clustered late-time volume: most
                     particles in NFW halos with a power-law multiplicity
                     function, the rest uniform; non-periodic (overloaded,
                     Sec. 2.2).
* ``batch_boxes`` -- many independent periodic boxes of log-uniform size,
                     half uniform and half clustered.
* ``serving_trace`` -- Poisson arrival times and box sizes for requests.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np


@dataclasses.dataclass
class Particles:
    """Float32 SoA particle set inside the box [0, L)^3."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    L: float
    periodic: bool = True
    skin: float = 0.0

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def pos64(self) -> np.ndarray:
        """(n, 3) float64 copy of the float32 positions (exact promotion)."""
        return np.stack([self.x, self.y, self.z], axis=1).astype(np.float64)


def _wrap_f32(v64: np.ndarray, L: float) -> np.ndarray:
    """Round to float32 and wrap into [0, L) in float32.

    Rounding can turn a value just below L into L itself; such values, and any
    that fall outside, are brought back by one period so that 0 <= v < L holds
    for the float32 result that both sides will read.
    """
    v = np.mod(v64, L).astype(np.float32)
    Lf = np.float32(L)
    v[v >= Lf] -= Lf
    v[v < 0] += Lf
    # a wrap in float32 can itself round onto L; pull such values just inside
    bad = v >= Lf
    if bad.any():
        v[bad] = np.nextafter(Lf, np.float32(0))
    return v


def _soa(pos: np.ndarray, L: float, periodic: bool = True, skin: float = 0.0) -> Particles:
    x = _wrap_f32(pos[:, 0], L)
    y = _wrap_f32(pos[:, 1], L)
    z = _wrap_f32(pos[:, 2], L)
    m = np.ones(x.shape[0], dtype=np.float32)
    return Particles(x, y, z, m, float(L), periodic, skin)


def uniform(n: int, L: float, seed: int) -> Particles:
    """n particles uniform in the periodic cube [0, L)^3."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * L
    return _soa(pos, L)


def zeldovich(ngrid: int, L: float, seed: int, rms: float = 0.5) -> Particles:
    """Float32 particles of ``zeldovich_pos64``."""
    return _soa(zeldovich_pos64(ngrid, L, seed, rms), L)


def zeldovich_pos64(ngrid: int, L: float, seed: int, rms: float = 0.5) -> np.ndarray:
    """(ngrid^3, 3) float64 positions in [0, L)^3: ngrid^3 particles on the lattice q = (i + 1/2) * L/ngrid, displaced by
    a Zel'dovich displacement psi with del.psi = -delta.

    delta is a Gaussian random field with P(k) ~ k^-2 for 0 < |k| <= pi/h
    (h = L/ngrid; a spherical cut at the Nyquist frequency) and zero beyond;
    psi(k) = i k delta(k) / k^2.  The field is scaled so that the 3-D rms of
    |psi| over the particles equals ``rms``.
    """
    rng = np.random.default_rng(seed)
    h = L / ngrid
    white = rng.standard_normal((ngrid, ngrid, ngrid))
    wk = np.fft.rfftn(white)
    del white
    k1 = 2.0 * np.pi * np.fft.fftfreq(ngrid, d=h)
    k1r = 2.0 * np.pi * np.fft.rfftfreq(ngrid, d=h)
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kz = k1r[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    kcut = np.pi / h
    amp = np.zeros_like(k2)
    ok = (k2 > 0) & (k2 <= kcut * kcut)
    amp[ok] = 1.0 / np.sqrt(k2[ok])  # sqrt(P(k)), P ~ k^-2
    dk = wk * amp
    del wk, amp
    inv_k2 = np.zeros_like(k2)
    inv_k2[ok] = 1.0 / k2[ok]
    shape = (ngrid, ngrid, ngrid)
    disp = []
    for kc in (kx, ky, kz):
        comp = np.fft.irfftn(1j * kc * dk * inv_k2, s=shape, axes=(0, 1, 2))
        disp.append(comp.reshape(-1))
    del dk
    psi = np.stack(disp, axis=1)
    cur = math.sqrt(float(np.mean(np.sum(psi * psi, axis=1))))
    if cur > 0:
        psi *= rms / cur
    idx = np.arange(ngrid, dtype=np.float64)
    qx, qy, qz = np.meshgrid(idx, idx, idx, indexing="ij")
    q = (np.stack([qx.reshape(-1), qy.reshape(-1), qz.reshape(-1)], axis=1) + 0.5) * h
    pos = np.mod(q + psi, L)
    pos[pos >= L] -= L
    return pos


def _powerlaw_counts(rng, total: int, lo: float, hi: float, slope: float) -> np.ndarray:
    """Integer halo particle counts drawn from dN/dN_h ~ N_h^-slope on
    [lo, hi] until they add up to ``total`` (the last one is trimmed)."""
    a = 1.0 - slope
    out = []
    acc = 0
    while acc < total:
        u = rng.random(4096)
        v = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
        c = np.maximum(np.floor(v).astype(np.int64), int(lo))
        cs = np.cumsum(c) + acc
        k = int(np.searchsorted(cs, total, side="left"))
        if k < len(c):
            c = c[: k + 1].copy()
            c[-1] -= int(cs[k] - total)
            out.append(c[c > 0])
            acc = total
        else:
            out.append(c)
            acc = int(cs[-1])
    return np.concatenate(out)


def _nfw_radii(rng, n: int, conc: float, r200: float) -> np.ndarray:
    """Radii of n particles of an NFW halo truncated at r200, by the inverse
    of the enclosed-mass profile mu(x) = ln(1+x) - x/(1+x), x = r/r_s."""
    xs = np.linspace(0.0, conc, 2049)
    mu = np.log1p(xs) - xs / (1.0 + xs)
    u = rng.random(n) * mu[-1]
    x = np.interp(u, mu, xs)
    return x * (r200 / conc)


def _iso_dirs(rng, n: int) -> np.ndarray:
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(1.0 - cz * cz)
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def _halos(rng, nhalo_parts: int, L: float, periodic: bool, cap: float | None) -> np.ndarray:
    hi = 1e5 if cap is None else max(100.0, min(1e5, cap))
    counts = _powerlaw_counts(rng, nhalo_parts, 100.0, hi, 1.9)
    pos = np.empty((nhalo_parts, 3), dtype=np.float64)
    at = 0
    for nh in counts:
        nh = int(nh)
        conc = rng.uniform(5.0, 10.0)
        r200 = (3.0 * nh / (800.0 * np.pi)) ** (1.0 / 3.0)
        centre = rng.random(3) * L
        p = centre + _iso_dirs(rng, nh) * _nfw_radii(rng, nh, conc, r200)[:, None]
        if not periodic:
            # particles that fall outside the (non-periodic) domain are redrawn
            for _ in range(64):
                out = np.any((p < 0.0) | (p >= L), axis=1)
                k = int(out.sum())
                if k == 0:
                    break
                p[out] = centre + _iso_dirs(rng, k) * _nfw_radii(rng, k, conc, r200)[:, None]
            p = np.clip(p, 0.0, np.nextafter(L, 0.0))
        pos[at: at + nh] = p
        at += nh
    return pos


def nfw_share(n: int, L: float, seed: int, skin: float = 3.0, halo_frac: float = 0.7,
              periodic: bool = False, halo_cap: float | None = None) -> Particles:
    """One GPU's share of a clustered volume.

    ``halo_frac`` of the particles sit in NFW halos: halo particle counts
    follow dN/dN_h ~ N_h^-1.9 on [1e2, 1e5] (optionally capped at
    ``halo_cap``), concentrations are uniform in [5, 10], r200 encloses 200
    times the mean density 1, radii follow the NFW enclosed mass inside r200,
    directions are isotropic and centres uniform.  The rest is uniform
    background.  Non-periodic by default with a passive skin of ``skin``
    (particle overloading, Sec. 2.2).
    """
    rng = np.random.default_rng(seed)
    nh = int(round(halo_frac * n))
    ph = _halos(rng, nh, L, periodic, halo_cap)
    pb = rng.random((n - nh, 3)) * L
    pos = np.concatenate([ph, pb], axis=0)
    # shuffle so that the input order carries no spatial structure
    pos = pos[rng.permutation(n)]
    return _soa(pos, L, periodic=periodic, skin=(0.0 if periodic else skin))


@dataclasses.dataclass
class BoxSpec:
    n: int
    L: float
    kind: str  # "uniform" | "clustered" | "zeldovich"
    seed: int


def batch_specs(nboxes: int = 64, seed: int = 4, lo: int = 16 ** 3, hi: int = 96 ** 3) -> list[BoxSpec]:
    """Box list for the batched form: particle counts log-uniform in
    [lo, hi], side L = N^(1/3) (density 1), alternating uniform and clustered
    (70 % in halos capped at N/10 particles), periodic."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(lo), np.log(hi), nboxes)).astype(np.int64)
    specs = []
    for b, nb in enumerate(ns):
        kind = "uniform" if b % 2 == 0 else "clustered"
        side = float(np.float32(float(nb) ** (1.0 / 3.0)))  # exact in float32
        specs.append(BoxSpec(int(nb), side, kind, int(seed * 1000 + b)))
    return specs


def make_box(spec: BoxSpec) -> Particles:
    if spec.kind == "uniform":
        return uniform(spec.n, spec.L, spec.seed)
    if spec.kind == "zeldovich":
        ng = int(round(spec.n ** (1.0 / 3.0)))
        return zeldovich(ng, spec.L, spec.seed)
    return nfw_share(spec.n, spec.L, spec.seed, periodic=True, halo_cap=spec.n / 10.0)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds from trace start
    ngrid: int      # Zel'dovich lattice side: N = ngrid^3, L = ngrid
    seed: int
    steps: int


def serving_trace(nreq: int = 2000, rate: float = 200.0, seed: int = 5,
                  ng_lo: int = 24, ng_hi: int = 128, steps: int = 10) -> list[Request]:
    """Poisson arrivals at ``rate`` per second; N log-uniform in
    [ng_lo^3, ng_hi^3] rounded to a cube ngrid^3; each request asks for
    ``steps`` stream-kick-stream steps of its own Zel'dovich box."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, nreq)
    t = np.cumsum(gaps) - gaps[0]
    logn = rng.uniform(np.log(ng_lo ** 3), np.log(ng_hi ** 3), nreq)
    ng = np.clip(np.round(np.exp(logn / 3.0)).astype(np.int64), ng_lo, ng_hi)
    return [Request(i, float(t[i]), int(ng[i]), int(seed * 100000 + i), steps) for i in range(nreq)]


@functools.lru_cache(maxsize=2)
def config(name: str) -> Particles:
    """The standard single-box workloads by name (cached: callers must not
    modify the returned arrays)."""
    if name == "uniform32":
        return uniform(32 ** 3, 32.0, 1)
    if name == "zeldovich128":
        return zeldovich(128, 128.0, 2)
    if name == "nfw256":
        return nfw_share(256 ** 3, 256.0, 3, skin=3.0)
    raise KeyError(name)


@dataclasses.dataclass
class PairSet:
    """One unit-mass source (index 0) and massless test particles around it
    in a periodic cube of side L: float32 positions, masses, and the FP64
    separation r and unit direction u (source -> test) of each test particle
    as the float32 positions realise them (minimum image)."""

    pos: np.ndarray   # (1 + ntest, 3) float32
    m: np.ndarray     # (1 + ntest,) float32: 1, 0, 0, ...
    r: np.ndarray     # (ntest,) float64
    u: np.ndarray     # (ntest, 3) float64
    L: float


def pm_test_pairs(nsrc: int, ntest: int, L: float, r_max: float, seed: int,
                  r_lo: float = 0.02) -> list:
    """Seeded test-pair sets for measuring the filtered grid force (the
    experiment of Sec. 2.3): each set has a source at a uniformly random
    position and ntest massless particles at separations uniform in
    [r_lo, r_max] with isotropic directions."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsrc):
        c = rng.random(3) * L
        r = rng.uniform(r_lo, r_max, ntest)
        u = rng.normal(size=(ntest, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        pos = np.mod(np.vstack([c[None, :], c[None, :] + r[:, None] * u]), L).astype(np.float32)
        pos[pos >= np.float32(L)] = 0
        d = pos[1:].astype(np.float64) - pos[0].astype(np.float64)
        d -= L * np.round(d / L)
        rr = np.linalg.norm(d, axis=1)
        m = np.zeros(ntest + 1, np.float32)
        m[0] = 1.0
        out.append(PairSet(pos, m, rr, d / rr[:, None], float(L)))
    return out
