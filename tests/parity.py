"""Shared helpers of the GPU parity tests: device upload, tolerance checks.

The tolerances are the ones the design fixes for float32 accelerations
against the FP64 oracle:
  relRMS = sqrt(sum |da|^2 / sum |a_ref|^2) <= 1e-5, and per particle
  |da_i| <= 1e-3 |a_ref,i| + 1e-6 S_i + A_i
where S_i is the sum of absolute pair terms and A_i the absolute weight of
pairs within 2^-18 r_max^2 of the cutoff (which float32 may classify either
way).  Passive particles and particles without partners must be exactly 0.
"""
from __future__ import annotations

import numpy as np
import torch

REL_RMS_TOL = 1e-5


def to_dev(p, dev="cuda:0"):
    return {k: torch.from_numpy(np.ascontiguousarray(getattr(p, k))).to(dev) for k in "xyzm"}


def accel_np(ax, ay, az):
    return torch.stack([ax, ay, az], 1).double().cpu().numpy()


def measure_accel(a_gpu: np.ndarray, ref: dict) -> dict:
    """Error figures only (no assertion)."""
    ar = ref["a"]
    err = np.linalg.norm(a_gpu - ar, axis=1)
    nref = np.linalg.norm(ar, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(nref > 0, err / nref, 0.0)
    return {"rel_rms": float(np.sqrt((err ** 2).sum() / max(float((nref ** 2).sum()), 1e-300))),
            "max_rel": float(rel.max()) if rel.size else 0.0}


def check_accel(a_gpu: np.ndarray, ref: dict, label: str = "") -> dict:
    """Asserts the tolerances; returns the measured error figures."""
    ar = ref["a"]
    err = np.linalg.norm(a_gpu - ar, axis=1)
    nref = np.linalg.norm(ar, axis=1)
    den = float((nref ** 2).sum())
    rel_rms = float(np.sqrt((err ** 2).sum() / den)) if den > 0 else float(np.sqrt((err ** 2).sum()))
    bound = 1e-3 * nref + 1e-6 * ref["S"] + ref["A"]
    bad = np.nonzero(err > bound)[0]
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(nref > 0, err / nref, 0.0)
    stats = {"rel_rms": rel_rms, "max_rel": float(rel.max()) if rel.size else 0.0,
             "n": int(ar.shape[0]), "n_bound_fail": int(bad.size)}
    assert rel_rms <= REL_RMS_TOL, "%s relRMS %.3e > %.0e" % (label, rel_rms, REL_RMS_TOL)
    assert bad.size == 0, "%s per-particle bound violated at %s (err %s bound %s)" % (
        label, bad[:5], err[bad[:5]], bound[bad[:5]])
    zero = ref["passive"] | (ref["npair"] == 0) & (ref["A"] == 0)
    assert np.all(a_gpu[zero] == 0.0), "%s passive / isolated particles must be exactly 0" % label
    return stats


def kick_accel_ref(pos64, vel, m, L, targets, r_max, eps, poly, dt):
    """FP64 reference for the kick of one stream-kick-stream step (Sec. 2.5)
    of sampled particles of a periodic box: every particle streams by
    v dt/2 (wrapped into [0, L)), then the oracle's force at those positions
    for `targets`.  Returns the oracle's result dict at the streamed
    positions (the acceleration the step kicks with)."""
    from oracle import oracle as O
    p = np.asarray(pos64, np.float64) + 0.5 * dt * np.asarray(vel, np.float64)
    p -= L * np.floor(p / L)
    p[p >= L] -= L
    return O.force(p[:, 0], p[:, 1], p[:, 2], m, L, r_max, eps, np.asarray(poly, np.float64),
                   targets=targets)


def position_slack(npair, m_max, h, eps):
    """Largest change of a target's acceleration when every coordinate of its
    pairs moves by at most u = ulp(h)/2 (the float32 rounding of a split
    offset in [0, h)): per pair |d(m f(s) d)/dd| <= m (|f| + 2 |f'| s) <=
    m (4 (s + eps)^-3/2 + 1) for the fitted p (|p| + 2 |p'| s < 1 on
    [0, 9]), and |delta d| <= 2 sqrt(3) u."""
    u = 0.5 * float(np.spacing(np.float32(h)))
    return 2.0 * np.sqrt(3.0) * u * m_max * (4.0 * eps ** -1.5 + 1.0) * np.asarray(npair, float)


def check_accel_slack(a_gpu: np.ndarray, ref: dict, slack, label: str = "") -> dict:
    """check_accel with an extra per-particle absolute slack (inputs that
    differ from the oracle's by a bounded rounding)."""
    ar = ref["a"]
    err = np.linalg.norm(a_gpu - ar, axis=1)
    nref = np.linalg.norm(ar, axis=1)
    den = float((nref ** 2).sum())
    rel_rms = float(np.sqrt((err ** 2).sum() / den)) if den > 0 else float(np.sqrt((err ** 2).sum()))
    bound = 1e-3 * nref + 1e-6 * ref["S"] + ref["A"] + slack
    bad = np.nonzero(err > bound)[0]
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(nref > 0, err / nref, 0.0)
    assert rel_rms <= REL_RMS_TOL, "%s relRMS %.3e > %.0e" % (label, rel_rms, REL_RMS_TOL)
    assert bad.size == 0, "%s per-particle bound violated at %s (err %s bound %s)" % (
        label, bad[:5], err[bad[:5]], bound[bad[:5]])
    return {"rel_rms": rel_rms, "max_rel": float(rel.max()) if rel.size else 0.0,
            "n": int(ar.shape[0])}
