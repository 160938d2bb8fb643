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
