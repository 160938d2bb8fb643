"""ctypes front end of the FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of bench.py, never by the product package.  Inputs are
numpy arrays; float32 particle data is promoted to float64 exactly before it
reaches the C code.  The shared library is compiled on first use (or by
``build()``) with gcc; it shares no source with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ERANGE, ENOMEM = 0, -22, -34, -12


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_grid_dims.argtypes = [P, dbl, P]
        lib.oracle_bin.argtypes = [P, P, P, i64, P, dbl, P, P, P, P]
        lib.oracle_force.argtypes = [P, P, P, P, i64, P, i32, dbl, dbl, dbl, P, P, i64,
                                     P, P, P, P, P, P, P, i32]
        lib.oracle_sks.argtypes = [P, P, P, P, P, P, P, i64, P, dbl, dbl, P, dbl, P, i32]
        lib.oracle_max_threads.argtypes = []
        for f in (lib.oracle_grid_dims, lib.oracle_bin, lib.oracle_force, lib.oracle_sks,
                  lib.oracle_max_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _box(L):
    Lv = np.asarray(L, dtype=np.float64)
    if Lv.ndim == 0:
        Lv = np.full(3, float(Lv))
    return np.ascontiguousarray(Lv)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def grid_dims(L, cell: float):
    nc = np.zeros(3, dtype=np.int32)
    rc = _load().oracle_grid_dims(_p(_box(L)), float(cell), _p(nc))
    if rc:
        raise ValueError("oracle_grid_dims: %d" % rc)
    return nc


def bin(x, y, z, L, cell: float):
    """Returns (offsets[n_cells+1], perm[n], cid[n]) as int32 arrays."""
    Lb = _box(L)
    nc = grid_dims(Lb, cell)
    n = int(np.asarray(x).shape[0])
    xs, ys, zs = _d(x), _d(y), _d(z)
    off = np.zeros(int(nc[0]) * int(nc[1]) * int(nc[2]) + 1, dtype=np.int32)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    cid = np.zeros(max(n, 1), dtype=np.int32)
    bad = np.zeros(1, dtype=np.int64)
    rc = _load().oracle_bin(_p(xs), _p(ys), _p(zs), n, _p(Lb), float(cell), _p(off), _p(perm),
                            _p(cid), _p(bad))
    if rc == ERANGE:
        raise ValueError("position out of [0, L) at index %d" % int(bad[0]))
    if rc:
        raise ValueError("oracle_bin: %d" % rc)
    return off, perm[:n], cid[:n]


def force(x, y, z, m, L, r_max: float, eps: float, poly, periodic: bool = True,
          skin: float = 0.0, targets=None, nthreads: int = 0):
    """Brute-force FP64 short-range accelerations.

    Returns a dict with 'a' (nt, 3), 'S' (nt), 'A' (nt), 'npair' (nt),
    'passive' (nt) for the requested targets (all particles if None)."""
    xs, ys, zs, ms = _d(x), _d(y), _d(z), _d(m)
    n = xs.shape[0]
    Lb = _box(L)
    c = _d(poly)
    assert c.shape == (6,)
    if targets is None:
        tg = None
        nt = n
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tg.shape[0]
    k = max(nt, 1)
    ax, ay, az = np.zeros(k), np.zeros(k), np.zeros(k)
    S, A = np.zeros(k), np.zeros(k)
    npair = np.zeros(k, dtype=np.int64)
    pas = np.zeros(k, dtype=np.int32)
    rc = _load().oracle_force(_p(xs), _p(ys), _p(zs), _p(ms), n, _p(Lb), int(bool(periodic)),
                              float(skin), float(r_max), float(eps), _p(c), _p(tg), nt,
                              _p(ax), _p(ay), _p(az), _p(S), _p(A), _p(npair), _p(pas),
                              int(nthreads))
    if rc:
        raise ValueError("oracle_force: %d" % rc)
    return {"a": np.stack([ax[:nt], ay[:nt], az[:nt]], axis=1), "S": S[:nt], "A": A[:nt],
            "npair": npair[:nt], "passive": pas[:nt].astype(bool)}


def sks(pos, vel, m, L, r_max: float, eps: float, poly, dt: float, nthreads: int = 0):
    """One FP64 stream-kick-stream step; returns (pos, vel, acc) copies."""
    P = [_d(pos[:, d]).copy() for d in range(3)]
    V = [_d(vel[:, d]).copy() for d in range(3)]
    ms = _d(m)
    n = ms.shape[0]
    acc = np.zeros(3 * max(n, 1))
    rc = _load().oracle_sks(_p(P[0]), _p(P[1]), _p(P[2]), _p(V[0]), _p(V[1]), _p(V[2]), _p(ms),
                            n, _p(_box(L)), float(r_max), float(eps), _p(_d(poly)), float(dt),
                            _p(acc), int(nthreads))
    if rc:
        raise ValueError("oracle_sks: %d" % rc)
    return (np.stack(P, axis=1), np.stack(V, axis=1), acc[: 3 * n].reshape(3, n).T.copy())
