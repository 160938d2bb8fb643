"""FP64 reference of the RCB-tree leaves (Sec. 2.4, figure of the RCB split;
Sec. 3.1, one tree per fixed bin).

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the CPU baseline of
bench.py may use it; the product never does).

The particles are first sorted into the chaining cells (the fixed bins of
the short-range scale).  Inside each bin a node is split in two by the plane
through its centre of mass perpendicular to the longest side of its
bounding box, recursively, until a node holds at most leaf_max particles.

Readings: the centre of mass is mass-weighted, in FP64 (the geometric mean
when the node's mass is zero); the sides are taken in FP64 from the float32
bounding box and ties go to the lowest axis; a particle goes to the lower
child when its coordinate is strictly below the plane; a node whose bounding
box is a point, whose plane leaves one side empty (possible only with
massless particles), or that sits 32 levels deep, is a leaf whatever its
size.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

MAX_DEPTH = 32


def _split(idx, pos, m, leaf_max, depth, out):
    if idx.size <= leaf_max or depth >= MAX_DEPTH:
        out.append(idx)
        return
    p = pos[idx]
    side = p.max(axis=0) - p.min(axis=0)
    ax = int(np.argmax(side))          # first maximum: lowest axis on ties
    if side[ax] <= 0.0:
        out.append(idx)
        return
    w = m[idx]
    mt = w.sum()
    com = (w * p[:, ax]).sum() / mt if mt > 0 else p[:, ax].mean()
    low = p[:, ax] < com
    if low.all() or not low.any():     # the plane leaves one side empty
        out.append(idx)
        return
    _split(idx[low], pos, m, leaf_max, depth + 1, out)
    _split(idx[~low], pos, m, leaf_max, depth + 1, out)


def leaves(x, y, z, m, L, cell: float, leaf_max: int):
    """List of leaves, each an int array of original particle indices."""
    pos = np.stack([np.asarray(x, np.float32), np.asarray(y, np.float32),
                    np.asarray(z, np.float32)], axis=1).astype(np.float64)
    m = np.asarray(m, dtype=np.float64)
    offsets, perm, _ = O.bin(pos[:, 0], pos[:, 1], pos[:, 2], L, cell)
    out = []
    for c in range(offsets.size - 1):
        idx = perm[offsets[c]:offsets[c + 1]].astype(np.int64)
        if idx.size:
            _split(idx, pos, m, leaf_max, 0, out)
    return out
