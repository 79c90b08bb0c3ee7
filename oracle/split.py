"""Coordinate split of the spectral embedding (oracle; test infrastructure only).

Paper: Algorithm 2 and Sec. 4.  The embedding drops the trivial eigenvector;
vertex i's j-th coordinate is entry i of eigenvector j+1 (1 <= j < d).  The
points are partitioned with multi-jagged (MJ), which recursively multisections
the point set along the dimensions in round-robin order, balancing the total
weight of the sections; cuts in one section need not line up with cuts in
another.

Reading taken (the paper gives no section counts, tie rule or tolerance):
for K = 2^m, every level bisects every current section along one coordinate,
level l using coordinate l mod ncoord (round robin).  Members of a section
are ordered by (coordinate value ascending, vertex id ascending), with -0 and
+0 equal.  The lower child receives the prefix whose weight W_lo minimises
|2 W_lo - W| (W = section weight), the shorter prefix on ties; with unit
weights this is the first floor(c/2) of c members.  Vertex weights must be
positive integers (with zero weights the minimiser is not unique).  Part ids are the branch
bits, most significant first.  Non-power-of-two K is not covered.
"""
from __future__ import annotations

import numpy as np


def is_pow2(K):
    return K >= 1 and (K & (K - 1)) == 0


def split_pow2(coords, K, vwgt=None):
    """Part vector (int32[n]) for K = 2^m from an n x ncoord coordinate array."""
    coords = np.asarray(coords)
    if coords.ndim == 1:
        coords = coords[:, None]
    n, ncoord = coords.shape
    if not is_pow2(K):
        raise ValueError("K must be a power of two")
    if np.isnan(coords).any():
        raise ValueError("NaN coordinate")
    m = K.bit_length() - 1
    if m > 0 and ncoord < 1:
        raise ValueError("need at least one coordinate")
    wts = np.ones(n, dtype=np.int64) if vwgt is None else np.asarray(vwgt, dtype=np.int64)
    if wts.size and wts.min() < 1:
        raise ValueError("vertex weights must be positive integers")
    part = np.zeros(n, dtype=np.int64)
    ids = np.arange(n, dtype=np.int64)
    for level in range(m):
        key = coords[:, level % ncoord].astype(np.float64) + 0.0   # -0 -> +0
        # all sections at once: order by (section, value, id); lexsort sorts
        # by the last key first
        order = np.lexsort((ids, key, part))
        sec = part[order]
        starts = np.flatnonzero(np.concatenate([[True], sec[1:] != sec[:-1]]))
        ends = np.concatenate([starts[1:], [n]])
        cw = np.cumsum(wts[order])                     # running weight over all
        newpart = part * 2
        for a, b in zip(starts, ends):
            base = cw[a - 1] if a > 0 else 0
            wlo = np.concatenate([[0], cw[a:b] - base])  # W_lo(p), p = 0..c
            total = int(wlo[-1])
            dev = np.abs(2 * wlo - total)
            p = int(np.argmin(dev))                    # first minimiser = shortest
            newpart[order[a + p:b]] += 1
        part = newpart
    return part.astype(np.int32)
