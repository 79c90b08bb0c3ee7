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
bits, most significant first.

General K (`split_mj`): the number of sections per level are the prime
factors of K in non-increasing order (K = 24 -> 3, 2, 2, 2), one level per
factor, coordinates round robin as above.  A level with p sections places,
in every current section, cut j (1 <= j < p) after the prefix whose weight
C minimises |p C - j W|, the shorter prefix on ties; the children are the
members between consecutive cuts, and part ids are the mixed-radix digits,
most significant first.  For p = 2 this is the bisection rule above.
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


def section_counts(K):
    """Sections per level for general K: the prime factors of K, largest first."""
    if K < 1:
        raise ValueError("K must be >= 1")
    f, k, q = [], K, 2
    while q * q <= k:
        while k % q == 0:
            f.append(q)
            k //= q
        q += 1
    if k > 1:
        f.append(k)
    return sorted(f, reverse=True)


def split_mj(coords, K, vwgt=None):
    """Part vector (int32[n]) for any K >= 1 from an n x ncoord coordinate array
    (the multi-jagged reading in the module docstring)."""
    coords = np.asarray(coords)
    if coords.ndim == 1:
        coords = coords[:, None]
    n, ncoord = coords.shape
    if np.isnan(coords).any():
        raise ValueError("NaN coordinate")
    counts = section_counts(K)
    if counts and ncoord < 1:
        raise ValueError("need at least one coordinate")
    wts = np.ones(n, dtype=np.int64) if vwgt is None else np.asarray(vwgt, dtype=np.int64)
    if wts.size and wts.min() < 1:
        raise ValueError("vertex weights must be positive integers")
    part = np.zeros(n, dtype=np.int64)
    ids = np.arange(n, dtype=np.int64)
    for level, p in enumerate(counts):
        key = coords[:, level % ncoord].astype(np.float64) + 0.0   # -0 -> +0
        order = np.lexsort((ids, key, part))
        sec = part[order]
        starts = np.flatnonzero(np.concatenate([[True], sec[1:] != sec[:-1]]))
        ends = np.concatenate([starts[1:], [n]])
        cw = np.cumsum(wts[order])
        newpart = part * p
        for a, b in zip(starts, ends):
            base = cw[a - 1] if a > 0 else 0
            C = np.concatenate([[0], cw[a:b] - base])     # C(P), P = 0..c
            total = int(C[-1])
            cuts = [int(np.argmin(np.abs(p * C - j * total))) for j in range(1, p)]
            bounds = [0] + cuts + [b - a]
            for child in range(p):
                newpart[order[a + bounds[child]:a + bounds[child + 1]]] += child
        part = newpart
    return part.astype(np.int32)
