"""Partition quality (oracle; test infrastructure only).

Paper: Sec. 3.1 (Graph Partitioning Problem).  An edge is cut when its end
vertices lie in different parts; the cutsize is the total cost of the cut
edges (Eq. 1).  The part weight W_k is the sum of the weights of its vertices
and the average part weight is W_avg = sum_k W_k / K.  The imbalance reported
is max_k W_k / W_avg (Sec. 6.3.6, nvGRAPH comparison).

Reading taken (Eq. 1 vs the tables of Sec. 6): Eq. 1 counts each undirected
edge once; the experiment tables report twice the number of cut edges.  Both
are returned.
"""
from __future__ import annotations

import math

import numpy as np

from .laplacian import row_index


def cutsize(rowptr, col, w, part):
    """Eq. 1, summed exactly.

    Each undirected edge {i, j} is stored twice in the symmetric CSR; it is
    counted once (from the entry with i < j).  Unit weights give an integer;
    float weights are summed with math.fsum, which returns the correctly
    rounded value of the exact sum.  Returns (cut, cut2x) with cut2x = 2*cut
    (the paper's reporting convention).
    """
    part = np.asarray(part, dtype=np.int64)
    r = row_index(rowptr)
    c = np.asarray(col, dtype=np.int64)
    sel = (r < c) & (part[r] != part[c])
    if w is None:
        cut = int(np.count_nonzero(sel))
        return float(cut), float(2 * cut)
    vals = np.asarray(w, dtype=np.float64)[sel]
    cut = math.fsum(vals.tolist())
    return cut, 2.0 * cut


def part_weights(part, K, vwgt=None):
    """W_k = sum of vertex weights in part k (unit weights if vwgt is None)."""
    part = np.asarray(part, dtype=np.int64)
    if part.size and (part.min() < 0 or part.max() >= K):
        raise ValueError("part id out of range")
    wts = np.ones(part.size, dtype=np.int64) if vwgt is None else np.asarray(vwgt, dtype=np.int64)
    out = np.zeros(K, dtype=np.int64)
    np.add.at(out, part, wts)
    return out


def imbalance(part, K, vwgt=None):
    """max_k W_k / W_avg = max_k W_k * K / sum_k W_k, with a single rounding."""
    pw = part_weights(part, K, vwgt)
    total = int(pw.sum())
    if total == 0:
        return 1.0
    return float(int(pw.max()) * K) / float(total)
