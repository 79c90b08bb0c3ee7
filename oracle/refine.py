"""Greedy refinement of a K-way partition (oracle; test infrastructure only).

Paper: Sec. 7 names a greedy improvement step as the way to refine the cut of
the spectral partition (and notes that KL/FM-style refinement is hard to
parallelise on a GPU); Sec. 3.1 calls a partition balanced when every part
weight W_k is below W_avg (1 + eps), and Sec. 6 runs every tool with
eps = 1 %.  Sec. 1 motivates repartitioning in place, on the accelerator.

The paper gives no algorithm, so this module fixes one (reading taken).  One
pass over partition pi, with c_v the vertex weights (1 when absent), w the
edge weights (1 when absent), conn(v, p) the total weight of the edges from v
to part p, and C the balance capacity (`capacity`):

  1. gains: for each vertex v with 1 <= deg(v) <= max_deg and a = pi(v), the
     target t(v) is the part p != a of some neighbour with the largest
     conn(v, p), the smallest p on ties; g(v) = conn(v, t) - conn(v, a).  v is
     a candidate when g(v) > 0.
  2. conflicts: candidates are ranked by (g descending, vertex id
     ascending).  For a candidate v, pi'(u) is t(u) for the candidates u
     ranked before v and pi(u) otherwise;
     g'(v) = sum_{u in N(v)} w_vu ([pi'(u) = t(v)] - [pi'(u) = a]).
     v stays a mover when g'(v) > 0.
  3. balance: for each part p, the movers into p in increasing vertex id;
     mover v is accepted when W_p + (weight of the movers into p with id
     <= v) <= C (departures are not credited).
  4. the accepted movers take their targets.

`refine` repeats passes while the exact cut strictly drops, up to `passes`
passes; a pass that does not lower the cut is discarded and ends the run.

Arithmetic is exact: integers for unit weights, `fractions.Fraction` of each
float weight otherwise, so every comparison is exact and independent of the
order of the additions.  Plain Python loops over vertices and edges: meant for
small graphs.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

MAX_DEG = 2048


def capacity(total_weight, K, eps):
    """Largest integer part weight c with c < (W / K)(1 + eps) (Sec. 3.1).

    Evaluated in IEEE double as written: x = (W / K) * (1 + eps), c = ceil(x) - 1.
    """
    x = (float(total_weight) / K) * (1.0 + eps)
    return int(math.ceil(x)) - 1


def _edge_values(col, w):
    if w is None:
        return [1] * len(col)
    return [Fraction(float(x)) for x in np.asarray(w).tolist()]


def exact_cut(rowptr, col, w, part):
    """Eq. 1 as an exact integer or Fraction (each undirected edge once)."""
    W = _edge_values(col, w)
    rp = np.asarray(rowptr).tolist()
    cl = np.asarray(col).tolist()
    total = 0
    for v in range(len(rp) - 1):
        for k in range(rp[v], rp[v + 1]):
            u = cl[k]
            if u > v and part[u] != part[v]:
                total += W[k]
    return total


def gains(rowptr, col, w, part, max_deg=MAX_DEG):
    """Step 1: (target, gain) per vertex; target -1 and gain 0 for non-candidates."""
    W = _edge_values(col, w)
    rp = np.asarray(rowptr).tolist()
    cl = np.asarray(col).tolist()
    part = [int(p) for p in part]
    n = len(rp) - 1
    tgt = [-1] * n
    gain = [0] * n
    for v in range(n):
        lo, hi = rp[v], rp[v + 1]
        if hi == lo or hi - lo > max_deg:
            continue
        conn = {}
        for k in range(lo, hi):
            p = part[cl[k]]
            conn[p] = conn.get(p, 0) + W[k]
        a = part[v]
        others = [p for p in conn if p != a]
        if not others:
            continue
        t = min(others, key=lambda p: (-conn[p], p))
        g = conn[t] - conn.get(a, 0)
        if g > 0:
            tgt[v] = t
            gain[v] = g
    return tgt, gain


def movers(rowptr, col, w, part, tgt, gain):
    """Step 2: the candidates whose gain stays positive when every candidate
    ranked before them has taken its target."""
    W = _edge_values(col, w)
    rp = np.asarray(rowptr).tolist()
    cl = np.asarray(col).tolist()
    part = [int(p) for p in part]

    def ranked_before(u, v):
        return gain[u] > gain[v] or (gain[u] == gain[v] and u < v)

    out = []
    for v in range(len(rp) - 1):
        if tgt[v] < 0:
            continue
        a, t = part[v], tgt[v]
        g2 = 0
        for k in range(rp[v], rp[v + 1]):
            u = cl[k]
            pu = tgt[u] if (tgt[u] >= 0 and ranked_before(u, v)) else part[u]
            if pu == t:
                g2 += W[k]
            elif pu == a:
                g2 -= W[k]
        if g2 > 0:
            out.append(v)
    return out


def refine_pass(rowptr, col, w, part, K, vwgt=None, eps=0.01, max_deg=MAX_DEG):
    """One pass (steps 1-4): returns (new part vector, number of accepted moves)."""
    part = np.asarray(part, dtype=np.int64)
    n = part.size
    c = np.ones(n, dtype=np.int64) if vwgt is None else np.asarray(vwgt, dtype=np.int64)
    Wp = [int(c[part == k].sum()) for k in range(K)]
    cap = capacity(int(c.sum()), K, eps)
    tgt, gain = gains(rowptr, col, w, part.tolist(), max_deg)
    mv = movers(rowptr, col, w, part.tolist(), tgt, gain)
    arrived = [0] * K
    new = part.copy()
    moved = 0
    for v in sorted(mv):
        t = tgt[v]
        arrived[t] += int(c[v])
        if Wp[t] + arrived[t] <= cap:
            new[v] = t
            moved += 1
    return new.astype(np.int32), moved


def refine(rowptr, col, w, part, K, vwgt=None, eps=0.01, passes=8, max_deg=MAX_DEG):
    """Passes while the exact cut strictly drops (at most `passes`).

    Returns (part, passes kept, total accepted moves of the kept passes)."""
    cur = np.asarray(part, dtype=np.int32).copy()
    cut = exact_cut(rowptr, col, w, cur.tolist())
    kept = 0
    moves = 0
    for _ in range(passes):
        new, moved = refine_pass(rowptr, col, w, cur, K, vwgt, eps, max_deg)
        if moved == 0:
            break
        c2 = exact_cut(rowptr, col, w, new.tolist())
        if not c2 < cut:
            break
        cur, cut = new, c2
        kept += 1
        moves += moved
    return cur, kept, moves
