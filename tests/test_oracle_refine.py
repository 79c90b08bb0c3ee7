"""Pins for oracle.refine (CPU only): brute-force cut differences from the
edge list, hand-worked passes, the balance rule and exactness."""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
from oracle import quality, refine


def _graph(n, p, seed, weighted):
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    u, v = iu[keep], ju[keep]
    w = rng.uniform(0.5, 1.5, u.size) if weighted else None
    return u, v, w, graphgen.csr_from_edges(n, u, v, w)


def _brute_cut(u, v, w, part):
    """Eq. 1 straight from the undirected edge list, in exact arithmetic."""
    tot = 0
    for e in range(u.size):
        if part[u[e]] != part[v[e]]:
            tot += 1 if w is None else Fraction(float(w[e]))
    return tot


def test_capacity():
    assert refine.capacity(6, 2, 0.01) == 3         # 3.03 -> 3
    assert refine.capacity(6, 2, 0.5) == 4          # 4.5 -> 4
    assert refine.capacity(100, 4, 0.0) == 24       # strict: W_k < 25
    assert refine.capacity(64, 2, 0.05) == 33       # 33.6 -> 33
    assert refine.capacity(2 ** 20, 64, 0.01) == 16547


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("seed,K", [(1, 2), (2, 3), (3, 5)])
def test_gains_are_best_single_move_cut_decrease(weighted, seed, K):
    u, v, w, g = _graph(30, 0.15, seed, weighted)
    part = np.random.default_rng(seed + 10).integers(0, K, g.n)
    tgt, gain = refine.gains(g.rowptr, g.col, g.w, part.tolist())
    base = _brute_cut(u, v, w, part)
    for x in range(g.n):
        dec = {}
        for p in range(K):
            if p == part[x]:
                continue
            q = part.copy()
            q[x] = p
            dec[p] = base - _brute_cut(u, v, w, q)
        best = max(dec.values())
        if best > 0:
            assert gain[x] == best
            assert tgt[x] == min(p for p in dec if dec[p] == best)
        else:
            assert tgt[x] == -1 and gain[x] == 0


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("seed,K", [(4, 2), (5, 4)])
def test_movers_gain_after_higher_ranked_moves(weighted, seed, K):
    """g'(v) is the cut decrease of moving v once every candidate ranked
    before it has taken its target."""
    u, v, w, g = _graph(40, 0.12, seed, weighted)
    part = np.random.default_rng(seed).integers(0, K, g.n)
    tgt, gain = refine.gains(g.rowptr, g.col, g.w, part.tolist())
    cands = [x for x in range(g.n) if tgt[x] >= 0]
    assert len(cands) > 5
    order = sorted(cands, key=lambda x: (-gain[x], x))
    mv = set(refine.movers(g.rowptr, g.col, g.w, part.tolist(), tgt, gain))
    for i, x in enumerate(order):
        q = part.copy()
        for y in order[:i]:
            q[y] = tgt[y]
        before = _brute_cut(u, v, w, q)
        q[x] = tgt[x]
        assert (x in mv) == (before - _brute_cut(u, v, w, q) > 0)


def test_hand_path_pass():
    # path 0-1-2-3-4-5, parts [0,0,1,0,1,1]: 2 and 3 both have gain 2 (2 is
    # ranked first); with 2 moved to part 0, vertex 3 would gain 0, so only 2
    # moves, when the balance allows part 0 to reach 4 vertices
    n = 6
    g = graphgen.csr_from_edges(n, np.arange(5), np.arange(1, 6))
    part = [0, 0, 1, 0, 1, 1]
    tgt, gain = refine.gains(g.rowptr, g.col, None, part)
    assert tgt == [-1, -1, 0, 1, -1, -1] and gain == [0, 0, 2, 2, 0, 0]
    assert refine.movers(g.rowptr, g.col, None, part, tgt, gain) == [2]
    new, moved = refine.refine_pass(g.rowptr, g.col, None, part, 2, eps=0.5)
    assert new.tolist() == [0, 0, 0, 0, 1, 1] and moved == 1
    # eps = 1 %: capacity 3, part 0 already holds 3
    new, moved = refine.refine_pass(g.rowptr, g.col, None, part, 2, eps=0.01)
    assert new.tolist() == part and moved == 0
    out, kept, moves = refine.refine(g.rowptr, g.col, None, part, 2, eps=0.5)
    assert out.tolist() == [0, 0, 0, 0, 1, 1] and kept == 1 and moves == 1
    assert quality.cutsize(g.rowptr, g.col, None, out)[0] == 1.0


def test_grid_bumps_are_straightened():
    # 8x8 grid split at x = 4 with two bumps: (x=4, y=3) in part 0 and
    # (x=3, y=5) in part 1; both return (gain 2 each, not adjacent)
    n, (u, v) = graphgen.grid2d_5pt(8, 8)
    g = graphgen.csr_from_edges(n, u, v)
    x = np.arange(n) % 8
    y = np.arange(n) // 8
    part = (x >= 4).astype(np.int32)
    part[3 * 8 + 4] = 0
    part[5 * 8 + 3] = 1
    assert quality.cutsize(g.rowptr, g.col, None, part)[0] == 12.0
    out, kept, moves = refine.refine(g.rowptr, g.col, None, part, 2, eps=0.05)
    assert np.array_equal(out, (x >= 4).astype(np.int32))
    assert quality.cutsize(g.rowptr, g.col, None, out)[0] == 8.0
    assert kept == 1 and moves == 2


def test_balance_rule_prefix_in_vertex_order():
    # star: centre 0 and leaves 7..13 in part 0, leaves 1..6 in part 1; each
    # leaf of part 1 gains 1 by joining part 0 (the centre gains nothing), and
    # the capacity admits only a prefix of them in vertex order
    n = 14
    g = graphgen.csr_from_edges(n, np.zeros(13, dtype=int), np.arange(1, 14))
    part = np.array([0] + [1] * 6 + [0] * 7)
    vw = np.array([1, 1, 2, 1, 1, 1, 1] + [1] * 7)
    # W = 15, K = 2, eps = 0.3 -> capacity ceil(9.75) - 1 = 9; W_0 = 8
    assert refine.capacity(15, 2, 0.3) == 9
    tgt, gain = refine.gains(g.rowptr, g.col, None, part.tolist())
    assert refine.movers(g.rowptr, g.col, None, part.tolist(), tgt, gain) == [1, 2, 3, 4, 5, 6]
    new, moved = refine.refine_pass(g.rowptr, g.col, None, part, 2, vwgt=vw, eps=0.3)
    # movers in id order: 8 + 1 = 9 <= 9 (1 in), + 2 = 11 > 9 (2 out),
    # + 1 = 12 > 9 (3 out), ...: only vertex 1 moves, although vertex 3
    # alone would still fit
    expect = part.copy()
    expect[1] = 0
    assert new.tolist() == expect.tolist() and moved == 1


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("seed,K", [(6, 2), (7, 3), (8, 6)])
def test_refine_invariants(weighted, seed, K):
    u, v, w, g = _graph(60, 0.08, seed, weighted)
    rng = np.random.default_rng(seed)
    part = rng.integers(0, K, g.n).astype(np.int32)
    vw = rng.integers(1, 4, g.n)
    eps = 0.3
    out, kept, moves = refine.refine(g.rowptr, g.col, g.w, part, K, vwgt=vw, eps=eps, passes=6)
    assert _brute_cut(u, v, w, out) <= _brute_cut(u, v, w, part)
    if kept:
        assert _brute_cut(u, v, w, out) < _brute_cut(u, v, w, part)
    cap = refine.capacity(int(vw.sum()), K, eps)
    W0 = np.bincount(part, weights=vw, minlength=K)
    W1 = np.bincount(out, weights=vw, minlength=K)
    # a part never grows past the capacity (parts above it only shrink)
    assert np.all((W1 <= np.maximum(W0, cap)))
    # one pass: the accepted movers into each part are a prefix by id
    new, _ = refine.refine_pass(g.rowptr, g.col, g.w, part, K, vwgt=vw, eps=eps)
    tgt, gain = refine.gains(g.rowptr, g.col, g.w, part.tolist())
    mv = refine.movers(g.rowptr, g.col, g.w, part.tolist(), tgt, gain)
    for p in range(K):
        into = [x for x in mv if tgt[x] == p]
        acc = [x for x in into if new[x] == p]
        assert acc == into[:len(acc)]
        assert W0[p] + vw[acc].sum() <= cap or not acc


def test_exact_tie_and_no_rounding():
    # centre 0 (part 0): edge 1.0 to part 0, edges 1.0, 2^-24, 2^-24 to part 1.
    # Exactly, conn to part 1 exceeds conn to part 0 by 2^-23; a float32 sum
    # in this order rounds it away (1 + 2^-24 -> 1)
    n = 5
    u = np.array([0, 0, 0, 0])
    v = np.array([1, 2, 3, 4])
    w = np.array([1.0, 1.0, 2.0 ** -24, 2.0 ** -24], dtype=np.float32)
    g = graphgen.csr_from_edges(n, u, v, w)
    part = [0, 0, 1, 1, 1]
    tgt, gain = refine.gains(g.rowptr, g.col, g.w, part)
    assert tgt[0] == 1 and gain[0] == Fraction(1, 2 ** 23)
    assert np.float32(np.float32(1.0) + np.float32(2.0 ** -24)) + np.float32(2.0 ** -24) \
        == np.float32(1.0)
    # exact tie: 0.5 + 0.25 against 0.75 is no gain
    w2 = np.array([0.75, 0.5, 0.25], dtype=np.float64)
    g2 = graphgen.csr_from_edges(4, np.array([0, 0, 0]), np.array([1, 2, 3]), w2)
    tgt, gain = refine.gains(g2.rowptr, g2.col, g2.w, [0, 0, 1, 1])
    assert tgt[0] == -1


def test_degree_limit_and_isolated():
    g = graphgen.csr_from_edges(6, np.zeros(4, dtype=int), np.arange(1, 5))   # 5 isolated
    part = [0, 1, 1, 1, 1, 0]
    tgt, _ = refine.gains(g.rowptr, g.col, None, part)
    assert tgt[0] == 1 and tgt[5] == -1
    tgt, _ = refine.gains(g.rowptr, g.col, None, part, max_deg=3)
    assert tgt[0] == -1
