"""Input generator checks (CPU only).

The paper's Table of test graphs lists "#edges" = nnz(A + A^T + I) of the
symmetrised matrix (Sec. 6.1); the 27-point Brick3D rows and the 5-point
ecology1 row (a 1000 x 1000 grid) are reproduced exactly by the generators.
"""
import numpy as np
import pytest

import graphgen


def _check_csr(g):
    rp, col = g.rowptr, g.col
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0)
    r = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(r != col)                                   # no self-loops
    key = r.astype(np.int64) * g.n + col
    assert np.all(np.diff(key) > 0)                           # sorted, no dups
    rkey = np.sort(col.astype(np.int64) * g.n + r)
    assert np.array_equal(key, rkey)                          # symmetric pattern
    if g.w is not None:
        mate = np.searchsorted(key, col.astype(np.int64) * g.n + r)
        assert np.array_equal(g.w, g.w[mate])                 # symmetric weights


def test_table_counts_brick3d_100_and_ecology1():
    n, (u, v) = graphgen.brick27(100, 100, 100)
    assert 2 * u.size + n == 26_463_592
    n, (u, v) = graphgen.grid2d_5pt(1000, 1000)
    assert 2 * u.size + n == 4_996_000


def test_workload_sizes():
    g = graphgen.config_graph("grid64")
    assert (g.n, g.n_edges) == (4096, 8064)
    _check_csr(g)
    n, (u, v) = graphgen.grid3d_7pt(128, 128, 128)
    assert (n, u.size) == (2_097_152, 6_242_304)
    n, (u, v) = graphgen.brick27(96, 96, 96)
    assert u.size == 11_254_460


def test_brick_with_long_range_edges():
    g = graphgen.config_graph("brick96lr", scale_down=8)      # 12^3
    n, (u, v) = graphgen.brick27(12, 12, 12)
    assert g.n_edges == u.size + int(round(0.01 * u.size))
    assert g.w.dtype == np.float32 and g.w.min() >= 0.5 and g.w.max() < 1.5
    _check_csr(g)


def test_rmat_recipe_small():
    g1 = graphgen.config_graph("rmat22", scale_down=1 << 10)   # scale 12
    g2 = graphgen.config_graph("rmat22", scale_down=1 << 10)
    assert np.array_equal(g1.col, g2.col)                      # seeded
    _check_csr(g1)
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    A = sp.csr_matrix((np.ones(g1.nnz), g1.col, g1.rowptr), shape=(g1.n, g1.n))
    assert csg.connected_components(A, directed=False)[0] == 1
    deg = np.diff(g1.rowptr)
    assert deg.max() > 10 * deg.mean()                        # irregular


def test_weighted_king_graph():
    g = graphgen.config_graph("king512", scale_down=32)        # 16 x 16
    assert g.n == 256 and g.w.dtype == np.float64
    assert g.n_edges == 2 * 15 * 16 + 2 * 15 * 15
    _check_csr(g)


def test_brick27_csr_equals_edge_list_build():
    n, (u, v) = graphgen.brick27(6, 5, 4)
    a = graphgen.csr_from_edges(n, u, v)
    b = graphgen.brick27_csr(6, 5, 4)
    assert np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.col, b.col)


def test_brick100_matches_the_paper_edge_count():
    # the paper's Brick3D 100^3 row counts nnz(A + A^T + I) = 26,463,592
    g = graphgen.config_graph("brick100", scale_down=1)
    assert g.n == 1_000_000
    assert int(g.rowptr[-1]) + g.n == 26_463_592


def test_perturb_weights_symmetric_and_bounded():
    n, (u, v) = graphgen.grid2d_9pt(20, 15)
    g = graphgen.csr_from_edges(n, u, v, graphgen.uniform_weights(u.size, 2, dtype=np.float64))
    h = graphgen.perturb_weights(g, 0.01, 3)
    iu = np.repeat(np.arange(n), np.diff(g.rowptr))
    f = h.w / g.w
    assert np.all((f >= 0.99 - 1e-15) & (f < 1.01))
    # the entry (i, j) and its mirror (j, i) carry the same weight
    key = iu * n + g.col
    mirror = g.col * n + iu
    order = np.argsort(key)
    pos = order[np.searchsorted(key[order], mirror)]
    assert np.array_equal(h.w, h.w[pos])
    assert np.unique(np.round(f, 6)).size > 100
    u1 = graphgen.perturb_weights(graphgen.csr_from_edges(n, u, v), 0.05, 1, dtype=np.float32)
    assert u1.w.dtype == np.float32 and abs(u1.w.astype(np.float64) - 1).max() <= 0.05 + 1e-7
