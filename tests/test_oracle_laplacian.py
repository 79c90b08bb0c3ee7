"""Pins for oracle.laplacian (CPU only)."""
import numpy as np
import pytest

import graphgen
from oracle import laplacian as lap
from tests import closed_forms as cf


def _random_weighted(n=40, p=0.15, seed=3):
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    u, v = iu[keep], ju[keep]
    w = graphgen.uniform_weights(u.size, seed + 1, dtype=np.float64)
    return graphgen.csr_from_edges(n, u, v, w), (u, v, w)


def test_constant_vector_maps_to_exact_zero():
    g, _ = _random_weighted()
    Y = lap.apply(g.rowptr, g.col, g.w, np.full((g.n, 3), 0.7312))
    assert np.all(Y == 0.0)


def test_quadratic_form_equals_edge_sum_bruteforce():
    g, (u, v, w) = _random_weighted()
    x = np.random.default_rng(0).standard_normal(g.n)
    edge_sum = 0.0
    for a, b, c in zip(u, v, w):           # every undirected edge once
        edge_sum += c * (x[a] - x[b]) ** 2
    assert x @ lap.apply(g.rowptr, g.col, g.w, x) == pytest.approx(edge_sum, rel=1e-13)


def test_apply_matches_entrywise_dense_D_minus_A_and_is_symmetric():
    g, _ = _random_weighted()
    L, d = lap.dense(g.rowptr, g.col, g.w)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((g.n, 4))
    Y = lap.apply(g.rowptr, g.col, g.w, X)
    assert np.allclose(Y, L @ X, rtol=0, atol=1e-12)
    assert np.allclose(L, L.T)
    assert np.allclose(d, lap.degrees(g.rowptr, g.col, g.w))
    y = rng.standard_normal(g.n)
    assert y @ Y[:, 0] == pytest.approx(X[:, 0] @ lap.apply(g.rowptr, g.col, g.w, y), rel=1e-12)


def test_sparse_form_matches_difference_form():
    g, _ = _random_weighted()
    X = np.random.default_rng(2).standard_normal((g.n, 3))
    a = lap.apply(g.rowptr, g.col, g.w, X)
    b = lap.apply_sparse(g.rowptr, g.col, g.w, X)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(X).max() * 10)


def test_degrees_bruteforce():
    g, (u, v, w) = _random_weighted()
    d = np.zeros(g.n)
    for a, b, c in zip(u, v, w):
        d[a] += c
        d[b] += c
    assert np.allclose(lap.degrees(g.rowptr, g.col, g.w), d, rtol=1e-14)


def test_degrees_are_exactly_rounded():
    # vertex 1 has weights 2^53, 1, 1: a left-to-right float sum gives 2^53
    g = graphgen.csr_from_edges(4, np.array([0, 1, 1]), np.array([1, 2, 3]),
                                np.array([2.0 ** 53, 1.0, 1.0]))
    assert lap.degrees(g.rowptr, g.col, g.w)[1] == 2.0 ** 53 + 2.0


@pytest.mark.parametrize("n", [7, 32])
def test_path_closed_form_eigenvectors(n):
    u = np.arange(n - 1)
    g = graphgen.csr_from_edges(n, u, u + 1)
    for k in range(n):
        v = cf.path_eigvec(n, k)
        lam = cf.path_eigval(n, k)
        r = lap.apply(g.rowptr, g.col, None, v) - lam * v
        assert np.abs(r).max() < 1e-12


def test_grid_closed_form_eigenvector():
    n, (u, v) = graphgen.grid3d_7pt(6, 5, 4)
    g = graphgen.csr_from_edges(n, u, v)
    shape = (4, 5, 6)            # C order: z, y, x
    for ks in [(1, 0, 0), (0, 2, 1), (3, 4, 5)]:
        x = cf.grid_eigvec(shape, ks)
        lam = sum(cf.path_eigval(s, k) for s, k in zip(shape, ks))
        assert np.abs(lap.apply(g.rowptr, g.col, None, x) - lam * x).max() < 1e-12


def test_regular_classification():
    n, (u, v) = graphgen.grid2d_5pt(10, 10)
    assert lap.is_regular(graphgen.csr_from_edges(n, u, v).rowptr)
    # star on 30 vertices: max degree 29, average 58/30 -> ratio 15 > 10
    star = graphgen.csr_from_edges(30, np.zeros(29, int), np.arange(1, 30))
    assert not lap.is_regular(star.rowptr)
    # star on 20 vertices: ratio 19 / (38/20) = 10 -> regular (<= 10)
    star = graphgen.csr_from_edges(20, np.zeros(19, int), np.arange(1, 20))
    assert lap.is_regular(star.rowptr)


def test_residual_norm_hand_example():
    # two vertices joined by an edge of weight 2: L = [[2,-2],[-2,2]], D = 2 I
    g = graphgen.csr_from_edges(2, np.array([0]), np.array([1]), np.array([2.0]))
    X = np.array([[1.0, 1.0], [1.0, 0.0]])
    theta = np.array([0.0, 2.0])
    LX = lap.apply(g.rowptr, g.col, g.w, X)       # [[0, 2], [0, -2]]
    # combinatorial: r_1 = [2,-2] - 2 [1,0] = [0,-2]; ||r|| = 2; scale 2 * ||x|| = 2
    rho = lap.residual_norms(LX, X, theta, np.ones(2))
    assert rho[0] == 0.0 and rho[1] == pytest.approx(1.0)
    # generalized: r_1 = [2,-2] - 2*2*[1,0] = [-2,-2]; ||r||_{D^-1} = sqrt(4/2+4/2) = 2;
    # ||x||_D = sqrt(2); scale = max(2, 2) * sqrt(2)
    rho = lap.residual_norms(LX, X, theta, np.array([2.0, 2.0]))
    assert rho[1] == pytest.approx(2.0 / (2.0 * np.sqrt(2.0)))


# ---- normalized Laplacian L_N = I - D^-1/2 A D^-1/2 (the equation after Eq. 2)

def test_normalized_entrywise_dense_matches_apply():
    g, _ = _random_weighted()
    LN = lap.dense_normalized(g.rowptr, g.col, g.w)
    X = np.random.default_rng(4).standard_normal((g.n, 3))
    assert np.allclose(lap.apply_normalized(g.rowptr, g.col, g.w, X), LN @ X, rtol=0, atol=1e-13)
    assert np.allclose(LN, LN.T, rtol=0, atol=1e-15)
    assert np.allclose(np.diag(LN), 1.0)


def test_normalized_eigenpairs_are_scaled_generalized_ones():
    # L_C x = lambda D x  <=>  L_N (D^1/2 x) = lambda (D^1/2 x): a library
    # generalized eigensolver on the (pinned) dense L_C and D fixes L_N's pairs
    import scipy.linalg
    g, _ = _random_weighted()
    L, d = lap.dense(g.rowptr, g.col, g.w)
    lam, X = scipy.linalg.eigh(L, np.diag(d))
    Y = np.sqrt(d)[:, None] * X
    LY = lap.apply_normalized(g.rowptr, g.col, g.w, Y)
    assert np.abs(LY - Y * lam[None, :]).max() < 1e-11
    assert lam.min() > -1e-12 and lam.max() <= 2.0 + 1e-12


def test_normalized_trivial_vector_and_regular_cycle_closed_form():
    n = 12
    u = np.arange(n)
    v = (u + 1) % n
    g = graphgen.csr_from_edges(n, u, v)
    # 2-regular: L_N = L_C / 2, eigenpairs (1 - cos(2 pi k / n), cos(2 pi k i / n))
    i = np.arange(n)
    for k in range(n // 2 + 1):
        x = np.cos(2 * np.pi * k * i / n)
        y = lap.apply_normalized(g.rowptr, g.col, None, x)
        assert np.abs(y - (1 - np.cos(2 * np.pi * k / n)) * x).max() < 1e-13
    # even cycle is bipartite: eigenvalue 2 on the alternating vector
    alt = (-1.0) ** i
    assert np.abs(lap.apply_normalized(g.rowptr, g.col, None, alt) - 2 * alt).max() < 1e-14
    # D^1/2 1 is in the kernel on an irregular weighted graph
    gw, _ = _random_weighted()
    s = np.sqrt(lap.degrees(gw.rowptr, gw.col, gw.w))
    assert np.abs(lap.apply_normalized(gw.rowptr, gw.col, gw.w, s)).max() < 1e-13 * s.max()


def test_normalized_rejects_isolated_vertex():
    g = graphgen.csr_from_edges(3, np.array([0]), np.array([1]))
    with pytest.raises(ValueError):
        lap.apply_normalized(g.rowptr, g.col, None, np.ones(3))


def test_normalized_sparse_form_matches_definition():
    g, _ = _random_weighted()
    X = np.random.default_rng(5).standard_normal((g.n, 3))
    a = lap.apply_normalized(g.rowptr, g.col, g.w, X)
    b = lap.apply_normalized_sparse(g.rowptr, g.col, g.w, X)
    assert np.allclose(a, b, rtol=0, atol=1e-13 * np.abs(X).max() * 10)
