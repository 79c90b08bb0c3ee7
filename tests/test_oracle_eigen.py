"""Pins for oracle.eigen (CPU only)."""
import numpy as np
import pytest

import graphgen
from oracle import eigen, laplacian as lap, precond
from tests import closed_forms as cf


@pytest.mark.parametrize("K,d", [(1, 1), (2, 2), (3, 2), (4, 3), (16, 5), (24, 5), (64, 7), (256, 9)])
def test_num_eigenvectors_eq4(K, d):
    # K = 4 -> 3 is the paper's worked example; K = 24 -> 5 (4 coordinates)
    assert eigen.num_eigenvectors(K) == d


def test_dense_grid_spectrum_matches_closed_form():
    n, (u, v) = graphgen.grid2d_5pt(12, 9)
    g = graphgen.csr_from_edges(n, u, v)
    L, d = lap.dense(g.rowptr, g.col, g.w)
    lam, V = eigen.smallest_dense(L, np.ones(n), 8)
    assert np.allclose(lam, cf.grid_eigvals((9, 12), 8), rtol=0, atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(8), atol=1e-12)
    # sign convention
    for k in range(8):
        i = np.argmax(np.abs(V[:, k]))
        assert V[i, k] > 0


def test_dense_generalized_on_torus_is_combinatorial_over_degree():
    n, u, v = cf.torus_edges(6, 5)
    g = graphgen.csr_from_edges(n, u, v)
    L, d = lap.dense(g.rowptr, g.col, g.w)
    assert np.all(d == 4)
    lam, V = eigen.smallest_dense(L, d, 6)
    assert np.allclose(lam, cf.torus_eigvals(6, 5)[:6] / 4.0, atol=1e-12)
    assert np.allclose(V.T @ (d[:, None] * V), np.eye(6), atol=1e-12)


def test_rayleigh_ritz_recovers_exact_pairs_from_mixed_basis():
    n, (u, v) = graphgen.grid2d_5pt(8, 8)
    g = graphgen.csr_from_edges(n, u, v)
    exact = np.stack([cf.grid_eigvec((8, 8), ks) for ks in [(0, 0), (1, 0), (0, 1)]], axis=1)
    rng = np.random.default_rng(0)
    S = np.hstack([exact @ rng.standard_normal((3, 3)), rng.standard_normal((n, 2))])
    theta, Y = eigen.rayleigh_ritz(S, lap.apply(g.rowptr, g.col, None, S), np.ones(n), 3)
    assert np.allclose(theta, cf.grid_eigvals((8, 8), 3), atol=1e-12)
    X = S @ Y
    assert np.allclose(X.T @ X, np.eye(3), atol=1e-10)


def _random_weighted(n, p, seed):
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    u, v = iu[keep], ju[keep]
    # a spanning path keeps the graph connected
    u = np.concatenate([u, np.arange(n - 1)])
    v = np.concatenate([v, np.arange(1, n)])
    key = np.unique(np.minimum(u, v) * n + np.maximum(u, v))
    u, v = key // n, key % n
    w = graphgen.uniform_weights(u.size, seed + 7, dtype=np.float64)
    return graphgen.csr_from_edges(n, u, v, w)


@pytest.mark.parametrize("problem", [lap.COMBINATORIAL, lap.GENERALIZED, lap.NORMALIZED])
@pytest.mark.parametrize("pc", ["none", "jacobi", "cheb", "gmres"])
def test_lobpcg_matches_dense_definition(problem, pc):
    g = _random_weighted(120, 0.04, 11)
    L, d = lap.dense(g.rowptr, g.col, g.w)
    bd = lap.bdiag(g.rowptr, g.col, g.w, problem)
    nev = 4
    if problem == lap.NORMALIZED:
        L = lap.dense_normalized(g.rowptr, g.col, g.w)
        diag = np.ones(g.n)
    else:
        diag = d
    lam, V = eigen.smallest_dense(L, bd, nev)
    hi = precond.gershgorin_bound(d, problem)
    dinv = 1.0 / d if problem == lap.GENERALIZED else None
    pcs = {"none": None,
           "jacobi": lambda R: precond.jacobi(R, diag),
           "cheb": lambda R: precond.chebyshev(g.rowptr, g.col, g.w, R, 8, hi / 30, hi, dinv,
                                               problem=problem)}
    if pc == "gmres":
        b = graphgen.normal_block(g.n, 1, 5)[:, 0]
        roots = precond.gmres_poly_roots(g.rowptr, g.col, g.w, problem, b, 8)
        pcs["gmres"] = lambda R: precond.gmres_poly_apply(g.rowptr, g.col, g.w, problem, R, roots)
    X0 = graphgen.normal_block(g.n, nev, 2)
    theta, X, it, rho = eigen.lobpcg(g.rowptr, g.col, g.w, problem, X0, pcs[pc], 1e-9)
    assert rho.max() <= 1e-8
    assert np.allclose(theta, lam, rtol=1e-10, atol=1e-13)
    assert eigen.subspace_sin(X, V, bd) < 1e-7
    assert np.allclose(X.T @ (bd[:, None] * X), np.eye(nev), atol=1e-10)


def test_lobpcg_grid64_matches_closed_form():
    g = graphgen.config_graph("grid64")
    d = lap.degrees(g.rowptr, g.col, g.w)
    X0 = graphgen.normal_block(g.n, 3, 2)
    theta, X, it, rho = eigen.lobpcg(g.rowptr, g.col, None, lap.COMBINATORIAL, X0,
                                     lambda R: precond.jacobi(R, d), 1e-6)
    exact = cf.grid_eigvals((64, 64), 4)
    assert exact[1] == pytest.approx(0.00240908758966, rel=1e-11)
    assert abs(theta[0]) < 1e-12
    assert np.allclose(theta[1:], exact[1:3], rtol=1e-8)
    span = np.stack([cf.grid_eigvec((64, 64), ks) for ks in [(0, 0), (1, 0), (0, 1)]], axis=1)
    assert eigen.subspace_sin(X, span, np.ones(g.n)) < 1e-4
    assert rho.max() <= 1e-6


def test_subspace_sin_small_angle():
    rng = np.random.default_rng(5)
    U = np.linalg.qr(rng.standard_normal((50, 3)))[0]
    E = rng.standard_normal((50, 3))
    E -= U @ (U.T @ E)
    E = np.linalg.qr(E)[0]            # orthonormal, orthogonal to U
    eps = 1e-9
    V = U + eps * E
    assert eigen.subspace_sin(U, V, np.ones(50)) == pytest.approx(eps, rel=1e-4)
