"""Pins for oracle.adjoint (CPU only): finite differences of a dense
eigensolve, agreement of the two evaluations, and exact homogeneity identities."""
import numpy as np
import pytest

import graphgen
from oracle import adjoint, eigen, laplacian as lap


def _graph(n, p, seed):
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    u = np.concatenate([iu[keep], np.arange(n - 1)])
    v = np.concatenate([ju[keep], np.arange(1, n)])
    key = np.unique(np.minimum(u, v) * n + np.maximum(u, v))
    u, v = key // n, key % n
    w = graphgen.uniform_weights(u.size, seed + 1, dtype=np.float64)
    return graphgen.csr_from_edges(n, u, v, w)


def _undirected(g):
    r = lap.row_index(g.rowptr)
    return np.flatnonzero(r < g.col)


def _mate(g):
    """Index of the reverse CSR entry of every entry."""
    r = lap.row_index(g.rowptr)
    key = r * g.n + g.col
    rkey = g.col.astype(np.int64) * g.n + r
    return np.searchsorted(key, rkey)


def _loss(g, w, problem, nev, a, C):
    L, d = lap.dense(g.rowptr, g.col, w)
    bd = d if problem == lap.GENERALIZED else np.ones(g.n)
    lam, V = eigen.smallest_dense(L, bd, nev)
    return a @ lam + np.sum(C * V)


@pytest.mark.parametrize("problem", [lap.COMBINATORIAL, lap.GENERALIZED])
def test_dense_gradient_matches_central_differences(problem):
    g = _graph(12, 0.3, 21)
    nev = 4
    rng = np.random.default_rng(2)
    a = rng.standard_normal(nev)
    C = rng.standard_normal((g.n, nev))
    grad, lam, V = adjoint.grad_dense(g.rowptr, g.col, g.w, problem, nev, a, C)
    mate = _mate(g)
    assert np.allclose(grad, grad[mate])           # symmetric per edge
    h = 1e-6
    for e in _undirected(g):
        wp = g.w.copy(); wp[e] += h; wp[mate[e]] += h
        wm = g.w.copy(); wm[e] -= h; wm[mate[e]] -= h
        fd = (_loss(g, wp, problem, nev, a, C) - _loss(g, wm, problem, nev, a, C)) / (2 * h)
        assert fd == pytest.approx(grad[e], rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("problem", [lap.COMBINATORIAL, lap.GENERALIZED])
def test_projected_gradient_matches_dense(problem):
    g = _graph(40, 0.1, 5)
    nev = 5
    rng = np.random.default_rng(3)
    a = rng.standard_normal(nev)
    C = rng.standard_normal((g.n, nev))
    gd, lam, V = adjoint.grad_dense(g.rowptr, g.col, g.w, problem, nev, a, C)
    gp = adjoint.grad_projected(g.rowptr, g.col, g.w, problem, lam, V, a, C)
    assert np.allclose(gp, gd, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("problem", [lap.COMBINATORIAL, lap.GENERALIZED])
def test_homogeneity_identities(problem):
    # lambda(c w) = c lambda(w) (combinatorial) or lambda(w) (generalized);
    # v(c w) = v(w) (combinatorial) or v(w)/sqrt(c) (generalized, D-normalised)
    g = _graph(200, 0.02, 8)
    nev = 4
    L, d = lap.dense(g.rowptr, g.col, g.w)
    bd = d if problem == lap.GENERALIZED else np.ones(g.n)
    lam, V = eigen.smallest_dense(L, bd, nev)
    und = _undirected(g)
    for k in range(1, nev):
        e = np.zeros(nev); e[k] = 1.0
        gr = adjoint.grad_projected(g.rowptr, g.col, g.w, problem, lam, V, e, None)
        expect = lam[k] if problem == lap.COMBINATORIAL else 0.0
        assert g.w[und] @ gr[und] == pytest.approx(expect, abs=1e-12 * max(1.0, lam[k]) + 1e-13)
    C = np.random.default_rng(1).standard_normal((g.n, nev))
    C[:, 0] = 0.0
    gr = adjoint.grad_projected(g.rowptr, g.col, g.w, problem, lam, V, None, C)
    expect = 0.0 if problem == lap.COMBINATORIAL else -0.5 * np.sum(C * V)
    assert g.w[und] @ gr[und] == pytest.approx(expect, rel=1e-8, abs=1e-9)


def _loss_normalized(g, w, nev, a, C):
    LN = lap.dense_normalized(g.rowptr, g.col, w)
    lam, Y = eigen.smallest_dense(LN, np.ones(g.n), nev)
    return a @ lam + np.sum(C * Y)


def test_normalized_dense_gradient_matches_central_differences():
    g = _graph(12, 0.3, 21)
    nev = 4
    rng = np.random.default_rng(4)
    a = rng.standard_normal(nev)
    C = rng.standard_normal((g.n, nev))
    grad, lam, Y = adjoint.grad_dense_normalized(g.rowptr, g.col, g.w, nev, a, C)
    mate = _mate(g)
    assert np.allclose(grad, grad[mate])
    h = 1e-6
    for e in _undirected(g):
        wp = g.w.copy(); wp[e] += h; wp[mate[e]] += h
        wm = g.w.copy(); wm[e] -= h; wm[mate[e]] -= h
        fd = (_loss_normalized(g, wp, nev, a, C) - _loss_normalized(g, wm, nev, a, C)) / (2 * h)
        assert fd == pytest.approx(grad[e], rel=1e-6, abs=1e-8)


def test_normalized_homogeneity_and_generalized_eigenvalue_gradient():
    # L_N(c w) = L_N(w): eigenvalues and unit eigenvectors are degree-0
    # homogeneous, so w . grad = 0 for any loss; the eigenvalues equal the
    # generalized ones, so their gradients agree with the generalized formula
    g = _graph(30, 0.15, 9)
    nev = 4
    und = _undirected(g)
    rng = np.random.default_rng(6)
    a = rng.standard_normal(nev)
    C = rng.standard_normal((g.n, nev))
    grad, lam, Y = adjoint.grad_dense_normalized(g.rowptr, g.col, g.w, nev, a, C)
    assert abs(g.w[und] @ grad[und]) < 1e-9
    gn, _, _ = adjoint.grad_dense_normalized(g.rowptr, g.col, g.w, nev, a, None)
    gg, lam_g, _ = adjoint.grad_dense(g.rowptr, g.col, g.w, lap.GENERALIZED, nev, a, None)
    assert np.allclose(lam, lam_g, atol=1e-12)
    assert np.allclose(gn, gg, rtol=1e-8, atol=1e-11)
