"""Pins for oracle.certify and the oracle's C/OpenMP product (CPU only).

The certificate is checked against spectra known independently of it:
closed forms of lattices (with the exact eigenvectors for the subspace angle)
and dense symmetric-definite solves of small weighted and power-law graphs.
A block edge placed inside a degenerate eigenvalue pair must give no
certificate at all (delta <= 0).
"""
import numpy as np
import pytest
import scipy.linalg

import graphgen
from oracle import certify, eigen, laplacian as lap
from tests import closed_forms as cf


def _rounding_slack(theta_max, norm_l):
    # the bounds hold in exact arithmetic; FP64 evaluation of the Ritz values
    # and of the dense reference adds a few ulps of ||L||
    return 64 * np.finfo(float).eps * max(norm_l, theta_max)


def test_omp_product_equals_difference_form():
    g = graphgen.config_graph("brick96lr", scale_down=8)       # 12^3 weighted + long range
    X = np.random.default_rng(3).standard_normal((g.n, 5))
    a = lap.apply(g.rowptr, g.col, g.w, X)
    for threads in (1, 3, 8):
        b = lap.apply_omp(g.rowptr, g.col, g.w, X, threads=threads)
        # same terms in the same CSR order: identical, whatever the threads
        assert np.array_equal(a, b)
    # L 1 = 0 exactly (difference form)
    assert not lap.apply_omp(g.rowptr, g.col, g.w, np.ones((g.n, 2))).any()


def test_omp_product_closed_form_eigenvector():
    n, (u, v) = graphgen.grid3d_7pt(9, 7, 5)
    g = graphgen.csr_from_edges(n, u, v)
    x = cf.grid_eigvec((5, 7, 9), (3, 1, 2))          # x fastest in the numbering
    lam = cf.path_eigval(9, 2) + cf.path_eigval(7, 1) + cf.path_eigval(5, 3)
    y = lap.apply_omp(g.rowptr, g.col, None, x)
    assert np.allclose(y, lam * x, atol=1e-13)


def test_degrees_fast_close_to_exact():
    g = graphgen.config_graph("king512", scale_down=16)
    a = lap.degrees(g.rowptr, g.col, g.w)
    b = lap.degrees_fast(g.rowptr, g.col, g.w)
    assert np.allclose(a, b, rtol=4 * np.finfo(float).eps, atol=0)


@pytest.mark.parametrize("prec", ["jacobi", "chebyshev"])
def test_certified_grid_closed_form(prec):
    """2D 5-point 24 x 20 grid: the 3 smallest (0 and the (1,0), (0,1) modes)
    are separated from the (1,1)/(2,0) modes; eigenvalues and the invariant
    subspace against the closed form."""
    sx, sy = 24, 20
    n, (u, v) = graphgen.grid2d_5pt(sx, sy)
    g = graphgen.csr_from_edges(n, u, v)
    r = certify.certified_eigenpairs(g.rowptr, g.col, g.w, lap.COMBINATORIAL, 3,
                                     guards=3, prec=prec, seed=11)
    exact = cf.grid_eigvals((sy, sx), 6)
    slack = _rounding_slack(exact[-1], 8.0)
    th = r["theta"][:3]
    assert np.all(th + slack >= exact[:3])                            # Courant-Fischer
    assert np.all(th - r["eig_bound"] - slack <= exact[:3])           # quadratic bound
    assert r["lam_d_lo"] <= exact[3] + slack                          # lambda_d lower bound
    E = np.stack([cf.grid_eigvec((sy, sx), k) for k in [(0, 0), (0, 1), (1, 0)]], axis=1)
    sin = eigen.subspace_sin(r["vectors"], E, np.ones(n))
    assert sin <= r["sin_bound"] + 1e-12
    assert r["sin_bound"] < 1e-6


def test_certified_rmat_generalized_vs_dense():
    """R-MAT scale 11 (LCC), generalized pencil: the certified values bracket
    the dense solve, and the true subspace angle is under the bound."""
    g = graphgen.rmat_graph(11, seed=1)
    L, d = lap.dense(g.rowptr, g.col, g.w)
    lam, V = scipy.linalg.eigh(L, np.diag(d))
    r = certify.certified_eigenpairs(g.rowptr, g.col, g.w, lap.GENERALIZED, 5, seed=5)
    slack = _rounding_slack(2.0, 2.0)
    th = r["theta"][:5]
    assert np.all(th + slack >= lam[:5])
    assert np.all(th - r["eig_bound"] - slack <= lam[:5])
    assert r["lam_d_lo"] <= lam[5] + slack
    sin = eigen.subspace_sin(r["vectors"], V[:, :5], d)
    assert sin <= r["sin_bound"] + 1e-9
    # the guard Ritz values are upper bounds of the next eigenvalues
    assert np.all(r["theta"][5:] + slack >= lam[5:9])


def test_certified_weighted_mesh_vs_dense():
    """27-point 7^3 brick + 1 % long-range edges, weights U[0.5, 1.5):
    combinatorial pencil against the dense solve, block of 4."""
    g = graphgen.config_graph("brick96lr", scale_down=14)
    L, d = lap.dense(g.rowptr, g.col, g.w)
    lam, V = np.linalg.eigh(L)
    r = certify.certified_eigenpairs(g.rowptr, g.col, g.w, lap.COMBINATORIAL, 4, seed=2)
    slack = _rounding_slack(lam[8], np.abs(lam).max())
    assert np.all(r["theta"][:4] + slack >= lam[:4])
    assert np.all(r["theta"][:4] - r["eig_bound"] - slack <= lam[:4])
    sin = eigen.subspace_sin(r["vectors"], V[:, :4], np.ones(g.n))
    assert sin <= r["sin_bound"] + 1e-9


def test_no_certificate_inside_a_degenerate_pair():
    """d = 2 on a square grid cuts the degenerate (1,0)/(0,1) pair: the wanted
    subspace is not determined, and the certificate must say so."""
    n, (u, v) = graphgen.grid2d_5pt(16, 16)
    g = graphgen.csr_from_edges(n, u, v)
    r = certify.certified_eigenpairs(g.rowptr, g.col, g.w, lap.COMBINATORIAL, 2,
                                     guards=3, seed=4)
    assert r["delta"] <= 1e-8
    assert r["sin_bound"] == np.inf or r["sin_bound"] > 1.0


def test_certify_block_of_a_perturbed_basis():
    """certify_block on a basis that is not converged: the bound still holds
    (it is a bound for any basis), here against the closed form."""
    sx, sy = 16, 12
    n, (u, v) = graphgen.grid2d_5pt(sx, sy)
    g = graphgen.csr_from_edges(n, u, v)
    E = np.stack([cf.grid_eigvec((sy, sx), k) for k in [(0, 0), (0, 1), (1, 0)]], axis=1)
    X = E + 1e-4 * np.random.default_rng(0).standard_normal(E.shape)
    op = lap.operator(g.rowptr, g.col, g.w, lap.COMBINATORIAL, fast=True)
    exact = cf.grid_eigvals((sy, sx), 4)
    c = certify.certify_block(op, np.ones(n), X, exact[3])
    sin = eigen.subspace_sin(X, E, np.ones(n))
    assert 1e-6 < sin <= c["sin_bound"]
    assert np.all(c["theta"] >= exact[:3] - 1e-14)
    assert np.all(c["theta"] - c["eig_bound"] <= exact[:3] + 1e-14)
