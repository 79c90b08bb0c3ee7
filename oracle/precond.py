"""LOBPCG preconditioners (oracle; test infrastructure only).

Paper: Sec. 5 (Preconditioners in Sphynx); Algorithm 1 applies the
preconditioner as "solve M H = R".

Jacobi (Sec. 5.1).  Reading taken: the text writes M = diag(A)^-1 while
Algorithm 1 solves M H = R; read together literally they would give
H = diag(A) R, which is not a preconditioner.  The standard Jacobi step is
taken instead: H = diag(L)^-1 R, i.e. h_ij = r_ij / d_i, for both the
combinatorial and the generalized problem (diag L_C = D in both).  For the
normalized problem diag(L_N) = I, so Jacobi leaves R unchanged.

Polynomial (Sec. 5.2).  The paper applies a degree-25 polynomial p(L) that
needs only sparse matrix products and notes that Chebyshev polynomials need
estimates of the extreme eigenvalues.  Here the polynomial is the Chebyshev
one: k steps of the Chebyshev iteration for L h = r started from h = 0 on the
interval [lo, hi], which yields h = p(L) r with deg p = k and
    1 - x p(x) = T_{k+1}((c - x)/e) / T_{k+1}(c/e),  c = (hi+lo)/2, e = (hi-lo)/2.
hi is a guaranteed upper bound of the spectrum (Gershgorin: 2 max_i d_i for
L_C, 2 for D^-1 L_C), so p > 0 on the whole spectrum and the preconditioner
is symmetric positive definite.  For the generalized problem the iteration
runs on D^-1 L_C with right-hand side D^-1 r; for the normalized problem on
L_N, whose spectrum lies in [0, 2] (it is similar to D^-1 L_C).
"""
from __future__ import annotations

import numpy as np

from . import laplacian


def jacobi(R, d):
    """H = diag(L)^-1 R with diag(L) = d (weighted degrees)."""
    return np.asarray(R, dtype=np.float64) / np.asarray(d, dtype=np.float64)[:, None]


def chebyshev(rowptr, col, w, R, degree, lo, hi, dinv=None,
              problem=laplacian.COMBINATORIAL):
    """h = p(L) r column-wise by `degree` Chebyshev steps (degree SpMMs).

    With dinv given, solves (D^-1 L) h = D^-1 r instead (generalized problem);
    with problem NORMALIZED the matrix is L_N.
    """
    L = laplacian.operator(rowptr, col, w, problem)
    R = np.asarray(R, dtype=np.float64)
    c = 0.5 * (hi + lo)
    e = 0.5 * (hi - lo)
    sigma = c / e
    scale = (lambda Z: Z) if dinv is None else (lambda Z: dinv[:, None] * Z)
    rhs = scale(R)
    rho_prev = 1.0 / sigma
    h_prev = np.zeros_like(R)
    h = rhs / c                     # first step from h = 0 needs no product
    for _ in range(degree):
        res = rhs - scale(L(h))
        rho = 1.0 / (2.0 * sigma - rho_prev)
        h_next = h + rho * rho_prev * (h - h_prev) + (2.0 * rho / e) * res
        h_prev, h = h, h_next
        rho_prev = rho
    return h


def chebyshev_scalar(x, degree, lo, hi):
    """p(x) from the closed form 1 - x p(x) = T_{k+1}((c-x)/e) / T_{k+1}(c/e)."""
    from numpy.polynomial import chebyshev as C
    c = 0.5 * (hi + lo)
    e = 0.5 * (hi - lo)
    coef = np.zeros(degree + 2)
    coef[-1] = 1.0
    x = np.asarray(x, dtype=np.float64)
    return (1.0 - C.chebval((c - x) / e, coef) / C.chebval(c / e, coef)) / x


def gershgorin_bound(d, problem):
    """Upper bound of the spectrum: 2 max d_i for L_C, 2 for D^-1 L_C and L_N."""
    if problem in (laplacian.GENERALIZED, laplacian.NORMALIZED):
        return 2.0
    return 2.0 * float(np.max(d)) if len(d) else 0.0
