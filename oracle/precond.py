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
              problem=laplacian.COMBINATORIAL, op=None):
    """h = p(L) r column-wise by `degree` Chebyshev steps (degree SpMMs).

    With dinv given, solves (D^-1 L) h = D^-1 r instead (generalized problem);
    with problem NORMALIZED the matrix is L_N.  op: the operator Z -> L Z when
    the caller has it already (large graphs).
    """
    L = laplacian.operator(rowptr, col, w, problem) if op is None else op
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


# ---- GMRES polynomial (Sec. 5.2: the paper's polynomial preconditioner)
#
# The polynomial is the GMRES residual polynomial pi of degree k + 1 of a
# (k+1)-step Krylov process from a start vector b, with p(x) = (1 - pi(x)) / x
# of degree k (the preconditioner M = p(A)).  Its roots are the harmonic Ritz
# values of that Krylov space; for the self-adjoint operators here (L_C, or
# D^-1 L_C in the D-inner product, or L_N) the process is Lanczos in the
# B-inner product and the harmonic Ritz values are the eigenvalues of the
# symmetric-definite pencil (H^T H, H_k) with H the (k+2) x (k+1) projection.
# The roots are applied in modified Leja order (first the largest, then each
# maximising the product of distances to the ones before), through
#   p(A) v = sum_i pi_{i-1}(A) v / theta_i,  pi_i = pi_{i-1} (I - A / theta_i).
# Reading taken (the paper gives no start vector): b is made B-orthogonal to
# the trivial eigenvector first, so the polynomial addresses the non-trivial
# spectrum.

def _ops(rowptr, col, w, problem):
    """(A, B diagonal, trivial vector) of the problem's preconditioned operator."""
    d = laplacian.degrees(rowptr, col, w)
    n = d.size
    if problem == laplacian.GENERALIZED:
        A = lambda Z: laplacian.apply(rowptr, col, w, Z) / (d if Z.ndim == 1 else d[:, None])
        return A, d, np.ones(n)
    if problem == laplacian.NORMALIZED:
        A = lambda Z: laplacian.apply_normalized(rowptr, col, w, Z)
        return A, np.ones(n), np.sqrt(d)
    A = lambda Z: laplacian.apply(rowptr, col, w, Z)
    return A, np.ones(n), np.ones(n)


def gmres_poly_roots(rowptr, col, w, problem, b, degree):
    """The degree + 1 roots (harmonic Ritz values, modified Leja order) of the
    GMRES residual polynomial from start vector b."""
    import scipy.linalg
    A, bd, z = _ops(rowptr, col, w, problem)
    k1 = degree + 1
    b = np.asarray(b, dtype=np.float64).copy()
    b -= z * ((z * bd) @ b) / ((z * bd) @ z)             # B-orthogonal to the trivial vector
    V = np.zeros((b.size, k1 + 1))
    H = np.zeros((k1 + 1, k1))
    V[:, 0] = b / np.sqrt(b @ (bd * b))
    for j in range(k1):
        wv = A(V[:, j])
        for _ in range(2):                               # Gram-Schmidt, twice
            h = V[:, :j + 1].T @ (bd * wv)
            wv = wv - V[:, :j + 1] @ h
            H[:j + 1, j] += h
        H[j + 1, j] = np.sqrt(wv @ (bd * wv))
        if H[j + 1, j] <= 1e-12 * np.abs(H[:j + 1, j]).max():
            # invariant Krylov space: its j + 1 Ritz values are exact roots
            k1 = j + 1
            H = H[:k1 + 1, :k1]
            H[k1, k1 - 1] = 0.0
            break
        V[:, j + 1] = wv / H[j + 1, j]
    Hk = 0.5 * (H[:k1, :k1] + H[:k1, :k1].T)
    theta = scipy.linalg.eigh(H.T @ H, Hk, eigvals_only=True)
    return leja_order(theta)


def leja_order(theta):
    """Modified Leja ordering: the largest |theta| first, then each next one
    maximises the sum of log distances to those already chosen (lowest index
    on ties)."""
    theta = np.asarray(theta, dtype=np.float64)
    left = list(range(theta.size))
    first = max(left, key=lambda i: (abs(theta[i]), -i))
    out = [first]
    left.remove(first)
    while left:
        score = [sum(np.log(abs(theta[i] - theta[j])) for j in out) for i in left]
        best = left[int(np.argmax(score))]
        out.append(best)
        left.remove(best)
    return theta[out]


def gmres_poly_apply(rowptr, col, w, problem, R, roots):
    """H = p(A) R' with p from the roots: R' = D^-1 R for the generalized
    problem (the preconditioner p(D^-1 L) D^-1, as for Chebyshev), R otherwise."""
    A, bd, z = _ops(rowptr, col, w, problem)
    R = np.asarray(R, dtype=np.float64)
    prod = R / bd[:, None] if problem == laplacian.GENERALIZED else R.copy()
    Y = np.zeros_like(prod)
    for i, t in enumerate(roots):
        Y = Y + prod / t
        if i < len(roots) - 1:
            prod = prod - A(prod) / t
    return Y
