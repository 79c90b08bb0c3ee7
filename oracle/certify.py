"""Certified eigenpairs for graphs too large for a dense solve (oracle; test
infrastructure only).

Paper: Sec. 3.2 (the pencils L_C x = lambda x, L_C x = lambda D x and
L_N y = lambda y) and Algorithm 1 (LOBPCG).  What the GPU path approximates is
the plain definition "the d smallest eigenpairs of (L, B)"; for graphs of
millions of vertices that definition cannot be written out densely, so this
module computes it the way Algorithm 1 does, in FP64, far past the solver's
tolerance, and states how far the result can be from the definition:

1. LOBPCG (`eigen.lobpcg`, Algorithm 1) on a block of d + g columns (g guard
   columns), the first d to a relative residual `tol` (1e-10 by default),
   the guards to `guard_tol`.
2. The Ritz vectors of the first d + g columns are B-orthonormalised again
   and their residuals recomputed with a fresh operator product:
   eps_i = ||L x_i - theta_i B x_i||_{B^-1}.
3. Gap.  Weinstein's theorem puts an eigenvalue within eps_d of theta_d.
   Under the ordering assumption (A) -- the Ritz values theta_0 <= ... are
   approximations of the d + g smallest eigenvalues, one each, so the one
   near theta_d is lambda_d -- the unwanted spectrum starts at
   lambda_d >= lam_d_lo = theta_d - eps_d, and the separation of the wanted
   block is delta = lam_d_lo - theta_{d-1}.
4. Eigenvalues.  Courant-Fischer gives lambda_i <= theta_i; the quadratic
   residual bound for a block of Ritz pairs (Mathias 1998; Sun 1991) gives
   theta_i - lambda_i <= ||R||_2^2 / delta, with R the residual block of the d
   wanted columns in the B^-1 norm (its Frobenius norm is used, an upper
   bound of ||R||_2).
5. Subspace.  Davis-Kahan's sin(Theta) theorem: the largest principal angle
   between the computed and the exact invariant subspace of the d smallest
   eigenvalues satisfies sin <= ||R||_F / delta.

Assumption (A) is not proved here (that would take an inertia count, i.e. a
sparse factorisation of L - sigma B, which does not fit for these graphs).
It is supported by (i) runs from independent start blocks that must agree,
and (ii) the tests of this module on graphs whose spectrum is known (closed
forms and dense solves), where the bounds are checked against the truth.

The same bounds, with the certified lam_d_lo, certify any other basis of the
wanted subspace (for instance the GPU's): `certify_block`.
"""
from __future__ import annotations

import time

import numpy as np

from . import eigen, laplacian, precond


def _borth(X, bd):
    """B-orthonormal basis of span(X) (Cholesky of the Gram matrix)."""
    G = X.T @ (bd[:, None] * X)
    C = np.linalg.cholesky(0.5 * (G + G.T))
    return np.linalg.solve(C, X.T).T


def residual_block(op, bd, X):
    """Rayleigh-Ritz of (L, B) on span(X) in FP64, then the B^-1-norm residual
    of every Ritz pair.  Returns (theta ascending, Ritz vectors, eps)."""
    Q = _borth(np.asarray(X, dtype=np.float64), bd)
    LQ = op(Q)
    A = Q.T @ LQ
    theta, Z = np.linalg.eigh(0.5 * (A + A.T))
    V = Q @ Z
    LV = LQ @ Z
    R = LV - (bd[:, None] * V) * theta[None, :]
    eps = np.sqrt(np.sum(R * R / bd[:, None], axis=0))
    return theta, V, eps


def certify_block(op, bd, X, lam_d_lo):
    """Bounds for span(X) (d columns) against the exact invariant subspace of
    the d smallest eigenvalues, given a lower bound lam_d_lo of the first
    unwanted eigenvalue.  Returns a dict with the Ritz values, eps, delta,
    the eigenvalue bound ||R||^2/delta and the subspace bound ||R||_F/delta
    (inf when delta <= 0)."""
    theta, V, eps = residual_block(op, bd, X)
    rF = float(np.sqrt(np.sum(eps ** 2)))
    delta = float(lam_d_lo - theta[-1])
    ok = delta > 0
    return {
        "theta": theta, "eps": eps, "delta": delta,
        "eig_bound": rF ** 2 / delta if ok else np.inf,
        "sin_bound": rF / delta if ok else np.inf,
        "vectors": V,
    }


def certified_eigenpairs(rowptr, col, w, problem, d, guards=4, tol=1e-10,
                         guard_tol=1e-8, X0=None, seed=7, maxiter=20000,
                         prec="jacobi", cheb_degree=25, cheb_ratio=1000.0,
                         log=None):
    """The d smallest eigenpairs of (L, B) with certified error bounds.

    problem: laplacian.COMBINATORIAL / GENERALIZED / NORMALIZED (Sec. 3.2).
    X0: n x (d + guards) start block, else N(0,1) from `seed`.
    prec: 'jacobi' (Sec. 5.1) or 'chebyshev' (Sec. 5.2, Chebyshev reading).
    Returns a dict: theta (d + guards Ritz values), eps, lam_d_lo, delta,
    eig_bound (per wanted value: theta_i - bound <= lambda_i <= theta_i),
    sin_bound, vectors (n x d, B-orthonormal, sign rule), iterations, seconds.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.size - 1
    nev = d + guards
    op = laplacian.operator(rowptr, col, w, problem, fast=True)
    deg = laplacian.degrees_fast(rowptr, col, w)
    bd = deg if problem == laplacian.GENERALIZED else np.ones(n)
    if X0 is None:
        X0 = np.random.default_rng(seed).standard_normal((n, nev))
    if prec == "jacobi":
        dL = np.ones(n) if problem == laplacian.NORMALIZED else deg
        pre = lambda R: precond.jacobi(R, dL)           # noqa: E731
    elif prec == "chebyshev":
        hi = precond.gershgorin_bound(deg, problem)
        dinv = 1.0 / deg if problem == laplacian.GENERALIZED else None
        pre = lambda R: precond.chebyshev(               # noqa: E731
            rowptr, col, w, R, cheb_degree, hi / cheb_ratio, hi, dinv=dinv,
            problem=problem, op=op)
    else:
        raise ValueError(prec)
    tolv = np.array([tol] * d + [guard_tol] * guards)
    t0 = time.time()
    theta, X, its, rho = eigen.lobpcg(rowptr, col, w, problem, X0, pre, tolv,
                                      maxiter=maxiter, op=op, bd=bd, log=log)
    secs = time.time() - t0
    # fresh residuals of the whole block, then the bounds of the wanted part
    th_all, V_all, eps_all = residual_block(op, bd, X)
    lam_d_lo = float(th_all[d] - eps_all[d])
    cert = certify_block(op, bd, V_all[:, :d], lam_d_lo)
    if log:
        log(f"certified: {its} iterations, {secs:.1f} s, delta {cert['delta']:.3e}")
    return {
        "theta": th_all, "eps": eps_all, "lam_d_lo": lam_d_lo,
        "delta": cert["delta"], "eig_bound": cert["eig_bound"],
        "sin_bound": cert["sin_bound"],
        "vectors": eigen.normalize_signs(cert["vectors"]),
        "iterations": int(its), "seconds": secs, "rho": rho,
    }
