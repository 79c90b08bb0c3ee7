"""Eigenpairs of the graph Laplacian (oracle; test infrastructure only).

Paper: Sec. 3.2 (problems L_C x = lambda x, L_C x = lambda D x and
L_N y = lambda y), Sec. 3.3 and
Algorithm 1 (LOBPCG), Sec. 4 and Eq. 4 (number of eigenvectors).

The plain definition of what the solver computes is "the d smallest eigenpairs
of the pencil (L, B)", B = I or D; `smallest_dense` writes that definition out
with a dense symmetric-definite eigensolver (a library primitive).  `lobpcg`
follows Algorithm 1 step by step and serves iteration-count comparisons and
medium-size graphs where a dense solve is too large.

Normalisation conventions (shared with the GPU path's documented contract,
not its code): eigenvectors are B-orthonormal, eigenvalues ascending, and
each vector's sign is chosen so that its entry of largest magnitude (lowest
index on ties) is positive.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import laplacian


def num_eigenvectors(K):
    """Eq. 4: d = floor(log2 K) + 1 (the trivial eigenvector included)."""
    if K < 1:
        raise ValueError("K must be >= 1")
    return int(K).bit_length()


def normalize_signs(V):
    """Flip each column so that its largest-magnitude entry is positive."""
    V = np.array(V, dtype=np.float64, copy=True)
    for k in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, k])))     # first index on ties
        if V[i, k] < 0:
            V[:, k] = -V[:, k]
    return V


def smallest_dense(L, bd, d):
    """The d smallest eigenpairs of L v = lambda B v with B = diag(bd)."""
    n = L.shape[0]
    lam, V = scipy.linalg.eigh(L, np.diag(bd), subset_by_index=[0, d - 1])
    return lam, normalize_signs(V)


def all_dense(L, bd):
    """Full eigendecomposition of the pencil (L, diag(bd)), ascending."""
    lam, V = scipy.linalg.eigh(L, np.diag(bd))
    return lam, V


def rayleigh_ritz(S, LS, bd, nev, drop=1e-12):
    """RR(S, nev) of Algorithm 1: Ritz pairs of (L, B) on span(S).

    A B-orthonormal basis Q = S C of span(S) is formed from the Gram matrix
    S^T B S (directions with relative weight below `drop` are discarded as
    linearly dependent); the projected matrix Q^T L Q is diagonalised and the
    nev smallest Ritz values are kept.  Returns (theta, Y) with X = S Y.
    """
    G = S.T @ (bd[:, None] * S)
    G = 0.5 * (G + G.T)
    A = S.T @ LS
    A = 0.5 * (A + A.T)
    s = np.sqrt(np.maximum(np.diag(G), 1e-300))
    Gs = G / np.outer(s, s)
    As = A / np.outer(s, s)
    sig, U = np.linalg.eigh(Gs)
    keep = sig > drop * sig.max()
    C = U[:, keep] / np.sqrt(sig[keep])[None, :]
    # second pass: C^T Gs C is the identity up to rounding amplified by the
    # small kept Gram eigenvalues; orthonormalise once more against it
    G2 = C.T @ Gs @ C
    sig2, U2 = np.linalg.eigh(0.5 * (G2 + G2.T))
    C = C @ (U2 / np.sqrt(sig2)[None, :])
    Ap = C.T @ As @ C
    Ap = 0.5 * (Ap + Ap.T)
    theta, Z = np.linalg.eigh(Ap)
    Y = (C @ Z[:, :nev]) / s[:, None]
    return theta[:nev], Y


def _bnormalize(Z, LZ, bd):
    """Scale the columns of Z (and of LZ = L Z alike) to unit B-norm (zero
    columns stay zero)."""
    nrm = np.sqrt(np.sum(bd[:, None] * Z * Z, axis=0))
    nrm = np.where(nrm > 0, nrm, 1.0)
    return Z / nrm[None, :], (None if LZ is None else LZ / nrm[None, :])


def lobpcg(rowptr, col, w, problem, X0, precond, tol, maxiter=10000,
           locking=True, op=None, bd=None, log=None, log_every=50):
    """Algorithm 1 (LOBPCG, Hetmaniuk-Lehoucq form) for L x = lambda B x
    (L = L_N and B = I for the normalized problem).

    precond: callable R -> H (the solve "M H = R"), or None for H = R.
    tol: bound on the relative residual rho_i of `laplacian.residual_norms`
    (a scalar, or one bound per column).
    locking: soft locking -- only unconverged columns contribute residual
    directions and conjugate directions (the "I" subsets of Algorithm 1).
    op, bd: the operator Z -> L Z and the diagonal of B, when the caller has
    them already (large graphs: `laplacian.operator(..., fast=True)`).
    log: callable(str) for a progress line every log_every iterations.
    Returns (theta, X, iterations, rho).

    Numerical safeguards that leave the iteration's subspaces unchanged (RR
    depends on span(S) only): the H and P columns are scaled to unit B-norm
    before each Rayleigh-Ritz step, and L X is recomputed with one product per
    iteration instead of being carried by recurrence, and so is L P (over
    hundreds of iterations to tolerances near 1e-10 the recurrences drift and
    the unscaled blocks can over- or underflow).
    """
    if bd is None:
        bd = laplacian.bdiag(rowptr, col, w, problem)
    L = laplacian.operator(rowptr, col, w, problem) if op is None else op
    tol = np.asarray(tol, dtype=np.float64)
    X = np.asarray(X0, dtype=np.float64)
    nev = X.shape[1]
    # initial Rayleigh-Ritz on the starting block
    theta, Y = rayleigh_ritz(X, L(X), bd, nev)
    X = X @ Y
    LX = L(X)
    rho = laplacian.residual_norms(LX, X, theta, bd)
    active = np.ones(nev, dtype=bool) if not locking else rho > tol
    P = np.zeros((X.shape[0], 0))
    LP = np.zeros_like(P)
    it = 0
    while it < maxiter and (rho > tol).any():
        act = np.flatnonzero(active) if locking else np.arange(nev)
        R = LX[:, act] - (bd[:, None] * X[:, act]) * theta[act][None, :]
        H = R if precond is None else precond(R)
        H, _ = _bnormalize(H, None, bd)
        LH = L(H)
        S = np.hstack([X, H, P])
        LS = np.hstack([LX, LH, LP])
        theta, Y = rayleigh_ritz(S, LS, bd, nev)
        X = S @ Y
        LX = L(X)
        rho = laplacian.residual_norms(LX, X, theta, bd)
        it += 1
        if log and it % log_every == 0:
            log(f"lobpcg it {it}: max rho {rho.max():.3e}, "
                f"unconverged {int((rho > tol).sum())}")
        active = rho > tol if locking else np.ones(nev, dtype=bool)
        # P_I <- [0, H_I, P_I] Y_I : the X rows of Y are dropped
        YI = Y[:, active] if locking else Y
        YI = YI.copy()
        YI[:nev, :] = 0.0
        P, _ = _bnormalize(S @ YI, None, bd)
        LP = L(P)
    # final residual from an explicit product (no recurrence drift)
    LX = L(X)
    rho = laplacian.residual_norms(LX, X, theta, bd)
    return theta, normalize_signs_b(X, bd), it, rho


def normalize_signs_b(X, bd):
    """B-normalise each column and apply the sign convention."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.sqrt(np.sum(bd[:, None] * X * X, axis=0))
    return normalize_signs(X / nrm[None, :])


def subspace_sin(U, V, bd):
    """Sine of the largest principal angle between span(U) and span(V) in the
    B-inner product: the largest B-norm of the part of an orthonormal basis
    vector of span(V) that lies outside span(U)."""
    def borth(Z):
        G = Z.T @ (bd[:, None] * Z)
        Lc = np.linalg.cholesky(0.5 * (G + G.T))
        return np.linalg.solve(Lc, Z.T).T
    Uq, Vq = borth(np.asarray(U, float)), borth(np.asarray(V, float))
    W = Vq - Uq @ (Uq.T @ (bd[:, None] * Vq))
    G = W.T @ (bd[:, None] * W)
    return float(np.sqrt(max(0.0, np.linalg.eigvalsh(0.5 * (G + G.T)).max())))
