"""Graph Laplacian in FP64 (oracle; test infrastructure only).

Paper: Sec. 3.2 (Spectral Graph Partitioning).  The combinatorial Laplacian is
L_C = D - A (Eq. 2); for weighted graphs the off-diagonal entries are the
negated edge weights and the diagonal holds the sum of incident weights (the
paragraph after Eq. 3).  The generalized problem is L_C x = lambda D x.  The
normalized Laplacian is L_N = I - D^-1/2 A D^-1/2 (the equation after Eq. 2),
with the standard problem L_N y = lambda y.

Reading taken (self-loops): the paper symmetrises inputs as A + A^T + I
(Sec. 6.1) but Eq. 2 only uses off-diagonal adjacency, so self-loops carry no
weight here; inputs have none.
"""
from __future__ import annotations

import math

import numpy as np

COMBINATORIAL = 0
GENERALIZED = 1
NORMALIZED = 2


def _weights(col, w):
    return np.ones(col.shape[0], dtype=np.float64) if w is None else np.asarray(w, dtype=np.float64)


def row_index(rowptr):
    """Row id of every CSR entry."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    return np.repeat(np.arange(rowptr.size - 1, dtype=np.int64), np.diff(rowptr))


def degrees(rowptr, col, w=None):
    """Weighted degree d_i = sum_j w_ij (the diagonal of L_C, Eq. 2 weighted),
    the exact sum rounded once (math.fsum), so no summation order enters."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    if w is None:
        return np.diff(rowptr).astype(np.float64)
    ww = np.asarray(w, dtype=np.float64)
    return np.array([math.fsum(ww[rowptr[i]:rowptr[i + 1]].tolist())
                     for i in range(rowptr.size - 1)], dtype=np.float64)


def pattern_degrees(rowptr):
    """Number of neighbours of each vertex (the paper's "degree")."""
    return np.diff(np.asarray(rowptr, dtype=np.int64))


def is_regular(rowptr):
    """Sec. 6.1: a graph is regular iff max degree / average degree <= 10."""
    deg = pattern_degrees(rowptr)
    n = deg.size
    if n == 0 or deg.sum() == 0:
        return True
    return deg.max() * n <= 10 * deg.sum()


def apply(rowptr, col, w, X):
    """Y = L_C X in FP64, written as (L x)_i = sum_j w_ij (x_i - x_j).

    This is (D - A) x of Eq. 2 with weights, summed in difference form so that
    a constant vector maps to exactly zero.
    """
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    ww = _weights(col, w)
    r = row_index(rowptr)
    contrib = ww[:, None] * (X[r] - X[np.asarray(col, dtype=np.int64)])
    Y = np.zeros_like(X)
    np.add.at(Y, r, contrib)
    return Y[:, 0] if squeeze else Y


def apply_sparse(rowptr, col, w, X):
    """Y = L_C X in FP64 as D X - A X with a library sparse product, for graphs
    too large for `apply`.  The same operator (Eq. 2 weighted); only the
    rounding order differs from the difference form."""
    import scipy.sparse as sp
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.size - 1
    A = sp.csr_matrix((_weights(col, w), np.asarray(col, dtype=np.int64), rowptr), shape=(n, n))
    d = np.asarray(A.sum(axis=1)).ravel()
    X = np.asarray(X, dtype=np.float64)
    return (d[:, None] * X if X.ndim == 2 else d * X) - A @ X


def apply_normalized(rowptr, col, w, X):
    """Y = L_N X in FP64 from the definition L_N = I - D^-1/2 A D^-1/2:
    y_i = x_i - sum_j w_ij x_j / sqrt(d_i d_j), d the weighted degrees."""
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    d = degrees(rowptr, col, w)
    if (d <= 0).any():
        raise ValueError("L_N needs every degree > 0")
    ww = _weights(col, w)
    r = row_index(rowptr)
    c = np.asarray(col, dtype=np.int64)
    contrib = (ww / np.sqrt(d[r] * d[c]))[:, None] * X[c]
    AX = np.zeros_like(X)
    np.add.at(AX, r, contrib)
    Y = X - AX
    return Y[:, 0] if squeeze else Y


def apply_normalized_sparse(rowptr, col, w, X):
    """Y = L_N X = X - D^-1/2 A D^-1/2 X with a library sparse product, for
    graphs too large for `apply_normalized` (same operator, other rounding)."""
    import scipy.sparse as sp
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.size - 1
    A = sp.csr_matrix((_weights(col, w), np.asarray(col, dtype=np.int64), rowptr), shape=(n, n))
    d = np.asarray(A.sum(axis=1)).ravel()
    if (d <= 0).any():
        raise ValueError("L_N needs every degree > 0")
    s = 1.0 / np.sqrt(d)
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        return X - s * (A @ (s * X))
    return X - s[:, None] * (A @ (s[:, None] * X))


def omp_operator(rowptr, col, w, threads=None):
    """Z -> L_C Z as a callable over the oracle's C/OpenMP loop
    (oracle/csrc/lap_omp.c): the same difference form as `apply`, each row's
    entries summed in CSR order, for graphs too large for `apply`.  The CSR
    arrays are converted once, here."""
    import ctypes
    from . import _native
    lib = _native.lib()
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    cc = np.ascontiguousarray(col, dtype=np.int32)
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    n = rp.size - 1
    nt = _native.default_threads() if threads is None else int(threads)

    def op(Z):
        Z = np.asarray(Z, dtype=np.float64)
        squeeze = Z.ndim == 1
        Zc = np.ascontiguousarray(Z.reshape(n, -1))
        Y = np.empty_like(Zc)
        lib.oracle_lap_apply(n, rp.ctypes.data, cc.ctypes.data,
                             None if ww is None else ww.ctypes.data,
                             Zc.ctypes.data, Zc.shape[1], Y.ctypes.data, nt)
        return Y[:, 0] if squeeze else Y
    return op


def apply_omp(rowptr, col, w, X, threads=None):
    """Y = L_C X through `omp_operator` (one call)."""
    return omp_operator(rowptr, col, w, threads)(X)


def operator(rowptr, col, w, problem, fast=False):
    """The matrix of the eigenproblem as a callable: L_C for the
    combinatorial and generalized problems, L_N for the normalized one.
    fast: use the C/OpenMP loop (`omp_operator`); L_N is then applied as
    D^-1/2 L_C D^-1/2, the same operator as `apply_normalized`."""
    if not fast:
        if problem == NORMALIZED:
            return lambda Z: apply_normalized(rowptr, col, w, Z)
        return lambda Z: apply(rowptr, col, w, Z)
    LC = omp_operator(rowptr, col, w)
    if problem != NORMALIZED:
        return LC
    d = degrees_fast(rowptr, col, w)
    if (d <= 0).any():
        raise ValueError("L_N needs every degree > 0")
    s = 1.0 / np.sqrt(d)

    def op(Z):
        Z = np.asarray(Z, dtype=np.float64)
        if Z.ndim == 1:
            return s * LC(s * Z)
        return s[:, None] * LC(s[:, None] * Z)
    return op


def degrees_fast(rowptr, col, w=None):
    """Weighted degrees for large graphs: each row's weights summed in FP64
    in CSR order (`degrees` rounds the exact sum once instead and is slow on
    large graphs; the two differ by at most a few units in the last place).
    Unit weights: the row lengths, exactly."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    if w is None:
        return np.diff(rowptr).astype(np.float64)
    ww = np.asarray(w, dtype=np.float64)
    n = rowptr.size - 1
    r = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    return np.bincount(r, weights=ww, minlength=n).astype(np.float64)


def dense_normalized(rowptr, col, w, n=None):
    """Dense L_N entry by entry: 1 on the diagonal, -w_ij / sqrt(d_i d_j) off it."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.size - 1 if n is None else n
    ww = _weights(col, w)
    d = degrees(rowptr, col, w)
    L = np.eye(n)
    for i in range(n):
        for k in range(rowptr[i], rowptr[i + 1]):
            j = int(col[k])
            L[i, j] -= ww[k] / math.sqrt(d[i] * d[j])
    return L


def dense(rowptr, col, w, n=None):
    """Dense (L_C, d) built entry by entry from Eq. 2: L_ii = d_i, L_ij = -w_ij."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.size - 1 if n is None else n
    ww = _weights(col, w)
    L = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for k in range(rowptr[i], rowptr[i + 1]):
            j = int(col[k])
            L[i, j] -= ww[k]
            L[i, i] += ww[k]
    return L, np.diag(L).copy()


def bdiag(rowptr, col, w, problem):
    """Diagonal of B: ones (combinatorial L_C x = lambda x, normalized
    L_N y = lambda y) or the weighted degrees (generalized, L_C x = lambda D x),
    Sec. 3.2."""
    n = len(rowptr) - 1
    if problem in (COMBINATORIAL, NORMALIZED):
        return np.ones(n, dtype=np.float64)
    return degrees(rowptr, col, w)


def residual_norms(LX, X, theta, bd):
    """Relative residuals rho_i of Ritz pairs (theta_i, x_i).

    Reading taken (the paper gives tolerance values, Sec. 6.3.2, but no norm):
      rho_i = ||L x_i - theta_i B x_i||_{B^-1} / (max(theta_i, theta_1) ||x_i||_B)
    i.e. the relative residual of the equivalent standard problem
    B^-1/2 L B^-1/2, with theta_1 (the smallest non-trivial Ritz value) as a
    floor so that the trivial pair theta_0 ~ 0 is measured on the same scale.
    theta must be sorted ascending.
    """
    X = np.asarray(X, dtype=np.float64)
    R = LX - (bd[:, None] * X) * theta[None, :]
    rn = np.sqrt(np.sum(R * R / bd[:, None], axis=0))
    xn = np.sqrt(np.sum(bd[:, None] * X * X, axis=0))
    floor = theta[1] if theta.size > 1 else theta[0]
    scale = np.maximum(theta, floor)
    scale = np.where(scale > 0, scale, 1.0)
    return rn / (scale * xn)
