"""Derivatives of Laplacian eigenpairs with respect to edge weights (oracle;
test infrastructure only).

The paper has no differentiation; the derivative follows from its weighted
Laplacian (Sec. 3.2, after Eq. 3): raising the weight w_e of edge e = {i, j}
by dw changes L_C by dw (e_i - e_j)(e_i - e_j)^T and, for the generalized
problem, D by dw (e_i e_i^T + e_j e_j^T).  Let M_k = dL - lambda_k dB.  For
B-orthonormal eigenvectors of L v = lambda B v with simple eigenvalues,
  d lambda_k = v_k^T M_k v_k,
  d v_k = sum_{j != k} v_j (v_j^T M_k v_k) / (lambda_k - lambda_j)
          - 1/2 v_k (v_k^T dB v_k),
(first-order perturbation theory for a symmetric-definite pencil).  For a loss
l(lambda, V) with partials g_lambda (per eigenvalue) and g_k = dl/dv_k, the
edge gradient is dl/dw_e = sum_k g_lambda_k dlambda_k/dw_e + g_k^T dv_k/dw_e.

Three evaluations:
  grad_dense      - the formula above with the full eigenbasis of a dense
                    pencil (tiny graphs);
  grad_dense_normalized - the same for L_N y = lambda y (B = I), with dL_N
                    written out densely per edge;
  grad_projected  - only the computed block V (eigenpairs 0..nev-1) is used;
                    the sum over eigenvectors outside the block is replaced by
                    mu_k, the solution of (L - lambda_k B) mu_k = g_k - B V V^T g_k
                    with V^T B mu_k = 0, found by a sparse direct solve of the
                    bordered system [[L - lambda_k B, B V], [V^T B, 0]].

Output format: one value per CSR entry; both stored directions of an
undirected edge carry the full derivative with respect to that edge's weight.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import laplacian, eigen


def _edge_terms(vi, vj, ui, uj, lam, generalized):
    """u^T M v for the edge {i, j}: (u_i-u_j)(v_i-v_j) - lam (u_i v_i + u_j v_j)."""
    t = (ui - uj) * (vi - vj)
    if generalized:
        t = t - lam * (ui * vi + uj * vj)
    return t


def grad_dense(rowptr, col, w, problem, nev, g_lam, g_V):
    """Full-eigenbasis edge gradient for the loss partials (g_lam, g_V) of the
    nev smallest eigenpairs.  Requires the nev smallest eigenvalues to be
    simple.  Returns (grad per CSR entry, lam[:nev], V[:, :nev])."""
    L, d = laplacian.dense(rowptr, col, w)
    gen = problem == laplacian.GENERALIZED
    bd = d if gen else np.ones_like(d)
    lam, V = eigen.all_dense(L, bd)
    # same sign convention as the solver contract
    V = eigen.normalize_signs(V)
    r = laplacian.row_index(rowptr)
    c = np.asarray(col, dtype=np.int64)
    n = V.shape[0]
    g_lam = np.zeros(nev) if g_lam is None else np.asarray(g_lam, float)
    g_V = np.zeros((n, nev)) if g_V is None else np.asarray(g_V, float)
    grad = np.zeros(r.size)
    for k in range(nev):
        vk = V[:, k]
        grad += g_lam[k] * _edge_terms(vk[r], vk[c], vk[r], vk[c], lam[k], gen)
        gk = g_V[:, k]
        if not gk.any():
            continue
        for j in range(n):
            if j == k:
                continue
            coef = (gk @ V[:, j]) / (lam[k] - lam[j])
            vj = V[:, j]
            grad += coef * _edge_terms(vk[r], vk[c], vj[r], vj[c], lam[k], gen)
        if gen:
            grad += -0.5 * (gk @ vk) * (vk[r] ** 2 + vk[c] ** 2)
    return grad, lam[:nev], V[:, :nev]


def dLN_dense(rowptr, col, w, a, b):
    """d L_N / d w_e for the edge e = {a, b} as a dense matrix, from
    L_N = I - S A S with S = D^-1/2: raising w_e by dw adds dw to A_ab and
    A_ba and to d_a and d_b, so dS = -1/2 D^-3/2 dD and
    dL_N = -(dS A S + S dA S + S A dS)."""
    L, d = laplacian.dense(rowptr, col, w)
    n = d.size
    A = np.diag(d) - L
    S = np.diag(1.0 / np.sqrt(d))
    dA = np.zeros((n, n))
    dA[a, b] = dA[b, a] = 1.0
    dd = np.zeros(n)
    dd[a] = dd[b] = 1.0
    dS = np.diag(-0.5 * d ** -1.5 * dd)
    return -(dS @ A @ S + S @ dA @ S + S @ A @ dS)


def grad_dense_normalized(rowptr, col, w, nev, g_lam, g_V):
    """Full-eigenbasis edge gradient for the normalized problem L_N y = lambda y
    (standard symmetric: d lambda_k = y_k^T dL_N y_k and
    d y_k = sum_{j != k} y_j (y_j^T dL_N y_k) / (lambda_k - lambda_j)), with
    dL_N formed densely for every edge (tiny graphs).  Returns
    (grad per CSR entry, lam[:nev], Y[:, :nev])."""
    LN = laplacian.dense_normalized(rowptr, col, w)
    n = LN.shape[0]
    lam, Y = eigen.all_dense(LN, np.ones(n))
    Y = eigen.normalize_signs(Y)
    g_lam = np.zeros(nev) if g_lam is None else np.asarray(g_lam, float)
    g_V = np.zeros((n, nev)) if g_V is None else np.asarray(g_V, float)
    r = laplacian.row_index(rowptr)
    c = np.asarray(col, dtype=np.int64)
    grad = np.zeros(r.size)
    cache = {}
    for q in range(r.size):
        a, b = int(min(r[q], c[q])), int(max(r[q], c[q]))
        if (a, b) not in cache:
            dL = dLN_dense(rowptr, col, w, a, b)
            P = Y.T @ dL @ Y[:, :nev]           # P[j, k] = y_j^T dL y_k
            tot = 0.0
            for k in range(nev):
                tot += g_lam[k] * P[k, k]
                gk = g_V[:, k]
                if gk.any():
                    coef = Y.T @ gk               # g_k . y_j
                    for j in range(n):
                        if j != k:
                            tot += coef[j] * P[j, k] / (lam[k] - lam[j])
            cache[(a, b)] = tot
        grad[q] = cache[(a, b)]
    return grad, lam[:nev], Y[:, :nev]


def _csr_matrix(rowptr, col, w, n):
    ww = np.ones(len(col)) if w is None else np.asarray(w, float)
    return sp.csr_matrix((ww, np.asarray(col, np.int64), np.asarray(rowptr, np.int64)), shape=(n, n))


def solve_mu(rowptr, col, w, problem, lam, V, g_V):
    """mu_k with (L - lambda_k B) mu_k = g_k - B V V^T g_k and V^T B mu_k = 0."""
    n, nev = V.shape
    A = _csr_matrix(rowptr, col, w, n)
    d = np.asarray(A.sum(axis=1)).ravel()
    Lc = sp.diags(d) - A
    gen = problem == laplacian.GENERALIZED
    bd = d if gen else np.ones(n)
    BV = bd[:, None] * V
    mu = np.zeros((n, nev))
    for k in range(nev):
        gk = g_V[:, k]
        if not gk.any():
            continue
        f = gk - BV @ (V.T @ gk)
        K = sp.bmat([[Lc - lam[k] * sp.diags(bd), sp.csr_matrix(BV)],
                     [sp.csr_matrix(BV.T), None]], format="csc")
        sol = spla.spsolve(K, np.concatenate([f, np.zeros(nev)]))
        mu[:, k] = sol[:n]
    return mu


def grad_projected(rowptr, col, w, problem, lam, V, g_lam, g_V):
    """Edge gradient from the computed block only (in-block terms explicit,
    out-of-block terms through mu_k).  V must be B-orthonormal eigenvectors."""
    lam = np.asarray(lam, float)
    V = np.asarray(V, float)
    n, nev = V.shape
    gen = problem == laplacian.GENERALIZED
    r = laplacian.row_index(rowptr)
    c = np.asarray(col, dtype=np.int64)
    g_lam = np.zeros(nev) if g_lam is None else np.asarray(g_lam, float)
    g_V = np.zeros((n, nev)) if g_V is None else np.asarray(g_V, float)
    grad = np.zeros(r.size)
    mu = solve_mu(rowptr, col, w, problem, lam, V, g_V) if g_V.any() else np.zeros_like(V)
    for k in range(nev):
        vk = V[:, k]
        grad += g_lam[k] * _edge_terms(vk[r], vk[c], vk[r], vk[c], lam[k], gen)
        gk = g_V[:, k]
        if not gk.any():
            continue
        for j in range(nev):
            if j == k:
                continue
            coef = (gk @ V[:, j]) / (lam[k] - lam[j])
            vj = V[:, j]
            grad += coef * _edge_terms(vk[r], vk[c], vj[r], vj[c], lam[k], gen)
        if gen:
            grad += -0.5 * (gk @ vk) * (vk[r] ** 2 + vk[c] ** 2)
        m = mu[:, k]
        grad += -_edge_terms(vk[r], vk[c], m[r], m[c], lam[k], gen)
    return grad
