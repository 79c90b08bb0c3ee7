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

Two evaluations:
  grad_dense      - the formula above with the full eigenbasis of a dense
                    pencil (tiny graphs);
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
