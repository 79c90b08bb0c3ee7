"""Certified eigenpair fixtures (tests/golden/certified_<name>.json) and the
accuracy gates built on them.

The fixtures hold, per workload, the oracle's Ritz values theta_0..theta_{d+g-1}
(g guard columns), their residual norms eps_i, the lower bounds
lam_lo_k = theta_k - eps_k of the eigenvalues, and the blocks k whose
separation is large enough to certify a subspace (see oracle.certify).

Gates for a basis V (n x d) returned by the GPU:
* eigenvalues: lambda_i in [theta_i - eig_bound, theta_i] (the oracle's
  certificate; where the d-block ends inside a degenerate eigenvalue and has
  no certificate, within eps_i of theta_i by Weinstein's theorem), so
  |lambda_gpu,i - lambda_i| <= |lambda_gpu,i - theta_i| + bound must be at
  most rel * theta_i (the trivial pair: at most rel * theta_1);
* subspace: for each separated leading block of k columns, the Davis-Kahan
  bound of the GPU's own residual against the certified lam_lo_k,
  sin <= ||R_k||_F / (lam_lo_k - theta_{k-1}(V)), computed in FP64 with the
  oracle's operator, must be at most 1e-3.
"""
import hashlib
import json
import os

import numpy as np

from oracle import certify, laplacian as lap

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, f"certified_{name}.json")) as f:
        return json.load(f)


def digest(g):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g.rowptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(g.col, dtype=np.int32).tobytes())
    if g.w is not None:
        h.update(np.ascontiguousarray(g.w, dtype=np.float64).tobytes())
    return h.hexdigest()


def problem_code(gold):
    return {"combinatorial": lap.COMBINATORIAL, "generalized": lap.GENERALIZED,
            "normalized": lap.NORMALIZED}[gold["problem"]]


def eigenvalue_errors(gold, lam):
    """Worst-case relative distance of each GPU eigenvalue from the certified
    interval of the exact one (trivial pair: relative to theta_1)."""
    th = np.asarray(gold["theta"])
    lam = np.asarray(lam, dtype=np.float64)
    d = lam.size
    # the block's quadratic bound when the block is separated; otherwise
    # (block edge inside a degenerate eigenvalue) each value's Weinstein
    # radius eps_i, which is first order but still far below the targets
    bound = gold["eig_bound"]
    if not np.isfinite(bound):
        bound = np.asarray(gold["eps"])[:d]
    err = np.abs(lam - th[:d]) + bound
    scale = th[:d].copy()
    scale[0] = th[1]
    return err / scale


def separated_blocks(gold, rel_gap, kmax=None):
    """Leading block sizes k (2 <= k <= kmax, default d) whose certified
    separation lam_lo_k - theta_{k-1} is at least rel_gap * theta_k."""
    th = np.asarray(gold["theta"])
    lo = np.asarray(gold["lam_lo"])
    kmax = gold["d"] if kmax is None else kmax
    return [k for k in range(2, kmax + 1) if lo[k] - th[k - 1] >= rel_gap * th[k]]


def subspace_bounds(g, gold, V, blocks):
    """{k: Davis-Kahan sine bound of span(V[:, :k]) against the exact
    invariant subspace of the k smallest eigenvalues} for k in blocks."""
    problem = problem_code(gold)
    op = lap.operator(g.rowptr, g.col, g.w, problem, fast=True)
    bd = (lap.degrees_fast(g.rowptr, g.col, g.w) if problem == lap.GENERALIZED
          else np.ones(g.n))
    V = np.asarray(V, dtype=np.float64)
    out = {}
    for k in blocks:
        c = certify.certify_block(op, bd, V[:, :k], gold["lam_lo"][k])
        out[k] = c["sin_bound"]
    return out
