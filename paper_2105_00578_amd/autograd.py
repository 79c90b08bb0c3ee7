"""torch.autograd.Function over the eigensolve, with the library's adjoint.

The edge weights enter as one float64 value per CSR entry (both directions
of an undirected edge hold the same weight).  The backward returns, for each
CSR entry, half of dl/dw_e of its edge, so that a symmetric parameterisation
w_csr = w_edge[edge_of_entry] receives the full derivative through autograd.
"""
from __future__ import annotations

import torch

from . import _lib


class EigFn(torch.autograd.Function):
    """(eigvals, V) = EigFn.apply(w_csr, handle, rowptr, col, nev, opts, X0).

    opts.precision must be FP64 (the adjoint works on FP64 eigenvectors).
    eigvals: float64[nev] (device), V: n x nev float64 (device), B-orthonormal.
    """

    @staticmethod
    def forward(ctx, w, handle, rowptr, col, nev, opts, X0=None):
        if opts.precision != _lib.FP64:
            raise ValueError("EigFn needs FP64 precision")
        w = w.detach().to(torch.float64).contiguous()
        g = _lib.Graph(handle, rowptr, col, w, validate=False)
        lam, V, st = _lib.eigensolve(handle, g, nev, opts, X0)
        ctx.handle = handle
        ctx.graph = g
        ctx.problem = opts.problem
        ctx.lam = lam
        ctx.stats = st
        ctx.save_for_backward(V)
        lam_t = torch.tensor(lam, dtype=torch.float64, device=V.device)
        return lam_t, V

    @staticmethod
    def backward(ctx, g_lam, g_V):
        (V,) = ctx.saved_tensors
        gl = None if g_lam is None else g_lam.detach().to("cpu", torch.float64).tolist()
        gv = None if g_V is None else g_V.detach().to(torch.float64).contiguous()
        grad = _lib.eig_backward(ctx.handle, ctx.graph, ctx.problem, ctx.lam, V, gl, gv)
        return 0.5 * grad, None, None, None, None, None, None
