"""Caller-supplied workspace: with a buffer of sphx_workspace_size bytes
(attached by the Python binding from a PyTorch tensor) the solve, partition,
adjoint and operator calls allocate no device memory of their own."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from tests.gpu_util import upload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [sx.FP64, sx.MIXED])
def test_partition_and_solve_use_the_callers_workspace(prec):
    h = sx.Handle(0)
    g = graphgen.config_graph("grid7_128", scale_down=8)          # 16^3 grid
    rp, col, w = upload(g)
    G = sx.Graph(h, rp, col, w)                                   # validation: no allocation
    assert sx.workspace_owned(h) == 0
    reg, _, _ = G.info()
    assert sx.workspace_owned(h) == 0
    opts = sx.options_default(reg, sx.PRECOND_CHEBYSHEV, precision=prec, tol=1e-4)
    for K in (4, 7, 24):                                          # K = 24: not a power of two
        lam, V, part, cut, imb, st = sx.partition(h, G, K, opts)
        assert sx.workspace_owned(h) == 0
    lam, V, st = sx.eigensolve(h, G, 5, opts)
    assert sx.workspace_owned(h) == 0
    X = torch.randn(g.n, 3, dtype=torch.float64, device=rp.device)
    sx.laplacian_apply(h, G, X)
    sx.laplacian_apply(h, G, X, problem=sx.NORMALIZED)
    sx.precond_apply(h, G, opts, X)
    assert sx.workspace_owned(h) == 0
    # the buffer the binding attached is at least the size the library asks for
    assert h._ws.numel() >= sx.workspace_size(h, G, 5, opts)


def test_backward_uses_the_callers_workspace():
    h = sx.Handle(0)
    g = graphgen.config_graph("king512", scale_down=32)          # 16 x 16 weighted
    rp, col, w = upload(g)
    G = sx.Graph(h, rp, col, w)
    opts = sx.options_default(True, sx.PRECOND_JACOBI, precision=sx.FP64,
                              problem=sx.GENERALIZED, tol=1e-12, max_iter=20000)
    lam, V, st = sx.eigensolve(h, G, 4, opts)
    gv = torch.randn(g.n, 4, dtype=torch.float64, device=rp.device)
    sx.eig_backward(h, G, sx.GENERALIZED, lam, V, g_vals=[0, 1, 1, 1], g_vecs=gv,
                    cg_tol=1e-8, allow_not_converged=True)
    assert sx.workspace_owned(h) == 0


def test_without_workspace_the_handle_allocates_and_releases():
    """The other side of the contract: with no workspace attached the library
    caches its own, and sphx_workspace_release frees it."""
    h = sx.Handle(0)
    g = graphgen.config_graph("grid64", scale_down=4)
    rp, col, w = upload(g)
    G = sx.Graph(h, rp, col, w)
    part = torch.zeros(g.n, dtype=torch.int32, device=rp.device)
    sx.quality(h, G, part, 4)            # the quality call attaches nothing
    assert sx.workspace_owned(h) > 0
    sx.workspace_release(h)
    assert sx.workspace_owned(h) == 0
