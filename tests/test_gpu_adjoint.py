"""Adjoint d(loss)/d(edge weights) on the GPU.

1. With the oracle's dense eigenpairs as input, the GPU gradient equals the
   oracle's full-basis (dense) gradient.
2. End to end through EigFn on a reduced copy of the differentiation workload
   (9-point grid, weights U[0.5, 1.5), loss = sum of the 4 smallest
   non-trivial eigenvalues + ||V - V_target||^2) vs the dense reference.
3. Central differences (h = 1e-6, FP64) of GPU eigensolves along a random
   direction, for the eigenvalue part of the loss.
4. Homogeneity identities at a larger size: combinatorial eigenvalues are
   degree-1 homogeneous in w (w . grad lambda = lambda), generalized ones
   degree-0 (w . grad lambda = 0).
"""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from oracle import adjoint, eigen, laplacian as lap
from tests.gpu_util import dev, random_graph, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


def _undirected(g):
    r = lap.row_index(g.rowptr)
    return np.flatnonzero(r < g.col)


@pytest.mark.parametrize("problem", [sx.COMBINATORIAL, sx.GENERALIZED])
def test_adjoint_matches_dense_reference(handle, problem):
    g = random_graph(60, 0.08, 13, np.float64)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    nev = 5
    rng = np.random.default_rng(1)
    a = rng.standard_normal(nev)
    C = rng.standard_normal((g.n, nev))
    gd, lam, V = adjoint.grad_dense(g.rowptr, g.col, g.w, problem, nev, a, C)
    grad = sx.eig_backward(handle, G, problem, lam, torch.from_numpy(V).to(dev()), a,
                           torch.from_numpy(C).to(dev()), cg_tol=1e-14,
                           cg_max_iter=5000).cpu().numpy()
    scale = np.abs(gd).max()
    assert np.abs(grad - gd).max() <= 1e-8 * scale


def _c5_like(side):
    n, (u, v) = graphgen.grid2d_9pt(side, side)
    w = graphgen.uniform_weights(u.size, 0, dtype=np.float64)
    return graphgen.csr_from_edges(n, u, v, w)


@pytest.mark.parametrize("problem", [sx.COMBINATORIAL, sx.GENERALIZED])
def test_eigfn_reduced_workload_vs_dense(handle, problem):
    g = _c5_like(24)
    rp, col, w = upload(g)
    nev = 7                                   # trivial + 4 in the loss + 2 guards
    opts = sx.Options(problem=problem, precond=sx.PRECOND_JACOBI, tol=1e-11,
                      precision=sx.FP64, max_iter=20000)
    wt = torch.from_numpy(g.w).to(dev()).requires_grad_(True)
    target = torch.from_numpy(graphgen.normal_block(g.n, 4, 3) / np.sqrt(g.n)).to(dev())
    lam, V = sx.EigFn.apply(wt, handle, rp, col, nev, opts, None)
    L, d = lap.dense(g.rowptr, g.col, g.w)
    bd = d if problem == sx.GENERALIZED else np.ones(g.n)
    Bt = torch.from_numpy(bd).to(dev())
    Vs = V[:, 1:5]
    sign = torch.sign(((Vs * Bt[:, None]) * target).sum(0)).detach()
    loss = lam[1:5].sum() + ((Vs * sign - target) ** 2).sum()
    loss.backward()
    grad = wt.grad.cpu().numpy()
    # dense reference with the same loss partials at the dense eigenpairs
    lam_d, V_d = eigen.smallest_dense(L, bd, nev)
    assert np.allclose(lam.detach().cpu().numpy(), lam_d, rtol=1e-9, atol=1e-13)
    sgn = np.sign(np.sum(V_d[:, 1:5] * bd[:, None] * target.cpu().numpy(), axis=0))
    gl = np.zeros(nev); gl[1:5] = 1.0
    gV = np.zeros((g.n, nev))
    gV[:, 1:5] = 2.0 * (V_d[:, 1:5] * sgn - target.cpu().numpy()) * sgn
    gd, _, _ = adjoint.grad_dense(g.rowptr, g.col, g.w, problem, nev, gl, gV)
    # autograd returns half of dl/dw_e on each of the two CSR entries
    assert np.abs(grad - 0.5 * gd).max() <= 1e-5 * np.abs(gd).max()


@pytest.mark.parametrize("problem", [sx.COMBINATORIAL, sx.GENERALIZED])
def test_central_differences_eigenvalue_loss(handle, problem):
    g = graphgen.rmat_graph(10, seed=4, weight_seed=5, weight_dtype=np.float64)
    rp, col, _ = upload(g)
    nev = 5
    opts = sx.Options(problem=problem, precond=sx.PRECOND_JACOBI, tol=1e-12,
                      precision=sx.FP64, max_iter=50000)

    def loss_at(wv):
        G = sx.Graph(handle, rp, col, torch.from_numpy(wv).to(dev()), validate=False)
        lam, V, st = sx.eigensolve(handle, G, nev, opts)
        return float(np.sum(lam[1:5])), lam, V
    base, lam, V = loss_at(g.w)
    G = sx.Graph(handle, rp, col, torch.from_numpy(g.w).to(dev()))
    gl = np.zeros(nev); gl[1:5] = 1.0
    grad = sx.eig_backward(handle, G, problem, lam, V, gl, None).cpu().numpy()
    und = _undirected(g)
    r = lap.row_index(g.rowptr)
    key = r * g.n + g.col
    mate = np.searchsorted(key, g.col.astype(np.int64) * g.n + r)
    delta = np.random.default_rng(2).standard_normal(g.nnz)
    delta = 0.5 * (delta + delta[mate])             # symmetric direction
    h = 1e-6
    fp, _, _ = loss_at(g.w + h * delta)
    fm, _, _ = loss_at(g.w - h * delta)
    fd = (fp - fm) / (2 * h)
    an = float(np.sum(grad[und] * delta[und]))
    assert fd == pytest.approx(an, rel=1e-5, abs=1e-9)


def test_homogeneity_identities_full_size_grid(handle):
    g = _c5_like(128)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    und = _undirected(g)
    for problem in (sx.COMBINATORIAL, sx.GENERALIZED):
        opts = sx.Options(problem=problem, precond=sx.PRECOND_JACOBI, tol=1e-9,
                          precision=sx.FP64, max_iter=50000)
        lam, V, st = sx.eigensolve(handle, G, 3, opts)
        from tests.test_gpu_eigensolve import check_rayleigh
        check_rayleigh(g, problem, lam, V.cpu().numpy(), 1e-10)
        for k in (1, 2):
            e = np.zeros(3); e[k] = 1.0
            grad = sx.eig_backward(handle, G, problem, lam, V, e, None).cpu().numpy()
            s = float(g.w[und] @ grad[und])
            expect = lam[k] if problem == sx.COMBINATORIAL else 0.0
            assert abs(s - expect) <= 1e-8 * lam[k]
