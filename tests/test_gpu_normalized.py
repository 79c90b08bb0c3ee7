"""The normalized problem L_N y = lambda y on the GPU against the oracle:
the L_N product, the preconditioners (Jacobi is the identity, Chebyshev runs
on L_N), the eigenpairs against a dense L_N solve, the adjoint against the
dense per-edge formula, and the full-size R-MAT workload with the paper's
default for irregular graphs with a polynomial preconditioner."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from oracle import adjoint, eigen, laplacian as lap, precond, split, quality
from tests.gpu_util import dev, random_graph, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


def _graph(wd=np.float64):
    return random_graph(300, 0.02, 31, wd)


@pytest.mark.parametrize("dtype,m", [(torch.float64, 1), (torch.float64, 4), (torch.float64, 5),
                                     (torch.float32, 4), (torch.float32, 3)])
def test_normalized_product_matches_oracle(handle, dtype, m):
    g = _graph()
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    X = graphgen.normal_block(g.n, m, 3)
    npd = np.float32 if dtype == torch.float32 else np.float64
    Xd = torch.from_numpy(X.astype(npd)).to(dev())
    Y = sx.laplacian_apply(handle, G, Xd, problem=sx.NORMALIZED).cpu().numpy()
    ref = lap.apply_normalized(g.rowptr, g.col, g.w, X.astype(npd).astype(np.float64))
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert np.abs(Y - ref).max() <= tol * np.abs(X).max() * 4
    # D^1/2 1 is in the kernel
    s = np.sqrt(lap.degrees(g.rowptr, g.col, g.w))
    Z = sx.laplacian_apply(handle, G, torch.from_numpy(s[:, None].copy()).to(dev()),
                           problem=sx.NORMALIZED).cpu().numpy()
    assert np.abs(Z).max() < 1e-13 * s.max()


def test_normalized_product_rejects_isolated_vertex(handle):
    g = graphgen.csr_from_edges(4, np.array([0, 1]), np.array([1, 2]))   # vertex 3 isolated
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    with pytest.raises(sx.SphynxError):
        sx.laplacian_apply(handle, G, torch.ones(4, 1, dtype=torch.float64, device=dev()),
                           problem=sx.NORMALIZED)


def test_normalized_preconditioners_match_oracle(handle):
    g = _graph()
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    R = graphgen.normal_block(g.n, 4, 9)
    Rd = torch.from_numpy(R).to(dev())
    J = sx.precond_apply(handle, G, sx.Options(problem=sx.NORMALIZED, precond=sx.PRECOND_JACOBI),
                         Rd).cpu().numpy()
    assert np.array_equal(J, R)                 # diag(L_N) = I
    deg, ratio = 25, 30.0
    opts = sx.Options(problem=sx.NORMALIZED, precond=sx.PRECOND_CHEBYSHEV, cheb_degree=deg,
                      cheb_ratio=ratio)
    H = sx.precond_apply(handle, G, opts, Rd).cpu().numpy()
    ref = precond.chebyshev(g.rowptr, g.col, g.w, R, deg, 2.0 / ratio, 2.0,
                            problem=lap.NORMALIZED)
    assert np.abs(H - ref).max() <= 1e-10 * np.abs(ref).max()


CASES = [(pc, prec) for pc in (sx.PRECOND_JACOBI, sx.PRECOND_CHEBYSHEV)
         for prec in (sx.FP64, sx.MIXED)]


@pytest.mark.parametrize("pc,prec", CASES)
def test_normalized_eigenpairs_vs_dense(handle, pc, prec):
    g = _graph(np.float64 if prec == sx.FP64 else np.float32)
    wo = g.w.astype(np.float64)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    nev = 5
    LN = lap.dense_normalized(g.rowptr, g.col, wo)
    lam_ref, Y_ref = eigen.smallest_dense(LN, np.ones(g.n), nev + 1)
    # FP32 vectors: the relative residual floor is near 1e-5 on this graph
    tol = 1e-9 if prec == sx.FP64 else 1e-4
    opts = sx.Options(problem=sx.NORMALIZED, precond=pc, tol=tol, precision=prec, seed=7,
                      cheb_degree=10, cheb_ratio=30.0, max_iter=5000)
    lam, Y, st = sx.eigensolve(handle, G, nev, opts)
    rel = 1e-6 if prec == sx.FP64 else 1e-4
    assert abs(lam[0]) <= rel * lam_ref[1]
    assert np.allclose(lam[1:], lam_ref[1:nev], rtol=rel, atol=0), (lam, lam_ref)
    Yh = Y.cpu().numpy().astype(np.float64)
    # unit 2-norm, orthonormal, Rayleigh quotients of the oracle L_N
    assert np.allclose(Yh.T @ Yh, np.eye(nev), atol=1e-10 if prec == sx.FP64 else 1e-5)
    rq = np.sum(Yh * lap.apply_normalized(g.rowptr, g.col, wo, Yh), axis=0)
    assert np.allclose(rq, lam, rtol=1e-9 if prec == sx.FP64 else 1e-5,
                       atol=1e-9 if prec == sx.FP64 else 1e-6 * lam_ref[nev - 1])
    gap = lam_ref[nev] - lam_ref[nev - 1]
    if np.sqrt(nev) * tol * lam_ref[nev - 1] / gap < 1e-4:
        assert eigen.subspace_sin(Yh, Y_ref[:, :nev], np.ones(g.n)) < 1e-3
    for k in range(nev):
        i = int(np.argmax(np.abs(Yh[:, k])))
        assert Yh[i, k] > 0
    # the trivial vector is D^1/2 1 / ||D^1/2 1||
    s = np.sqrt(lap.degrees(g.rowptr, g.col, wo))
    assert np.abs(Yh[:, 0] - s / np.linalg.norm(s)).max() < (1e-8 if prec == sx.FP64 else 1e-4)


def test_normalized_and_generalized_share_eigenvalues(handle):
    g = graphgen.rmat_graph(11, seed=3)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    reg, _, _ = G.info()
    opts = sx.options_default(reg, sx.PRECOND_CHEBYSHEV, tol=1e-8, precision=sx.FP64)
    assert opts.problem == sx.NORMALIZED          # irregular + polynomial (Sec. 6.3.1)
    lam_n, Y, _ = sx.eigensolve(handle, G, 4, opts)
    opts.problem = sx.GENERALIZED
    lam_g, X, _ = sx.eigensolve(handle, G, 4, opts)
    assert np.allclose(lam_n[1:], lam_g[1:], rtol=1e-7)


@pytest.mark.parametrize("with_vecs", [False, True])
def test_normalized_adjoint_vs_dense(handle, with_vecs):
    g = random_graph(60, 0.08, 13, np.float64)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    nev = 4
    rng = np.random.default_rng(5)
    a = rng.standard_normal(nev)
    C = rng.standard_normal((g.n, nev)) if with_vecs else None
    ref, lam, Y = adjoint.grad_dense_normalized(g.rowptr, g.col, g.w, nev, a, C)
    Yd = torch.from_numpy(Y.copy()).to(dev())
    Cd = None if C is None else torch.from_numpy(C).to(dev())
    grad = sx.eig_backward(handle, G, sx.NORMALIZED, lam, Yd, a, Cd).cpu().numpy()
    assert np.allclose(grad, ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("prec", [sx.MIXED, sx.FP64])
def test_rmat22_normalized_chebyshev_k16(handle, prec):
    """R-MAT scale 22 (LCC), the default for irregular graphs with a polynomial
    preconditioner (normalized problem, piecewise start, tol 1e-2), K = 16."""
    g = graphgen.config_graph("rmat22")
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    reg, _, _ = G.info()
    opts = sx.options_default(reg, sx.PRECOND_CHEBYSHEV, precision=prec)
    assert opts.problem == sx.NORMALIZED
    lam, Y, part, cut, imb, st = sx.partition(handle, G, 16, opts)
    Y = Y.cpu().numpy().astype(np.float64)
    part = part.cpu().numpy()
    LY = lap.apply_normalized_sparse(g.rowptr, g.col, None, Y)
    nrm = np.sum(Y * Y, axis=0)
    rq = np.sum(Y * LY, axis=0) / nrm
    assert np.allclose(nrm, 1.0, atol=1e-5)
    assert np.allclose(rq, lam, rtol=1e-6, atol=1e-9)
    rho = lap.residual_norms(LY, Y, np.asarray(lam), np.ones(g.n))
    assert rho.max() <= 1e-2 * (1.5 if prec == sx.MIXED else 1.0 + 1e-6)
    ref = split.split_pow2(Y[:, 1:], 16)     # exact widening of the GPU's coordinates
    assert np.array_equal(part, ref)
    c_ref, _ = quality.cutsize(g.rowptr, g.col, None, ref)
    assert cut == c_ref
    assert imb == quality.imbalance(ref, 16)
