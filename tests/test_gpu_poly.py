"""GMRES polynomial preconditioner (Sec. 5.2) on the GPU against the oracle:
the roots from the same start vector, the apply with the same roots, and
LOBPCG with this preconditioner against dense eigenpairs and the closed form."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from oracle import eigen, laplacian as lap, precond
from tests import closed_forms as cf
from tests.gpu_util import dev, random_graph, upload

pytestmark = pytest.mark.gpu

PROBLEMS = {sx.COMBINATORIAL: lap.COMBINATORIAL, sx.GENERALIZED: lap.GENERALIZED,
            sx.NORMALIZED: lap.NORMALIZED}


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


def _graphs():
    n, (u, v) = graphgen.grid2d_9pt(32, 32)
    king = graphgen.csr_from_edges(n, u, v, graphgen.uniform_weights(u.size, 2, dtype=np.float64))
    return {"rand_f64": random_graph(400, 0.02, 5, np.float64),
            "rmat11": graphgen.rmat_graph(11, seed=3),
            "king32": king}


GRAPHS = _graphs()


def _upload(g):
    rp, col, w = upload(g)
    return rp, col, w


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("problem", list(PROBLEMS))
@pytest.mark.parametrize("degree", [8, 25])
def test_poly_roots_match_oracle(handle, name, problem, degree):
    g = GRAPHS[name]
    rp, col, w = _upload(g)
    G = sx.Graph(handle, rp, col, w)
    b = graphgen.normal_block(g.n, 1, 11)[:, 0]
    ref = precond.gmres_poly_roots(g.rowptr, g.col, g.w, PROBLEMS[problem], b, degree)
    got = sx.poly_roots(handle, G, problem, degree, torch.from_numpy(b).to(dev()))
    assert got.size == ref.size == degree + 1
    assert np.allclose(np.sort(got), np.sort(ref), rtol=1e-7, atol=0)
    assert got[0] == pytest.approx(ref[0], rel=1e-7)      # Leja order starts at the largest


@pytest.mark.parametrize("problem", list(PROBLEMS))
@pytest.mark.parametrize("dtype,m", [(torch.float64, 1), (torch.float64, 4), (torch.float64, 7),
                                     (torch.float32, 3), (torch.float32, 8)])
def test_poly_apply_matches_oracle(handle, problem, dtype, m):
    g = GRAPHS["rand_f64"]
    rp, col, w = _upload(g)
    G = sx.Graph(handle, rp, col, w)
    b = graphgen.normal_block(g.n, 1, 12)[:, 0]
    roots = precond.gmres_poly_roots(g.rowptr, g.col, g.w, PROBLEMS[problem], b, 12)
    R = graphgen.normal_block(g.n, m, 13)
    npd = np.float32 if dtype == torch.float32 else np.float64
    Rd = torch.from_numpy(R.astype(npd)).to(dev())
    H = sx.poly_apply(handle, G, problem, roots, Rd).cpu().numpy().astype(np.float64)
    ref = precond.gmres_poly_apply(g.rowptr, g.col, g.w, PROBLEMS[problem],
                                   R.astype(npd).astype(np.float64), roots)
    tol = 1e-10 if dtype == torch.float64 else 2e-4
    assert np.abs(H - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("problem", list(PROBLEMS))
@pytest.mark.parametrize("prec", [sx.FP64, sx.MIXED])
def test_eigensolve_gmres_vs_dense(handle, problem, prec):
    g = random_graph(400, 0.015, 21, np.float64 if prec == sx.FP64 else np.float32)
    wo = g.w.astype(np.float64)
    rp, col, w = _upload(g)
    G = sx.Graph(handle, rp, col, w)
    nev = 5
    if problem == sx.NORMALIZED:
        L = lap.dense_normalized(g.rowptr, g.col, wo)
        bd = np.ones(g.n)
    else:
        L, d = lap.dense(g.rowptr, g.col, wo)
        bd = d if problem == sx.GENERALIZED else np.ones(g.n)
    lam_ref, V_ref = eigen.smallest_dense(L, bd, nev + 1)
    tol = 1e-9 if prec == sx.FP64 else 1e-4
    opts = sx.Options(problem=problem, precond=sx.PRECOND_GMRES, cheb_degree=10, tol=tol,
                      precision=prec, seed=7, max_iter=5000)
    lam, V, st = sx.eigensolve(handle, G, nev, opts)
    rel = 1e-6 if prec == sx.FP64 else 1e-4
    assert abs(lam[0]) <= rel * lam_ref[1]
    assert np.allclose(lam[1:], lam_ref[1:nev], rtol=rel, atol=0), (lam, lam_ref)
    Vh = V.cpu().numpy().astype(np.float64)
    assert np.allclose(Vh.T @ (bd[:, None] * Vh), np.eye(nev),
                       atol=1e-10 if prec == sx.FP64 else 1e-5)
    gap = lam_ref[nev] - lam_ref[nev - 1]
    if np.sqrt(nev) * tol * lam_ref[nev - 1] / gap < 1e-4:
        assert eigen.subspace_sin(Vh, V_ref[:, :nev], bd) < 1e-3


@pytest.mark.parametrize("prec", [sx.MIXED, sx.FP64])
def test_grid128_gmres_polynomial_k64(handle, prec):
    """The benchmark grid with the paper's polynomial (GMRES, degree 25)."""
    g = graphgen.config_graph("grid7_128")
    rp, col, w = _upload(g)
    G = sx.Graph(handle, rp, col, w)
    opts = sx.options_default(True, sx.PRECOND_GMRES, precision=prec, seed=12345)
    lam, V, st = sx.eigensolve(handle, G, 7, opts)
    exact = cf.grid_eigvals((128, 128, 128), 8)
    rel = 1e-4 if prec == sx.MIXED else 1e-6
    assert abs(lam[0]) < rel * exact[1]
    assert np.allclose(lam[1:], exact[1:7], rtol=rel, atol=0)
    assert max(st.rho) <= 1e-3 * (1.5 if prec == sx.MIXED else 1.0 + 1e-6)
