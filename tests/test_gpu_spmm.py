"""Laplacian product and preconditioners: GPU vs the FP64 oracle.

FP64 and FP32 results are checked componentwise against the a-priori
rounding bound of a difference-form row sum: |y_i - yhat_i| <=
(deg_i + 3) u sum_j w_ij |x_i - x_j| (u the unit roundoff of the precision;
the oracle evaluates the same rounded inputs in FP64).  Jacobi is one
correctly rounded division on both sides, so it must be bit-exact.
"""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from oracle import laplacian as lap, precond
from tests.gpu_util import dev, random_graph, star_graph, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


def _grid(nx, ny):
    n, (u, v) = graphgen.grid2d_5pt(nx, ny)
    return graphgen.csr_from_edges(n, u, v)


def _king(side, wd):
    n, (u, v) = graphgen.grid2d_9pt(side, side)
    return graphgen.csr_from_edges(n, u, v, graphgen.uniform_weights(u.size, 0, dtype=wd))


def _graphs():
    return {
        "grid_unit": _grid(37, 29),
        "rand_f32": random_graph(700, 0.02, 3, np.float32),
        "rand_f64": random_graph(500, 0.03, 4, np.float64),
        "star_hub": star_graph(40000),                 # hub row > 16384 entries
        "rmat12": graphgen.rmat_graph(12, seed=5),      # mid-degree rows
        "brick_lr": graphgen.config_graph("brick96lr", scale_down=12),
        "king64_f64": _king(64, np.float64),          # weighted, > 1024 rows
        "brick24_lr": graphgen.config_graph("brick96lr", scale_down=4),   # F32, 13824 rows
    }


GRAPHS = _graphs()


def _bound(g, X, eps):
    r = lap.row_index(g.rowptr)
    ww = np.ones(g.nnz) if g.w is None else g.w.astype(np.float64)
    s = np.zeros_like(X)
    np.add.at(s, r, ww[:, None] * np.abs(X[r] - X[g.col]))
    deg = np.diff(g.rowptr)[:, None]
    return (deg + 3) * eps * s + 1e-300


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("m", [1, 3, 4, 7, 8, 16])
def test_spmm_matches_oracle(handle, name, dtype, m):
    g = GRAPHS[name]
    rp64 = name in ("rand_f64", "star_hub")
    # FP32 vectors use FP32 weights; FP64 vectors the graph's own (or FP64)
    wd = None if g.w is None else (np.float32 if dtype == torch.float32 else np.float64)
    rp, col, w = upload(g, rowptr64=rp64, wdtype=wd)
    G = sx.Graph(handle, rp, col, w)
    X = graphgen.normal_block(g.n, m, 11 + m).astype(np.float32 if dtype == torch.float32 else np.float64)
    Y = sx.laplacian_apply(handle, G, torch.from_numpy(X).to(dev())).cpu().numpy()
    wo = None if g.w is None else g.w.astype(wd).astype(np.float64)
    ref = lap.apply(g.rowptr, g.col, wo, X.astype(np.float64))
    eps = 2.0 ** -24 if dtype == torch.float32 else 2.0 ** -53
    gg = graphgen.Graph(g.n, g.rowptr, g.col, wo)
    err = np.abs(Y.astype(np.float64) - ref)
    assert np.all(err <= _bound(gg, X.astype(np.float64), eps)), err.max()
    # constant vectors map to exact zeros (difference form)
    C = torch.full((g.n, m), 0.3721, dtype=dtype, device=dev())
    assert torch.count_nonzero(sx.laplacian_apply(handle, G, C)) == 0


def test_spmm_deterministic(handle):
    g = GRAPHS["rmat12"]
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    X = torch.from_numpy(graphgen.normal_block(g.n, 5, 1).astype(np.float32)).to(dev())
    a = sx.laplacian_apply(handle, G, X)
    b = sx.laplacian_apply(handle, G, X)
    assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("name", ["rand_f64", "star_hub", "grid_unit", "king64_f64",
                                  "brick24_lr"])
def test_jacobi_bit_exact(handle, dtype, name):
    g = GRAPHS[name]
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    npd = np.float32 if dtype == torch.float32 else np.float64
    R = graphgen.normal_block(g.n, 5, 7).astype(npd)
    opts = sx.Options(precond=sx.PRECOND_JACOBI)
    H = sx.precond_apply(handle, G, opts, torch.from_numpy(R).to(dev())).cpu().numpy()
    d = lap.degrees(g.rowptr, g.col, g.w)
    ref = precond.jacobi(R.astype(np.float64), d).astype(npd)
    assert np.array_equal(H, ref)


@pytest.mark.parametrize("problem", [sx.COMBINATORIAL, sx.GENERALIZED])
@pytest.mark.parametrize("name", ["rand_f64", "rmat12", "brick_lr"])
def test_chebyshev_matches_oracle(handle, problem, name):
    g = GRAPHS[name]
    wd = None if g.w is None else np.float64
    rp, col, w = upload(g, wdtype=wd)
    G = sx.Graph(handle, rp, col, w)
    wo = None if g.w is None else g.w.astype(np.float64)
    R = graphgen.normal_block(g.n, 4, 9)
    deg, ratio = 25, 30.0
    opts = sx.Options(precond=sx.PRECOND_CHEBYSHEV, problem=problem, cheb_degree=deg,
                      cheb_ratio=ratio)
    H = sx.precond_apply(handle, G, opts, torch.from_numpy(R).to(dev())).cpu().numpy()
    d = lap.degrees(g.rowptr, g.col, wo)
    hi = precond.gershgorin_bound(d, problem)
    dinv = 1.0 / d if problem == sx.GENERALIZED else None
    ref = precond.chebyshev(g.rowptr, g.col, wo, R, deg, hi / ratio, hi, dinv)
    scale = np.abs(ref).max()
    assert np.abs(H - ref).max() <= 1e-10 * scale


def test_spmm_full_size_grid128_sampled(handle):
    """3D 7-point 128^3 (the benchmark workload), m = 7, FP32: sampled rows vs
    the oracle row by row, plus exact zeros on a constant block."""
    g = graphgen.config_graph("grid7_128")
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w, validate=True)
    X = graphgen.normal_block(g.n, 7, 3).astype(np.float32)
    Y = sx.laplacian_apply(handle, G, torch.from_numpy(X).to(dev())).cpu().numpy()
    rows = np.random.default_rng(0).choice(g.n, 2000, replace=False)
    X64 = X.astype(np.float64)
    for i in rows:
        nb = g.col[g.rowptr[i]:g.rowptr[i + 1]]
        ref = (X64[i][None, :] - X64[nb]).sum(axis=0)
        bound = (len(nb) + 3) * 2.0 ** -24 * np.abs(X64[i][None, :] - X64[nb]).sum(axis=0)
        assert np.all(np.abs(Y[i] - ref) <= bound + 1e-300)
    C = torch.ones((g.n, 7), dtype=torch.float32, device=dev())
    assert torch.count_nonzero(sx.laplacian_apply(handle, G, C)) == 0


def _path_plus(n, extra):
    u = np.concatenate([np.arange(n - 1), [extra[0]]])
    v = np.concatenate([np.arange(1, n), [extra[1]]])
    return graphgen.csr_from_edges(n, u, v)


@pytest.mark.parametrize("case,bytes_", [("fits", 2), ("overflows", 4), ("permuted", 4),
                                         ("grid", 2)])
def test_int16_column_offsets(handle, case, bytes_):
    """Unit-weight graphs of at most 48 neighbours per row are read through
    int16 offsets from the row when every offset fits (|offset| <= 32767),
    else through the int32 columns; both give the oracle's product."""
    if case == "fits":
        g = _path_plus(40000, (5, 5 + 32767))
    elif case == "overflows":
        g = _path_plus(40000, (5, 5 + 32768))
    else:
        n, (u, v) = graphgen.grid3d_7pt(40, 40, 40)
        if case == "permuted":
            p = np.random.default_rng(2).permutation(n)
            u, v = p[u], p[v]
        g = graphgen.csr_from_edges(n, u, v)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    for dtype, m in ((torch.float32, 4), (torch.float32, 8), (torch.float64, 2)):
        X = graphgen.normal_block(g.n, m, 5).astype(np.float32 if dtype == torch.float32
                                                    else np.float64)
        Y = sx.laplacian_apply(handle, G, torch.from_numpy(X).to(dev())).cpu().numpy()
        ref = lap.apply(g.rowptr, g.col, None, X.astype(np.float64))
        eps = 2.0 ** -24 if dtype == torch.float32 else 2.0 ** -53
        assert np.all(np.abs(Y - ref) <= _bound(g, X.astype(np.float64), eps))
    opts = sx.Options(precond=sx.PRECOND_JACOBI, tol=1e-2, precision=sx.MIXED, max_iter=3)
    _, _, st = sx.eigensolve(handle, G, 3, opts, allow_not_converged=True)
    assert st.col_index_bytes == bytes_
