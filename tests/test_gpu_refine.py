"""Greedy refinement (Sec. 7, balance of Sec. 3.1) on the GPU against the
oracle: bit-exact part vectors, pass and move counts, exact cut and
imbalance; and warm-start repartitioning (Sec. 1) with the previous
eigenvectors as the initial block."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from oracle import eigen, laplacian as lap, quality, refine
from tests.gpu_util import dev, random_graph, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


def _check(handle, g, part0, K, eps, vw=None, passes=8, wdtype=None):
    rp, col, w = upload(g, wdtype=wdtype)
    vwd = None if vw is None else torch.from_numpy(vw.astype(np.int32)).to(dev())
    G = sx.Graph(handle, rp, col, w, vwgt=vwd)
    pd = torch.from_numpy(np.asarray(part0, dtype=np.int32)).to(dev())
    cut, imb, kept, moves = sx.refine(handle, G, pd, K, eps=eps, max_passes=passes)
    wo = None if g.w is None else (g.w if wdtype is None else g.w.astype(wdtype))
    ref, kept_ref, moves_ref = refine.refine(g.rowptr, g.col, wo, part0, K, vwgt=vw, eps=eps,
                                             passes=passes)
    got = pd.cpu().numpy()
    assert np.array_equal(got, ref)
    assert (kept, moves) == (kept_ref, moves_ref)
    assert cut == quality.cutsize(g.rowptr, g.col, wo, ref)[0]
    assert imb == quality.imbalance(ref, K, vw)
    return got, kept, moves


@pytest.mark.parametrize("wd", [None, np.float32, np.float64])
@pytest.mark.parametrize("K,eps", [(2, 0.3), (3, 0.01), (7, 0.1), (40, 0.5)])
def test_refine_random_partition_matches_oracle(handle, wd, K, eps):
    g = random_graph(1500, 0.006, 5, wd)
    part0 = np.random.default_rng(K).integers(0, K, g.n).astype(np.int32)
    _, kept, moves = _check(handle, g, part0, K, eps)
    assert kept >= 1 and moves > 0


@pytest.mark.parametrize("K", [3, 16])
def test_refine_weighted_vertices(handle, K):
    g = random_graph(2000, 0.004, 8, np.float32)
    rng = np.random.default_rng(K + 1)
    vw = rng.integers(1, 9, g.n)
    part0 = rng.integers(0, K, g.n).astype(np.int32)
    _check(handle, g, part0, K, 0.05, vw=vw)


def test_refine_mid_and_high_degree_rows(handle):
    """R-MAT rows of degree 33..2048 take the block-per-row path; a star hub of
    degree 3000 never moves (both sides)."""
    r = graphgen.rmat_graph(11, seed=3)
    leaves = 3000
    n = r.n + leaves + 1
    iu = np.repeat(np.arange(r.n), np.diff(r.rowptr))
    keep = iu < r.col
    u = np.concatenate([iu[keep], np.full(leaves, r.n), np.arange(r.n + 1, n - 1),
                        [0]])
    v = np.concatenate([r.col[keep], np.arange(r.n + 1, n), np.arange(r.n + 2, n),
                        [r.n]])
    g = graphgen.csr_from_edges(n, u, v)
    deg = np.diff(g.rowptr)
    assert deg.max() > 2048 and np.count_nonzero((deg > 32) & (deg <= 2048)) > 10
    part0 = np.random.default_rng(1).integers(0, 5, g.n).astype(np.int32)
    got, _, _ = _check(handle, g, part0, 5, 0.2)
    assert got[r.n] == part0[r.n]


def test_refine_exact_fixed_point_decision(handle):
    # vertex 0 (part 0): edge 1 to part 0, edges 1, 2^-24, 2^-24 to part 1,
    # whose vertices form a triangle of unit edges (so they stay): the gain of
    # 0 is 2^-23 exactly (a float32 sum in CSR order would round it away), and
    # 0 moves on both sides
    u = np.array([0, 0, 0, 0, 2, 2, 3])
    v = np.array([1, 2, 3, 4, 3, 4, 4])
    w = np.array([1.0, 1.0, 2.0 ** -24, 2.0 ** -24, 1.0, 1.0, 1.0], dtype=np.float32)
    g = graphgen.csr_from_edges(5, u, v, w)
    tgt, gain = refine.gains(g.rowptr, g.col, g.w, [0, 0, 1, 1, 1])
    assert tgt == [1, -1, -1, -1, -1]
    got, kept, moves = _check(handle, g, np.array([0, 0, 1, 1, 1]), 2, 1.0)
    assert got.tolist() == [1, 0, 1, 1, 1] and (kept, moves) == (1, 1)


def test_refine_balance_prefix(handle):
    n = 14
    g = graphgen.csr_from_edges(n, np.zeros(13, dtype=int), np.arange(1, 14))
    part = np.array([0] + [1] * 6 + [0] * 7, dtype=np.int32)
    vw = np.array([1, 1, 2, 1, 1, 1, 1] + [1] * 7)
    got, kept, moves = _check(handle, g, part, 2, 0.3, vw=vw, passes=1)
    assert moves == 1 and got[1] == 0 and got[3] == 1


def test_refine_no_passes_and_errors(handle):
    g = random_graph(300, 0.02, 2)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    p0 = np.random.default_rng(0).integers(0, 4, g.n).astype(np.int32)
    pd = torch.from_numpy(p0).to(dev())
    cut, imb, kept, moves = sx.refine(handle, G, pd, 4, max_passes=0)
    assert (kept, moves) == (0, 0) and np.array_equal(pd.cpu().numpy(), p0)
    assert cut == quality.cutsize(g.rowptr, g.col, None, p0)[0]
    bad = pd.clone()
    bad[7] = 4
    with pytest.raises(sx.SphynxError):
        sx.refine(handle, G, bad, 4)
    with pytest.raises(sx.SphynxError):
        sx.refine(handle, G, pd, 4, eps=-0.1)


@pytest.mark.parametrize("name,K", [("rmat11", 16), ("grid64", 4)])
def test_refine_spectral_partition(handle, name, K):
    """Refinement of the GPU's own spectral partition equals the oracle's
    refinement of the same part vector."""
    g = graphgen.rmat_graph(11, seed=3) if name == "rmat11" else graphgen.config_graph("grid64")
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    reg, _, _ = G.info()
    opts = sx.options_default(reg, sx.PRECOND_JACOBI, precision=sx.FP64, seed=4)
    lam, V, part, cut0, imb0, st = sx.partition(handle, G, K, opts)
    part0 = part.cpu().numpy()
    cut, imb, kept, moves = sx.refine(handle, G, part, K, eps=0.01)
    ref, kept_ref, moves_ref = refine.refine(g.rowptr, g.col, None, part0, K, eps=0.01)
    assert np.array_equal(part.cpu().numpy(), ref)
    assert (kept, moves) == (kept_ref, moves_ref)
    assert cut <= cut0 and imb < 1.01


@pytest.mark.parametrize("graph,K", [("brick100", 24), ("rmat22", 16)])
def test_refine_full_size_properties(handle, graph, K):
    """Full-size spectral partitions: the refined cut equals the oracle's cut
    of the returned vector, never exceeds the spectral cut, and every part
    that grew stays within the capacity."""
    g = graphgen.config_graph(graph)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    reg, _, _ = G.info()
    pc = sx.PRECOND_JACOBI if graph == "brick100" else sx.PRECOND_CHEBYSHEV
    opts = sx.options_default(reg, pc, precision=sx.MIXED, seed=5)
    lam, V, part, cut0, imb0, st = sx.partition(handle, G, K, opts)
    p0 = part.cpu().numpy()
    eps = 0.01
    cut, imb, kept, moves = sx.refine(handle, G, part, K, eps=eps)
    p1 = part.cpu().numpy()
    assert cut == quality.cutsize(g.rowptr, g.col, None, p1)[0]
    assert imb == quality.imbalance(p1, K)
    assert cut <= cut0
    if kept:
        assert cut < cut0 and moves > 0
    cap = refine.capacity(g.n, K, eps)
    W0 = np.bincount(p0, minlength=K)
    W1 = np.bincount(p1, minlength=K)
    assert np.all(W1 <= np.maximum(W0, cap))
    assert np.count_nonzero(p0 != p1) <= moves


# ---- warm-start repartitioning

@pytest.mark.parametrize("problem", [sx.COMBINATORIAL, sx.GENERALIZED, sx.NORMALIZED])
def test_warm_start_repartition(handle, problem):
    """Weights change by up to 1 %: the solve started from the previous
    eigenvectors converges in fewer iterations to the eigenpairs of the new
    graph (dense oracle), and its partition matches the oracle split."""
    n0, (u, v) = graphgen.grid2d_9pt(24, 20)
    g0 = graphgen.csr_from_edges(n0, u, v, graphgen.uniform_weights(u.size, 3,
                                                                     dtype=np.float64))
    g1 = graphgen.perturb_weights(g0, 0.01, 4)
    K = 8
    nev = sx.num_eigenvectors(K)
    opts = sx.Options(problem=problem, precond=sx.PRECOND_JACOBI, tol=1e-8,
                      precision=sx.FP64, seed=9, max_iter=5000)
    rp, col, w = upload(g0)
    G0 = sx.Graph(handle, rp, col, w)
    lam0, V0, part0, _, _, st0 = sx.partition(handle, G0, K, opts)
    rp1, col1, w1 = upload(g1)
    G1 = sx.Graph(handle, rp1, col1, w1)
    lam_c, V_c, part_c, _, _, st_cold = sx.partition(handle, G1, K, opts)
    opts.init = sx.INIT_USER
    lam1, V1, part1, cut1, imb1, st1 = sx.partition(handle, G1, K, opts, X0=V0)
    assert st1.iterations < st_cold.iterations
    if problem == sx.NORMALIZED:
        L = lap.dense_normalized(g1.rowptr, g1.col, g1.w)
        bd = np.ones(g1.n)
    else:
        L, d = lap.dense(g1.rowptr, g1.col, g1.w)
        bd = d if problem == sx.GENERALIZED else np.ones(g1.n)
    lam_ref, _ = eigen.smallest_dense(L, bd, nev + 1)
    assert abs(lam1[0]) <= 1e-7 * lam_ref[1]
    assert np.allclose(lam1[1:], lam_ref[1:nev], rtol=1e-7, atol=0)
    from oracle import split
    ref = split.split_mj(V1.cpu().numpy()[:, 1:], K)
    assert np.array_equal(part1.cpu().numpy(), ref)
