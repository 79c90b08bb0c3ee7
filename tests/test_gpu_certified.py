"""GPU eigenpairs against the oracle's certified eigenpairs at full size.

Workloads (tests/golden/certified_<name>.json, written by
tests/golden/make_certified.py from graphgen + oracle only):
* rmat22: R-MAT scale 22 LCC, generalized problem, Jacobi, K = 16 (d = 5),
  MIXED and FP64;
* brick96lr: 27-point 96^3 + 1 % long-range edges, FP32 weights U[0.5, 1.5),
  combinatorial, Jacobi, K = 256 (d = 9), MIXED and FP64;
* king512, rmat18: the differentiation workloads (weights U[0.5, 1.5) FP64,
  generalized, 7 eigenpairs), FP64.

Gates: eigenvalues within 1e-6 relative (FP64) or 1e-4 (MIXED) of the
certified interval of the exact eigenvalue; for every leading block whose
certified separation is at least `gap` of its next eigenvalue, the
Davis-Kahan bound of the GPU basis (its own residual, FP64, oracle operator)
at most 1e-3.  The solver tolerance of each case is tighter than the
workload's default so that these accuracies are reachable: eigenvalue error
is quadratic and the subspace error linear in the residual over the gap.
For C3/C4 the part vector and its cut / imbalance are also checked against
the oracle split of the GPU's coordinates, bit for bit.
"""
import numpy as np
import pytest

import graphgen
import paper_2105_00578_amd as sx
from oracle import quality, split
from tests import certified
from tests.gpu_util import upload

pytestmark = pytest.mark.gpu

# gap = None: no subspace gate.  R-MAT 22's generalized spectrum is one tight
# cluster (theta_1..theta_8 within 0.4 %, the block edge lambda_5 - theta_4 =
# 1.3e-5, relative 7e-5): FP32 vectors (residual floor near 1e-6 relative) can
# reach the eigenvalue accuracy but no subspace of it is certifiable at 1e-3,
# so angle parity is unpinned there in mixed precision.
CASES = [
    # name, precision, K (None: eigensolve of nev), nev, precond, tol, rel, gap
    ("rmat22", sx.FP64, 16, 5, sx.PRECOND_JACOBI, 1e-8, 1e-6, 5e-5),
    ("rmat22", sx.MIXED, 16, 5, sx.PRECOND_JACOBI, 1e-5, 1e-4, None),
    ("brick96lr", sx.FP64, 256, 9, sx.PRECOND_JACOBI, 1e-7, 1e-6, 5e-4),
    ("brick96lr", sx.MIXED, 256, 9, sx.PRECOND_JACOBI, 1e-5, 1e-4, 3e-2),
    ("king512", sx.FP64, None, 7, sx.PRECOND_CHEBYSHEV, 1e-8, 1e-6, 2e-3),
    ("rmat18", sx.FP64, None, 7, sx.PRECOND_JACOBI, 1e-8, 1e-6, 1e-3),
]

_GRAPHS = {}


def _graph(name):
    if name not in _GRAPHS:
        _GRAPHS.clear()                     # one large graph resident at a time
        _GRAPHS[name] = graphgen.config_graph(name)
    return _GRAPHS[name]


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


@pytest.mark.parametrize("name,prec,K,nev,pre,tol,rel,gap", CASES,
                         ids=[f"{c[0]}-{'fp64' if c[1] == sx.FP64 else 'mixed'}" for c in CASES])
def test_certified_eigenpairs(handle, name, prec, K, nev, pre, tol, rel, gap):
    gold = certified.load(name)
    g = _graph(name)
    assert (g.n, g.nnz) == (gold["n"], gold["nnz"])
    assert certified.digest(g) == gold["sha256"], "graph differs from the certified one"
    problem = {"combinatorial": sx.COMBINATORIAL, "generalized": sx.GENERALIZED}[gold["problem"]]
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    reg, _, _ = G.info()
    opts = sx.options_default(reg, pre, precision=prec, problem=problem, tol=tol,
                              max_iter=50000)
    if K is None:
        lam, V, st = sx.eigensolve(handle, G, nev, opts)
        part = None
    else:
        lam, V, part, cut, imb, st = sx.partition(handle, G, K, opts)
    Vh = V.cpu().numpy()
    err = certified.eigenvalue_errors(gold, lam)
    blocks = [] if gap is None else certified.separated_blocks(gold, gap, kmax=nev)
    sins = certified.subspace_bounds(g, gold, Vh, blocks)
    print(f"\n{name} {'FP64' if prec == sx.FP64 else 'MIXED'} tol {tol}: "
          f"{st.iterations} its (promoted {st.promoted}), max rel eig err {err.max():.3e}, "
          f"blocks {blocks} sin bounds {[f'{s:.2e}' for s in sins.values()]}", flush=True)
    assert err.max() <= rel, (err, lam, gold["theta"][:nev])
    if gap is not None:
        assert blocks, "no separated block to certify"
        assert max(sins.values()) <= 1e-3, sins
    if part is not None:
        part = part.cpu().numpy()
        ref = split.split_mj(Vh[:, 1:], K) if K & (K - 1) else split.split_pow2(Vh[:, 1:], K)
        assert np.array_equal(part, ref)
        c_ref, _ = quality.cutsize(g.rowptr, g.col, g.w, ref)
        assert cut == c_ref and imb == quality.imbalance(ref, K)
