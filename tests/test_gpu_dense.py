"""Dense LOBPCG kernels alone: FP64-MFMA Gram products vs numpy, and the
one-workgroup Rayleigh-Ritz vs a library symmetric-definite eigensolver."""
import numpy as np
import pytest
import scipy.linalg
import torch

import paper_2105_00578_amd as sx
from paper_2105_00578_amd import _lib
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n,m,act,use_p,gen", [
    (1000, 3, [], False, False),
    (777, 5, [0, 2, 4], True, True),
    (5000, 7, [1, 2, 3, 4, 5, 6, 0], True, False),
    (333, 16, list(range(16)), True, True),
    (64, 9, [8], False, True),
    # two-tile widths: 17 and 21, 24 (the compact pair of tiles), 27 (three tiles)
    (4099, 7, [0, 1, 2, 3, 4], True, False),
    (6000, 7, [1, 2, 3, 4, 5, 6, 0], True, True),
    (2500, 8, list(range(8)), True, False),
    (3001, 9, list(range(9)), True, True),
])
def test_block_gram_vs_numpy(handle, dtype, n, m, act, use_p, gen):
    rng = np.random.default_rng(n + m)
    blocks = [rng.standard_normal((n, m)).astype(dtype) for _ in range(6)]
    X, LX, H, LH, P, LP = blocks
    b = rng.uniform(1, 5, n) if gen else None
    t = [torch.from_numpy(a).to(dev()) for a in blocks]
    use_h = len(act) > 0
    GA, GB = _lib.block_gram(handle, t[0], t[1], t[2] if use_h else None,
                             t[3] if use_h else None, t[4] if use_p and use_h else None,
                             t[5] if use_p and use_h else None, act,
                             None if b is None else torch.from_numpy(b).to(dev()))
    f = lambda a: a.astype(np.float64)
    S = [f(X)]
    LS = [f(LX)]
    if use_h:
        S.append(f(H)[:, act]); LS.append(f(LH)[:, act])
        if use_p:
            S.append(f(P)[:, act]); LS.append(f(LP)[:, act])
    S = np.hstack(S); LS = np.hstack(LS)
    bb = np.ones(n) if b is None else b
    refA = S.T @ LS
    refB = S.T @ (bb[:, None] * S)
    iu = np.triu_indices(S.shape[1])
    # an upper entry (i, j) of S^T L S may be formed as s_i . (L s)_j or as
    # s_j . (L s)_i (the same number for a symmetric L); these random blocks
    # make the two differ, so each entry must match one of them
    tol = 1e-12 * np.abs(refA).max()
    a, at = refA[iu], refA.T[iu]
    ok = np.isclose(GA[iu], a, rtol=1e-12, atol=tol) | np.isclose(GA[iu], at, rtol=1e-12, atol=tol)
    assert ok.all()
    assert np.allclose(GB[iu], refB[iu], rtol=1e-12, atol=1e-12 * np.abs(refB).max())


@pytest.mark.parametrize("w,m", [(3, 3), (9, 3), (15, 5), (21, 7), (27, 9), (48, 16)])
def test_rayleigh_ritz_vs_eigh(handle, w, m):
    rng = np.random.default_rng(w)
    Z = rng.standard_normal((200, w))
    GB = Z.T @ Z
    A = rng.standard_normal((w, w))
    GA = A + A.T
    Y, th, kept, bd = _lib.rayleigh_ritz(handle, m, GA, GB)
    ref = scipy.linalg.eigh(GA, GB, eigvals_only=True)[:m]
    assert bd == 0 and kept == w
    assert np.allclose(th, ref, rtol=1e-10, atol=1e-10)
    assert np.allclose(Y.T @ GB @ Y, np.eye(m), atol=1e-9)
    assert np.allclose(GA @ Y, GB @ Y @ np.diag(th), atol=1e-8 * np.abs(GA).max())


def test_rayleigh_ritz_drops_dependent_p_block(handle):
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((100, 6))
    Z = np.hstack([Z, Z[:, :2] @ rng.standard_normal((2, 2))])   # 2 dependent columns
    GB = Z.T @ Z
    M = rng.standard_normal((100, 100))
    GA = Z.T @ (M + M.T) @ Z          # projections of one operator
    Y, th, kept, bd = _lib.rayleigh_ritz(handle, 3, GA, GB, p_begin=6)
    assert bd == 0 and kept == 6
    ref = scipy.linalg.eigh(GA[:6, :6], GB[:6, :6], eigvals_only=True)[:3]
    assert np.allclose(th, ref, rtol=1e-8)
