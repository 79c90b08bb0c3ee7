"""Pins for oracle.precond, oracle.split and oracle.quality (CPU only)."""
import os

import numpy as np
import pytest

import graphgen
from oracle import laplacian as lap, precond, quality, split
from tests import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- precond

def test_jacobi_hand_example():
    R = np.array([[2.0, -4.0], [3.0, 9.0]])
    assert np.array_equal(precond.jacobi(R, np.array([2.0, 3.0])), [[1.0, -2.0], [1.0, 3.0]])


@pytest.mark.parametrize("degree,ratio", [(1, 4.0), (5, 10.0), (25, 30.0)])
def test_chebyshev_on_eigenvectors_matches_closed_form(degree, ratio):
    n = 40
    u = np.arange(n - 1)
    g = graphgen.csr_from_edges(n, u, u + 1)
    d = lap.degrees(g.rowptr, g.col, None)
    hi = precond.gershgorin_bound(d, lap.COMBINATORIAL)
    assert hi == 4.0
    ks = [1, 7, 20, 39]
    V = np.stack([cf.path_eigvec(n, k) for k in ks], axis=1)
    H = precond.chebyshev(g.rowptr, g.col, None, V, degree, hi / ratio, hi)
    for col, k in enumerate(ks):
        mu = cf.path_eigval(n, k)
        p = precond.chebyshev_scalar(mu, degree, hi / ratio, hi)
        assert p > 0
        assert np.allclose(H[:, col], p * V[:, col], rtol=1e-10, atol=1e-12)


def test_chebyshev_generalized_on_torus():
    n, u, v = cf.torus_edges(5, 4)
    g = graphgen.csr_from_edges(n, u, v)
    d = lap.degrees(g.rowptr, g.col, None)
    # torus eigenvector cos(2 pi a x / nx); D^-1 L has eigenvalue lam/4
    x = np.cos(2 * np.pi * 2 * (np.arange(n) % 5) / 5)
    lam = 2 - 2 * np.cos(2 * np.pi * 2 / 5)
    H = precond.chebyshev(g.rowptr, g.col, None, x[:, None], 6, 0.1, 2.0, dinv=1.0 / d)
    # h = p(D^-1 L) D^-1 r = p(lam/4) x / 4
    p = precond.chebyshev_scalar(lam / 4, 6, 0.1, 2.0)
    assert np.allclose(H[:, 0], p * x / 4, atol=1e-12)


def test_chebyshev_normalized_on_torus():
    n, u, v = cf.torus_edges(5, 4)
    g = graphgen.csr_from_edges(n, u, v)
    # 4-regular: L_N = L_C / 4, so the torus eigenvector has eigenvalue lam/4
    x = np.cos(2 * np.pi * 2 * (np.arange(n) % 5) / 5)
    lam = 2 - 2 * np.cos(2 * np.pi * 2 / 5)
    H = precond.chebyshev(g.rowptr, g.col, None, x[:, None], 6, 0.1, 2.0,
                          problem=lap.NORMALIZED)
    p = precond.chebyshev_scalar(lam / 4, 6, 0.1, 2.0)
    assert np.allclose(H[:, 0], p * x, atol=1e-12)
    assert precond.gershgorin_bound(np.array([3.0, 9.0]), lap.NORMALIZED) == 2.0


def test_chebyshev_polynomial_positive_on_spectrum():
    xs = np.linspace(1e-6, 12.0, 2001)
    assert np.all(precond.chebyshev_scalar(xs, 25, 12.0 / 30, 12.0) > 0)


# ---------------------------------------------------------------- split

def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_split_golden_hand_example():
    rows = _read_golden("split_k4_hand.txt")
    coords = np.array([[float(r[0]), float(r[1])] for r in rows])
    expect = np.array([int(r[2]) for r in rows])
    assert np.array_equal(split.split_pow2(coords, 4), expect)


def test_split_weighted_hand_example():
    # one coordinate, weights 3,1,1,1 (sorted order by value): W = 6;
    # prefixes W_lo = 0,3,4,5,6 -> |2W_lo - 6| = 6,0,2,4,6 -> prefix of 1
    coords = np.array([0.4, 0.1, 0.3, 0.2])
    vw = np.array([1, 3, 1, 1])
    assert list(split.split_pow2(coords, 2, vw)) == [1, 0, 1, 1]
    # weights 1,2,2,1 sorted: W = 6: W_lo = 0,1,3,5,6 -> 6,4,0,4,6 -> prefix 2
    vw = np.array([1, 1, 2, 2])       # sorted by value: ids 1,3,2,0 weights 1,2,2,1
    assert list(split.split_pow2(coords, 2, vw)) == [1, 0, 1, 0]


@pytest.mark.parametrize("n,K", [(1000, 64), (37, 8), (5, 4), (4, 4), (130, 2)])
def test_split_sizes_and_order(n, K):
    rng = np.random.default_rng(n)
    coords = rng.standard_normal((n, 6))
    part = split.split_pow2(coords, K)
    sizes = np.bincount(part, minlength=K)
    assert sizes.min() >= n // K and sizes.max() <= -(-n // K)
    # first level: everything in the lower half precedes the upper half on coord 0
    lo = coords[(part >> (K.bit_length() - 2)) == 0, 0] if K > 1 else None
    hi = coords[(part >> (K.bit_length() - 2)) == 1, 0] if K > 1 else None
    assert lo.max() <= hi.min()


def test_split_ties_broken_by_vertex_id_and_signed_zero():
    coords = np.zeros((10, 1))
    coords[::2, 0] = -0.0
    part = split.split_pow2(coords, 2)
    assert list(part) == [0] * 5 + [1] * 5


def test_split_matches_bruteforce_recursive_sort():
    rng = np.random.default_rng(9)
    n, K = 23, 8
    coords = np.round(rng.standard_normal((n, 3)), 1)     # many exact ties
    def brute(ids, level):
        if level == 3:
            return {i: 0 for i in ids}
        order = sorted(ids, key=lambda i: (coords[i, level], i))
        low, high = order[: len(order) // 2], order[len(order) // 2:]
        out = {}
        for i, p in brute(low, level + 1).items():
            out[i] = p
        for i, p in brute(high, level + 1).items():
            out[i] = p + (1 << (2 - level))
        return out
    b = brute(list(range(n)), 0)
    assert list(split.split_pow2(coords, K)) == [b[i] for i in range(n)]


# ---------------------------------------------------------------- quality

def test_cut_grid_halves_and_quadrants():
    g = graphgen.config_graph("grid64")
    x = np.arange(g.n) % 64
    y = np.arange(g.n) // 64
    assert quality.cutsize(g.rowptr, g.col, None, (x >= 32).astype(int)) == (64.0, 128.0)
    quad = (x >= 32).astype(int) + 2 * (y >= 32).astype(int)
    assert quality.cutsize(g.rowptr, g.col, None, quad)[0] == 128.0
    assert quality.imbalance(quad, 4) == 1.0


@pytest.mark.slow
def test_cut_grid128_blocks():
    g = graphgen.config_graph("grid7_128")
    i = np.arange(g.n)
    x, y, z = i % 128, (i // 128) % 128, i // (128 * 128)
    part = (x // 32) + 4 * (y // 32) + 16 * (z // 32)
    # 3 cut planes per axis, 128^2 edges each
    assert quality.cutsize(g.rowptr, g.col, None, part)[0] == 9 * 128 * 128


def test_cut_equals_quarter_quadratic_form_and_kway_identity():
    rng = np.random.default_rng(4)
    n, p = 60, 0.1
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    w = graphgen.uniform_weights(int(keep.sum()), 5, dtype=np.float64)
    g = graphgen.csr_from_edges(n, iu[keep], ju[keep], w)
    part = rng.integers(0, 2, n)
    x = 2.0 * part - 1.0
    q = x @ lap.apply(g.rowptr, g.col, g.w, x) / 4.0      # Sec. 3.2
    assert quality.cutsize(g.rowptr, g.col, g.w, part)[0] == pytest.approx(q, rel=1e-13)
    part = rng.integers(0, 5, n)
    chi = np.stack([(part == k).astype(float) for k in range(5)], axis=1)
    tot = 0.5 * np.sum(chi * lap.apply(g.rowptr, g.col, g.w, chi))
    assert quality.cutsize(g.rowptr, g.col, g.w, part)[0] == pytest.approx(tot, rel=1e-13)


def test_cut_sum_is_exact():
    # 2^53 + 1 + 1: naive left-to-right float sum loses both ones
    g = graphgen.csr_from_edges(4, np.array([0, 1, 2]), np.array([1, 2, 3]),
                                np.array([2.0 ** 53, 1.0, 1.0]))
    cut, _ = quality.cutsize(g.rowptr, g.col, g.w, np.array([0, 1, 0, 1]))
    assert cut == 2.0 ** 53 + 2.0


def test_part_weights_and_imbalance():
    part = np.array([0, 0, 1, 2, 2, 2])
    assert list(quality.part_weights(part, 3)) == [2, 1, 3]
    assert quality.imbalance(part, 3) == 1.5
    assert quality.imbalance(part, 3, vwgt=np.array([1, 1, 4, 1, 1, 0])) == 4 * 3 / 8
    with pytest.raises(ValueError):
        quality.part_weights(np.array([0, 3]), 3)


# ---- general K (multi-jagged with prime-factor section counts)

def test_split_mj_section_counts():
    assert split.section_counts(24) == [3, 2, 2, 2]
    assert split.section_counts(1) == []
    assert split.section_counts(64) == [2] * 6
    assert split.section_counts(7) == [7]
    assert split.section_counts(90) == [5, 3, 3, 2]


def test_split_mj_hand_examples():
    # 7 unit points on a line, K = 3: cut j after the prefix C minimising
    # |3 C - 7 j|: j = 1 -> C = 2 (|6 - 7| = 1), j = 2 -> C = 5 (|15 - 14| = 1)
    assert split.split_mj(np.arange(7.0), 3).tolist() == [0, 0, 1, 1, 1, 2, 2]
    # weights 1,1,1,1,5 (W = 9), K = 3: j = 1 -> C = 3 (|9 - 9| = 0);
    # j = 2 -> C = 4 (|12 - 18| = 6 beats |27 - 18| = 9)
    got = split.split_mj(np.arange(5.0), 3, vwgt=np.array([1, 1, 1, 1, 5]))
    assert got.tolist() == [0, 0, 0, 1, 2]
    # K = 6 on 12 points with two coordinates: level 1 (3 sections) on the
    # first, level 2 (2 sections) on the second within each section
    x = np.arange(12.0)
    y = np.array([5, 4, 3, 2, 1, 0, 11, 10, 9, 8, 7, 6], dtype=float)
    got = split.split_mj(np.stack([x, y], axis=1), 6)
    # sections {0..3}, {4..7}, {8..11}; lower halves by y: {2,3}, {4,5}, {10,11}
    assert got.tolist() == [1, 1, 0, 0, 2, 2, 3, 3, 5, 5, 4, 4]


@pytest.mark.parametrize("K", [2, 4, 16, 64])
def test_split_mj_equals_pow2_rule(K):
    rng = np.random.default_rng(K)
    C = rng.standard_normal((500, 6))
    w = rng.integers(1, 5, 500)
    assert np.array_equal(split.split_mj(C, K), split.split_pow2(C, K))
    assert np.array_equal(split.split_mj(C, K, w), split.split_pow2(C, K, w))


@pytest.mark.parametrize("n,K", [(1000, 24), (997, 3), (500, 6), (300, 7), (1000, 30), (64, 12)])
def test_split_mj_unit_sizes_and_line_order(n, K):
    rng = np.random.default_rng(n + K)
    C = rng.standard_normal((n, 4))
    part = split.split_mj(C, K)
    sizes = np.bincount(part, minlength=K)
    assert sizes.min() >= n // K and sizes.max() <= -(-n // K)
    # one coordinate: the parts are consecutive intervals along the line
    x = rng.permutation(n).astype(float)
    p1 = split.split_mj(x, K)
    assert np.all(np.diff(p1[np.argsort(x)]) >= 0)


def test_split_mj_relabelling_invariance():
    rng = np.random.default_rng(9)
    C = rng.standard_normal((400, 4))
    perm = rng.permutation(400)
    a = split.split_mj(C, 24)
    b = split.split_mj(C[perm], 24)
    assert np.array_equal(a[perm], b)


# ---- GMRES polynomial (Sec. 5.2)

def _kn_graph(n=9):
    iu, ju = np.triu_indices(n, 1)
    return graphgen.csr_from_edges(n, iu, ju)


def test_gmres_poly_exact_inverse_on_few_eigenvalues():
    # 6x5 torus: few distinct eigenvalues; with degree >= their count - 1 the
    # GMRES residual polynomial vanishes on the spectrum and p(L) = L^+ on 1^perp
    n, u, v = cf.torus_edges(6, 5)
    g = graphgen.csr_from_edges(n, u, v)
    L, d = lap.dense(g.rowptr, g.col, g.w)
    lam = np.unique(np.round(np.linalg.eigvalsh(L), 9))
    deg = len(lam) - 2                       # roots = degree + 1 = distinct non-zero eigenvalues
    b = np.random.default_rng(1).standard_normal(n)
    roots = precond.gmres_poly_roots(g.rowptr, g.col, None, lap.COMBINATORIAL, b, deg)
    assert np.allclose(np.sort(roots), lam[1:], rtol=1e-8)
    r = np.random.default_rng(2).standard_normal((n, 2))
    r -= r.mean(axis=0)
    H = precond.gmres_poly_apply(g.rowptr, g.col, None, lap.COMBINATORIAL, r, roots)
    assert np.allclose(L @ H, r, atol=1e-8)


def test_gmres_poly_minimises_residual_over_krylov():
    # pi(A) b has the least norm among residual polynomials of degree k + 1:
    # compare with a least-squares fit over the Krylov basis
    g = _random_weighted_graph()
    L, d = lap.dense(g.rowptr, g.col, g.w)
    b = np.random.default_rng(3).standard_normal(g.n)
    b -= b.mean()
    k = 6
    roots = precond.gmres_poly_roots(g.rowptr, g.col, g.w, lap.COMBINATORIAL, b, k)
    pb = b.copy()
    for t in roots:
        pb = pb - (L @ pb) / t
    Kr = np.stack([np.linalg.matrix_power(L, j) @ b for j in range(1, k + 2)], axis=1)
    c, *_ = np.linalg.lstsq(Kr, b, rcond=None)
    best = np.linalg.norm(b - Kr @ c)
    assert np.linalg.norm(pb) == pytest.approx(best, rel=1e-6)
    # on an eigenvector v (eigenvalue mu) the apply gives p(mu) v with
    # 1 - mu p(mu) = pi(mu) = prod (1 - mu / theta_i)
    lam_all, Vall = np.linalg.eigh(L)
    for q in (1, 5, g.n - 1):
        mu, v = lam_all[q], Vall[:, q]
        Hv = precond.gmres_poly_apply(g.rowptr, g.col, g.w, lap.COMBINATORIAL, v[:, None], roots)
        pi = np.prod(1 - mu / roots)
        assert np.allclose(Hv[:, 0], (1 - pi) / mu * v, atol=1e-9 * max(1, abs((1 - pi) / mu)))


def _random_weighted_graph(n=40, p=0.15, seed=3):
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    u = np.concatenate([iu[keep], np.arange(n - 1)])
    v = np.concatenate([ju[keep], np.arange(1, n)])
    key = np.unique(np.minimum(u, v) * n + np.maximum(u, v))
    u, v = key // n, key % n
    return graphgen.csr_from_edges(n, u, v, graphgen.uniform_weights(u.size, seed, dtype=np.float64))


def test_gmres_poly_generalized_equals_normalized_and_leja():
    # D^-1 L (D-inner product) from b and L_N from D^1/2 b share the Krylov
    # projection, hence the roots; p(D^-1 L) D^-1 r = D^-1/2 p(L_N) D^-1/2 r
    g = _random_weighted_graph()
    d = lap.degrees(g.rowptr, g.col, g.w)
    b = np.random.default_rng(4).standard_normal(g.n)
    rg = precond.gmres_poly_roots(g.rowptr, g.col, g.w, lap.GENERALIZED, b, 8)
    rn = precond.gmres_poly_roots(g.rowptr, g.col, g.w, lap.NORMALIZED, np.sqrt(d) * b, 8)
    assert np.allclose(rg, rn, rtol=1e-9)
    assert rg[0] == np.max(np.abs(rg))
    R = np.random.default_rng(5).standard_normal((g.n, 3))
    Hg = precond.gmres_poly_apply(g.rowptr, g.col, g.w, lap.GENERALIZED, R, rg)
    s = 1 / np.sqrt(d)
    Hn = precond.gmres_poly_apply(g.rowptr, g.col, g.w, lap.NORMALIZED, s[:, None] * R, rg)
    assert np.allclose(Hg, s[:, None] * Hn, rtol=1e-9, atol=1e-12)
    # roots lie in the non-trivial spectrum of D^-1 L (within [lambda_1, 2])
    L, _ = lap.dense(g.rowptr, g.col, g.w)
    ev = np.sort(np.linalg.eigvals(L / d[:, None]).real)
    assert rg.min() >= ev[1] * (1 - 1e-9) and rg.max() <= ev[-1] * (1 + 1e-9)
