"""Seeded synthetic graph and block generators.

This module is shared by the CPU oracle and the GPU path's tests and benchmark.
It only builds inputs (edge lists, CSR arrays, random weights, random initial
blocks); it contains none of the partitioning method's arithmetic.

Graph families follow the workloads of the Sphynx paper (arXiv 2105.00578):
  * structured meshes: 2D 5-point and 9-point grids, 3D 7-point and 27-point
    ("Brick3D") stencils with non-periodic boundaries (Section 5.1, Dataset);
  * power-law graphs: R-MAT with parameters (a, b, c, d), standing in for the
    paper's irregular web and social graphs, which are not available here;
  * a 27-point mesh with a fraction of random long-range edges.

Preprocessing mirrors the paper's: self-loops are dropped (the Laplacian has
no use for them), the pattern is symmetrised and deduplicated, and only the
largest connected component is kept (Section 5.1, Dataset).

All CSR outputs are symmetric, have sorted column indices within each row, no
self-loops and no duplicates.  Edge weights, when present, are equal on both
directions of an undirected edge.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Graph", "grid_edges", "grid2d_5pt", "grid2d_9pt", "grid3d_7pt", "brick27",
    "rmat_edges", "add_long_range", "csr_from_edges", "largest_component",
    "uniform_weights", "normal_block", "config_graph", "CONFIGS",
]


@dataclasses.dataclass
class Graph:
    """Symmetric CSR graph held in host numpy arrays.

    rowptr: int64[n+1]; col: int32[nnz]; w: None (unit weights) or
    float32/float64[nnz]; name: human-readable recipe.
    """
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    def degree_counts(self) -> np.ndarray:
        return np.diff(self.rowptr)


# ----------------------------------------------------------------------------
# structured meshes
# ----------------------------------------------------------------------------

def _half_offsets(dim: int, full: bool) -> list:
    """Neighbour offsets whose first non-zero component is positive.

    full=True gives the 3^dim - 1 stencil (9-point in 2D, 27-point in 3D);
    full=False gives the axis-aligned 2*dim stencil (5-point, 7-point).
    """
    out = []
    for off in itertools.product((-1, 0, 1), repeat=dim):
        if not any(off):
            continue
        if not full and sum(1 for o in off if o) != 1:
            continue
        first = next(o for o in off if o)
        if first > 0:
            out.append(off)
    return out


def grid_edges(shape: Sequence[int], offsets: Sequence[Tuple[int, ...]]):
    """Undirected edge list (u < v not required) of a non-periodic lattice.

    Vertices are numbered in C order over `shape` (last axis fastest).
    """
    shape = tuple(int(s) for s in shape)
    idx = np.arange(int(np.prod(shape)), dtype=np.int64).reshape(shape)
    us, vs = [], []
    for off in offsets:
        src = []
        dst = []
        for o, s in zip(off, shape):
            if o > 0:
                src.append(slice(0, s - o)); dst.append(slice(o, s))
            elif o < 0:
                src.append(slice(-o, s)); dst.append(slice(0, s + o))
            else:
                src.append(slice(0, s)); dst.append(slice(0, s))
        us.append(idx[tuple(src)].ravel())
        vs.append(idx[tuple(dst)].ravel())
    return np.concatenate(us), np.concatenate(vs)


def grid2d_5pt(nx: int, ny: int):
    return nx * ny, grid_edges((ny, nx), _half_offsets(2, full=False))


def grid2d_9pt(nx: int, ny: int):
    return nx * ny, grid_edges((ny, nx), _half_offsets(2, full=True))


def grid3d_7pt(nx: int, ny: int, nz: int):
    return nx * ny * nz, grid_edges((nz, ny, nx), _half_offsets(3, full=False))


def brick27(nx: int, ny: int, nz: int):
    """27-point stencil on a non-periodic nx*ny*nz brick (Galeri "Brick3D")."""
    return nx * ny * nz, grid_edges((nz, ny, nx), _half_offsets(3, full=True))


def brick27_csr(nx: int, ny: int, nz: int, name: str = "") -> "Graph":
    """CSR of the 27-point brick built row by row (no edge list or sort):
    the same graph as csr_from_edges on brick27, for sizes where the edge
    list would be large.  Rows are vertices z*ny*nx + y*nx + x."""
    n = nx * ny * nz
    offs = sorted(((dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                   if (dz, dy, dx) != (0, 0, 0)),
                  key=lambda o: o[0] * ny * nx + o[1] * nx + o[2])
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    del idx
    valid = np.empty((n, len(offs)), dtype=bool)
    for q, (dz, dy, dx) in enumerate(offs):
        valid[:, q] = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
                       & (z + dz >= 0) & (z + dz < nz))
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    delta = np.array([o[0] * ny * nx + o[1] * nx + o[2] for o in offs], dtype=np.int64)
    col = np.empty(int(rowptr[-1]), dtype=np.int32)
    rows = np.arange(n, dtype=np.int64)
    # fill by rows in chunks: columns of a row are its valid offsets in
    # increasing delta order, hence sorted
    chunk = 1 << 20
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        cand = rows[lo:hi, None] + delta[None, :]
        col[rowptr[lo]:rowptr[hi]] = cand[valid[lo:hi]].astype(np.int32)
    return Graph(n=n, rowptr=rowptr, col=col, w=None, name=name or f"brick27_{nx}x{ny}x{nz}")


# ----------------------------------------------------------------------------
# R-MAT and long-range edges
# ----------------------------------------------------------------------------

def rmat_edges(scale: int, edge_factor: int, a: float, b: float, c: float,
               seed: int, chunk: int = 1 << 23):
    """R-MAT edge samples (with self-loops and duplicates, as drawn).

    Each of the 2^scale * edge_factor samples descends `scale` levels of the
    adjacency quadtree, choosing quadrant (0,0), (0,1), (1,0), (1,1) with
    probabilities a, b, c, d = 1 - a - b - c.  No noise is added.
    """
    n = 1 << scale
    m = n * edge_factor
    rng = np.random.default_rng(seed)
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.int64)
        t = np.zeros(hi - lo, dtype=np.int64)
        for lev in range(scale):
            u = rng.random(hi - lo)
            sbit = u >= ab
            tbit = ((u >= a) & (u < ab)) | (u >= abc)
            s |= sbit.astype(np.int64) << lev
            t |= tbit.astype(np.int64) << lev
        src[lo:hi] = s
        dst[lo:hi] = t
    return n, src, dst


def add_long_range(n: int, u: np.ndarray, v: np.ndarray, count: int, seed: int):
    """Append `count` extra undirected edges with uniform random endpoints.

    Self-loops and edges already present (in either direction) are resampled,
    so the result has exactly len(u) + count distinct undirected edges.
    """
    rng = np.random.default_rng(seed)
    lo = np.minimum(u, v).astype(np.int64)
    hi = np.maximum(u, v).astype(np.int64)
    existing = np.unique(lo * n + hi)
    extra = np.empty(0, dtype=np.int64)
    need = count
    while need > 0:
        a = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        b = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        keep = a != b
        a, b = a[keep], b[keep]
        key = np.minimum(a, b) * n + np.maximum(a, b)
        # drop duplicates among the new draws (keep first occurrence) and
        # anything already present
        _, first = np.unique(key, return_index=True)
        first.sort()
        key = key[first]
        key = key[~np.isin(key, existing)]
        key = key[~np.isin(key, extra)]
        key = key[:need]
        extra = np.concatenate([extra, key])
        need = count - extra.size
    eu = extra // n
    ev = extra % n
    return np.concatenate([u.astype(np.int64), eu]), np.concatenate([v.astype(np.int64), ev])


# ----------------------------------------------------------------------------
# cleaning and CSR assembly
# ----------------------------------------------------------------------------

def _dedup_undirected(n: int, u: np.ndarray, v: np.ndarray):
    keep = u != v
    u, v = u[keep], v[keep]
    key = np.minimum(u, v).astype(np.int64) * n + np.maximum(u, v)
    key = np.unique(key)
    return key // n, key % n


def largest_component(n: int, u: np.ndarray, v: np.ndarray):
    """Keep the largest connected component; relabel by increasing old id.

    Returns (n_new, u_new, v_new, old_ids) where old_ids[new] = old label.
    Ties between equally large components go to the one holding the smallest
    vertex id.
    """
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    if u.size == 0:
        return (1 if n else 0), u, v, np.arange(min(n, 1), dtype=np.int64)
    adj = sp.coo_matrix((np.ones(u.size, dtype=np.int8), (u, v)), shape=(n, n)).tocsr()
    ncomp, lab = csg.connected_components(adj, directed=False)
    sizes = np.bincount(lab, minlength=ncomp)
    best = np.flatnonzero(sizes == sizes.max())
    # component containing the smallest vertex id among the largest ones
    first_vertex = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(first_vertex, lab, np.arange(n, dtype=np.int64))
    comp = best[np.argmin(first_vertex[best])]
    old_ids = np.flatnonzero(lab == comp).astype(np.int64)
    new_of_old = np.full(n, -1, dtype=np.int64)
    new_of_old[old_ids] = np.arange(old_ids.size, dtype=np.int64)
    keep = lab[u] == comp
    return old_ids.size, new_of_old[u[keep]], new_of_old[v[keep]], old_ids


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray,
                   w: Optional[np.ndarray] = None, name: str = "") -> Graph:
    """Symmetric CSR from a list of distinct undirected edges (u != v).

    Each edge is stored in both directions; columns are sorted within rows.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = src * n + dst
    if w is None:
        key.sort()
        wv = None
    else:
        order = np.argsort(key, kind="stable")
        key = key[order]
        wv = np.concatenate([w, w])[order]
    s = key // n
    col = (key % n).astype(np.int32)
    counts = np.bincount(s, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return Graph(n=n, rowptr=rowptr, col=col, w=wv, name=name)


# ----------------------------------------------------------------------------
# random values
# ----------------------------------------------------------------------------

def uniform_weights(count: int, seed: int, lo: float = 0.5, hi: float = 1.5,
                    dtype=np.float32) -> np.ndarray:
    """i.i.d. uniform edge weights in [lo, hi), drawn in float64 then cast."""
    rng = np.random.default_rng(seed)
    return (lo + (hi - lo) * rng.random(count)).astype(dtype)


def perturb_weights(g: Graph, rel: float, seed: int, dtype=np.float64) -> Graph:
    """The same graph with every edge weight scaled by a factor in
    [1 - rel, 1 + rel) (unit weights taken as 1): a workload whose weights
    drift between repartitionings.  The factor of an edge is a hash of its
    end points and the seed, so both stored directions get the same value."""
    iu = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr))
    a = np.minimum(iu, g.col).astype(np.int64)
    b = np.maximum(iu, g.col).astype(np.int64)
    h = (a * 1000003 + b * 7919 + seed * 104729) % 1000
    f = 1.0 + rel * (h / 500.0 - 1.0)
    base = np.ones(g.col.size) if g.w is None else g.w.astype(np.float64)
    return Graph(n=g.n, rowptr=g.rowptr, col=g.col, w=(base * f).astype(dtype),
                 name=f"{g.name}+drift{rel:g}")


def normal_block(n: int, m: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n x m row-major block of i.i.d. N(0, 1) values (initial LOBPCG block)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, m)).astype(dtype)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    # name: description
    "grid64": "2D 5-point grid 64x64, unit weights",
    "grid7_128": "3D 7-point grid 128^3, unit weights",
    "rmat22": "R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), LCC, unit weights",
    "brick96lr": "3D 27-point 96^3 + 1% long-range edges, weights U[0.5,1.5) fp32",
    "king512": "2D 9-point grid 512x512, weights U[0.5,1.5) fp64",
    "rmat18": "R-MAT scale 18, edge factor 16, LCC, weights U[0.5,1.5) fp64",
    "brick100": "Galeri Brick3D 27-point 100^3, unit weights (the paper's synthetic mesh)",
    "brick200": "Galeri Brick3D 27-point 200^3, unit weights",
    "brick400": "Galeri Brick3D 27-point 400^3, unit weights",
}


def rmat_graph(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1, weight_seed: Optional[int] = None,
               weight_dtype=np.float32, permute: bool = True) -> Graph:
    """R-MAT graph: sample, permute labels (seeded), dedup, drop loops, LCC."""
    n, s, t = rmat_edges(scale, edge_factor, a, b, c, seed)
    if permute:
        perm = np.random.default_rng(seed + 1000003).permutation(n).astype(np.int64)
        s = perm[s]
        t = perm[t]
    u, v = _dedup_undirected(n, s, t)
    del s, t
    n2, u, v, _ = largest_component(n, u, v)
    w = None
    if weight_seed is not None:
        w = uniform_weights(u.size, weight_seed, dtype=weight_dtype)
    return csr_from_edges(n2, u, v, w, name=f"rmat{scale}_ef{edge_factor}")


def config_graph(name: str, graph_seed: int = 1, weight_seed: int = 0,
                 scale_down: int = 1) -> Graph:
    """Build one of the named workloads.

    scale_down > 1 shrinks the lattice side lengths (or R-MAT scale by
    log2(scale_down)) for fast tests with the same recipe.
    """
    if name == "grid64":
        s = max(2, 64 // scale_down)
        n, (u, v) = grid2d_5pt(s, s)
        return csr_from_edges(n, u, v, None, name=f"grid5_{s}x{s}")
    if name == "grid7_128":
        s = max(2, 128 // scale_down)
        n, (u, v) = grid3d_7pt(s, s, s)
        return csr_from_edges(n, u, v, None, name=f"grid7_{s}^3")
    if name == "rmat22":
        sc = 22 - int(np.log2(scale_down))
        return rmat_graph(sc, seed=graph_seed)
    if name == "brick96lr":
        s = max(3, 96 // scale_down)
        n, (u, v) = brick27(s, s, s)
        extra = int(round(0.01 * u.size))
        u, v = add_long_range(n, u, v, extra, seed=graph_seed)
        w = uniform_weights(u.size, weight_seed, dtype=np.float32)
        return csr_from_edges(n, u, v, w, name=f"brick27_{s}^3+1%lr")
    if name == "king512":
        s = max(3, 512 // scale_down)
        n, (u, v) = grid2d_9pt(s, s)
        w = uniform_weights(u.size, weight_seed, dtype=np.float64)
        return csr_from_edges(n, u, v, w, name=f"grid9_{s}x{s}")
    if name == "rmat18":
        sc = 18 - int(np.log2(scale_down))
        return rmat_graph(sc, seed=graph_seed, weight_seed=weight_seed,
                          weight_dtype=np.float64)
    if name in ("brick100", "brick200", "brick400"):
        s = max(3, int(name[5:]) // scale_down)
        return brick27_csr(s, s, s, name=f"brick27_{s}^3")
    raise KeyError(name)
