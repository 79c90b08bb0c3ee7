"""Helpers shared by the GPU tests (device upload of generator outputs)."""
import numpy as np
import pytest
import torch

import graphgen

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def dev():
    return torch.device("cuda", 0)


def upload(g, rowptr64=False, wdtype=None):
    """(rowptr, col, w) device tensors of a graphgen.Graph."""
    rp = torch.from_numpy(g.rowptr.astype(np.int64 if rowptr64 else np.int32)).to(dev())
    col = torch.from_numpy(g.col.astype(np.int32)).to(dev())
    w = None
    if g.w is not None:
        wa = g.w if wdtype is None else g.w.astype(wdtype)
        w = torch.from_numpy(np.ascontiguousarray(wa)).to(dev())
    return rp, col, w


def random_graph(n, p, seed, wdtype=None, connected=True):
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    u, v = iu[keep], ju[keep]
    if connected:
        u = np.concatenate([u, np.arange(n - 1)])
        v = np.concatenate([v, np.arange(1, n)])
    key = np.unique(np.minimum(u, v) * n + np.maximum(u, v))
    u, v = key // n, key % n
    w = None
    if wdtype is not None:
        w = graphgen.uniform_weights(u.size, seed + 1, dtype=wdtype)
    return graphgen.csr_from_edges(n, u, v, w)


def star_graph(leaves, extra_seed=0):
    """Hub vertex 0 joined to `leaves` vertices, plus a path among the leaves."""
    n = leaves + 1
    u = np.concatenate([np.zeros(leaves, dtype=np.int64), np.arange(1, leaves)])
    v = np.concatenate([np.arange(1, n), np.arange(2, n)])
    return graphgen.csr_from_edges(n, u, v)
