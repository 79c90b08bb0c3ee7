"""Textbook closed forms used to pin the oracle (independent of its code).

Path graph P_n (unit weights): eigenvalues 2 - 2 cos(pi k / n), eigenvectors
cos(pi k (i + 1/2) / n), k = 0..n-1.  A non-periodic lattice is the Cartesian
product of paths, so its eigenvalues are sums and its eigenvectors tensor
products.  Cycle C_n: 2 - 2 cos(2 pi k / n).  A torus is the product of cycles
and is exactly regular, so its generalized spectrum is the combinatorial one
divided by the degree.
"""
import itertools

import numpy as np


def path_eigval(n, k):
    return 2.0 - 2.0 * np.cos(np.pi * k / n)


def path_eigvec(n, k):
    i = np.arange(n)
    return np.cos(np.pi * k * (i + 0.5) / n)


def grid_eigvals(shape, count):
    """The `count` smallest eigenvalues of the lattice with side lengths shape."""
    vals = []
    ranges = [range(min(s, 8)) for s in shape]
    for ks in itertools.product(*ranges):
        vals.append(sum(path_eigval(s, k) for s, k in zip(shape, ks)))
    vals.sort()
    return np.array(vals[:count])


def grid_eigvec(shape, ks):
    """Tensor-product eigenvector, vertex numbering in C order over shape."""
    v = np.ones(1)
    for s, k in zip(shape, ks):
        v = np.multiply.outer(v, path_eigvec(s, k))
    return v.ravel()


def torus_edges(nx, ny):
    idx = np.arange(nx * ny).reshape(ny, nx)
    u = np.concatenate([idx.ravel(), idx.ravel()])
    v = np.concatenate([np.roll(idx, -1, axis=1).ravel(), np.roll(idx, -1, axis=0).ravel()])
    return nx * ny, u, v


def torus_eigvals(nx, ny):
    a = np.arange(nx)[:, None]
    b = np.arange(ny)[None, :]
    return np.sort((4 - 2 * np.cos(2 * np.pi * a / nx) - 2 * np.cos(2 * np.pi * b / ny)).ravel())
