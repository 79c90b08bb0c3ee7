"""MI355X (gfx950) spectral graph partitioner -- Python binding of libsphynx.

Method: Sphynx (arXiv 2105.00578): the d = floor(log2 K) + 1 smallest
eigenpairs of the graph Laplacian by preconditioned LOBPCG (Algorithm 1),
the spectral embedding and a coordinate split into K parts (Algorithm 2).

This module only marshals arguments to the C ABI declared in
include/sphynx.h; every step runs in the library's HIP kernels.  PyTorch
provides device memory and the current stream.  The functions carry the C
names without the ``sphx_`` prefix.
"""
from ._lib import (  # noqa: F401
    SphynxError, Options, Stats, Handle, Graph, lib, library_path,
    status_string, num_eigenvectors, options_default,
    laplacian_apply, precond_apply, poly_roots, poly_apply, eigensolve, split, quality, refine, partition,
    eig_backward, workspace_size, set_workspace, workspace_owned, workspace_release,
    quality_noalloc, backward_info,
    COMBINATORIAL, GENERALIZED, NORMALIZED, PRECOND_NONE, PRECOND_JACOBI, PRECOND_CHEBYSHEV, PRECOND_GMRES,
    FP64, MIXED, INIT_RANDOM, INIT_PIECEWISE, INIT_USER,
)
from .autograd import EigFn  # noqa: F401
