"""Every boundary error code is reachable (graph validation runs on the GPU)."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from tests.gpu_util import dev, random_graph, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return sx.Handle(0)


def _t(a, dt):
    return torch.from_numpy(np.asarray(a, dtype=dt)).to(dev())


def _code(fn):
    with pytest.raises(sx.SphynxError) as e:
        fn()
    return e.value.code


def test_validation_codes(handle):
    # path 0-1-2 : rowptr [0,1,3,4], col [1,0,2,1]
    rp = [0, 1, 3, 4]
    col = [1, 0, 2, 1]
    sx.Graph(handle, _t(rp, np.int32), _t(col, np.int32))          # valid
    assert _code(lambda: sx.Graph(handle, _t(rp, np.int32), _t([1, 0, 2, 0], np.int32))) == -3
    assert _code(lambda: sx.Graph(handle, _t([0, 1, 3, 4], np.int32),
                                  _t([1, 2, 0, 1], np.int32))) == -2   # unsorted row 1
    assert _code(lambda: sx.Graph(handle, _t([0, 2, 4, 5], np.int32),
                                  _t([0, 1, 0, 2, 1], np.int32))) == -5  # self-loop
    assert _code(lambda: sx.Graph(handle, _t([0, 1, 3, 4], np.int32),
                                  _t([1, 0, 7, 1], np.int32))) == -2   # col out of range
    assert _code(lambda: sx.Graph(handle, _t(rp, np.int32), _t(col, np.int32),
                                  w=_t([1.0, 1.0, -2.0, -2.0], np.float32))) == -4
    assert _code(lambda: sx.Graph(handle, _t(rp, np.int32), _t(col, np.int32),
                                  w=_t([1.0, 1.0, np.nan, np.nan], np.float64))) == -4
    assert _code(lambda: sx.Graph(handle, _t(rp, np.int32), _t(col, np.int32),
                                  w=_t([1.0, 1.0, 2.0, 3.0], np.float64))) == -3  # asym weight
    assert _code(lambda: sx.Graph(handle, _t(rp, np.int32), _t(col, np.int32),
                                  vwgt=_t([1, 0, 1], np.int32))) == -4


def test_argument_codes(handle):
    g = random_graph(50, 0.1, 1)
    rp, col, w = upload(g)
    G = sx.Graph(handle, rp, col, w)
    opts = sx.Options()
    assert _code(lambda: sx.partition(handle, G, 1, opts)) == -1      # K < 2
    assert _code(lambda: sx.partition(handle, G, G.n + 1, opts)) == -1   # K > n
    assert _code(lambda: sx.partition(handle, G, 1, opts)) == -1
    assert _code(lambda: sx.eigensolve(handle, G, 50, opts)) == -1   # nev >= n
    bad = sx.Options(tol=-1.0)
    assert _code(lambda: sx.eigensolve(handle, G, 3, bad)) == -1
    # isolated vertex + generalized problem
    g2 = graphgen.csr_from_edges(4, np.array([0, 1]), np.array([1, 2]))
    rp2, col2, _ = upload(g2)
    G2 = sx.Graph(handle, rp2, col2)
    assert _code(lambda: sx.eigensolve(handle, G2, 2, sx.Options(problem=sx.GENERALIZED))) == -1


def test_malformed_row_ptr_of_a_neighbour_row(handle):
    """A neighbour row whose bounds leave [0, nnz] is rejected (code -2)
    before the symmetry search would read col[] outside the array."""
    col = _t([1, 0, 2, 1], np.int32)
    # row 2 claims entries up to 1000 although nnz = 4 (row 1 searches row 2)
    assert _code(lambda: sx.Graph(handle, _t([0, 1, 3, 1000], np.int32), col)) == -2
    # row_ptr[n] > nnz by one
    assert _code(lambda: sx.Graph(handle, _t([0, 1, 3, 5], np.int32), col)) == -2
    # a negative row bound in the middle
    assert _code(lambda: sx.Graph(handle, _t([0, 1, -5, 4], np.int32), col)) == -2
