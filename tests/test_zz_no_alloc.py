"""sphx_quality_noalloc (fixed device scratch, no allocation) against
sphx_quality, bit for bit, on two calls in a row, the second smaller."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2105_00578_amd as sx
from tests.gpu_util import dev, upload

pytestmark = pytest.mark.gpu


def _parts(n, K, seed):
    return torch.from_numpy(
        np.random.default_rng(seed).integers(0, K, n).astype(np.int32)).to(dev())


@pytest.mark.parametrize("name,sd", [("brick96lr", 4), ("grid7_128", 4), ("king512", 8)])
def test_noalloc_quality_matches_quality(name, sd):
    h = sx.Handle(0)
    cases = []
    for scale, K in ((sd, 300), (2 * sd, 5)):        # second call: smaller graph and K
        g = graphgen.config_graph(name, scale_down=scale)
        rp, col, w = upload(g)
        cases.append((sx.Graph(h, rp, col, w), g.n, K))
    for G, n, K in cases:
        part = _parts(n, K, K)
        a = sx.quality_noalloc(h, G, part, K)
        b = sx.quality(h, G, part, K)
        assert a == b
        assert sum(a[3]) == n
    # the no-alloc calls never made the handle allocate (the quality calls
    # afterwards do; release them and call the no-alloc path again)
    sx.workspace_release(h)
    G, n, K = cases[1]
    part = _parts(n, K, 99)
    sx.quality_noalloc(h, G, part, K)
    assert sx.workspace_owned(h) == 0


def test_noalloc_rejects_large_k():
    h = sx.Handle(0)
    g = graphgen.config_graph("grid64", scale_down=8)
    rp, col, w = upload(g)
    G = sx.Graph(h, rp, col, w)
    part = torch.zeros(g.n, dtype=torch.int32, device=dev())
    with pytest.raises(sx.SphynxError) as e:
        sx.quality_noalloc(h, G, part, 65537)
    assert e.value.code == -8


def test_noalloc_fresh_handles_share_the_array():
    """Two handles on one GPU use the same array, one after the other."""
    g = graphgen.config_graph("brick96lr", scale_down=8)
    outs = []
    for _ in range(2):
        h = sx.Handle(0)
        rp, col, w = upload(g)
        G = sx.Graph(h, rp, col, w)
        part = _parts(g.n, 64, 3)
        outs.append(sx.quality_noalloc(h, G, part, 64))
        assert sx.workspace_owned(h) == 0
    assert outs[0] == outs[1]
