"""The certified eigenpair fixtures are consistent (CPU only): the two
independent oracle runs stored in each agree within their certificates, the
stored bounds follow from the stored Ritz values and residuals, and the
fixture's graph is the generator's graph (same digest)."""
import os

import numpy as np
import pytest

import graphgen
from tests import certified

NAMES = [n for n in ("rmat22", "brick96lr", "king512", "rmat18")
         if os.path.exists(os.path.join(certified.GOLDEN, f"certified_{n}.json"))]


@pytest.mark.parametrize("name", NAMES)
def test_independent_runs_agree(name):
    gold = certified.load(name)
    d = gold["d"]
    a, b = (np.asarray(r["theta"]) for r in gold["runs"])
    ea, eb = (np.asarray(r["eps"]) for r in gold["runs"])
    # wanted values: both runs within their (tiny) bounds plus rounding
    tol_w = 1e-12 * a[d - 1] + 2 * gold["eig_bound"]
    assert np.all(np.abs(a[:d] - b[:d]) <= tol_w)
    # guard values (converged to guard_tol): within their Weinstein radii
    assert np.all(np.abs(a[d:] - b[d:]) <= ea[d:] + eb[d:] + 1e-12 * a[-1])
    # every run converged: relative residuals at the tolerance, or at the
    # FP64 floor of the recomputed residual where that is higher (king512:
    # eigenvalues near 1e-5 against ||D^-1 L|| <= 2 leave about 2e-10)
    th = a
    scale = np.maximum(th, th[1])
    assert np.all(ea[:d] <= np.maximum(1.01 * gold["tol"], 1e-9) * scale[:d])


@pytest.mark.parametrize("name", NAMES)
def test_stored_bounds_follow_from_ritz_values(name):
    gold = certified.load(name)
    th, eps, lo = (np.asarray(gold[k]) for k in ("theta", "eps", "lam_lo"))
    d = gold["d"]
    assert np.allclose(lo, th - eps, rtol=0, atol=1e-300)
    assert np.all(np.diff(th) >= 0)
    assert gold["delta"] == pytest.approx(lo[d] - th[d - 1], rel=1e-9)
    rF = np.sqrt(np.sum(eps[:d] ** 2))
    if gold["delta"] > 0:
        # the stored bounds come from a fresh residual of the d wanted columns
        # (Rayleigh-Ritz on their span), eps from the whole block's: they
        # agree to their last digits only
        assert gold["sin_bound"] == pytest.approx(rF / gold["delta"], rel=1e-2)
        assert gold["eig_bound"] == pytest.approx(rF ** 2 / gold["delta"], rel=2e-2)


@pytest.mark.slow
@pytest.mark.parametrize("name", [n for n in NAMES if n in ("king512", "rmat18")])
def test_fixture_graph_is_the_generators(name):
    gold = certified.load(name)
    g = graphgen.config_graph(name)
    assert (g.n, g.nnz) == (gold["n"], gold["nnz"])
    assert certified.digest(g) == gold["sha256"]
