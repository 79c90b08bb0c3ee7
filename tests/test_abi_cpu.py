"""The C ABI library loads and exports every declared symbol (CPU only; no
compute call needs a GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sphynx.h")
LIB = os.path.join(ROOT, "paper_2105_00578_amd", "libsphynx.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sphx_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2105_00578_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_host_only_entry_points(lib):
    lib.sphx_num_eigenvectors.restype = ctypes.c_int
    assert [lib.sphx_num_eigenvectors(k) for k in (1, 2, 4, 24, 64, 256, 0)] == \
        [1, 2, 3, 5, 7, 9, -1]
    lib.sphx_status_string.restype = ctypes.c_char_p
    assert lib.sphx_status_string(0) == b"ok"
    assert b"symmetric" in lib.sphx_status_string(-3)


def test_python_binding_defaults():
    import paper_2105_00578_amd as sx
    reg = sx.options_default(True, sx.PRECOND_JACOBI)
    assert (reg.problem, reg.tol, reg.init) == (sx.COMBINATORIAL, 1e-3, sx.INIT_RANDOM)
    irr = sx.options_default(False, sx.PRECOND_JACOBI)
    assert (irr.problem, irr.tol, irr.init) == (sx.GENERALIZED, 1e-2, sx.INIT_PIECEWISE)
    cheb = sx.options_default(True, sx.PRECOND_CHEBYSHEV)
    assert cheb.cheb_degree == 25
    assert sx.num_eigenvectors(64) == 7


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    lib.sphx_create.restype = ctypes.c_int
    assert lib.sphx_create(ctypes.byref(h), 0, None) < 0


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with status 2
    and a message, before any device work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout + r.stderr
