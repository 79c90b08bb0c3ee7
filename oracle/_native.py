"""Loader of the oracle's C helpers (test infrastructure only).

`oracle/csrc/lap_omp.c` holds the oracle's OpenMP Laplacian product.  It is
compiled with gcc into `oracle/liboracle.so` (by the package build, or here on
first use when the library is missing or older than its source).  Nothing of
the product library is linked or included.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "lap_omp.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc -O2 -fopenmp (every call when force)."""
    if (not force and os.path.exists(LIB)
            and os.path.getmtime(LIB) >= os.path.getmtime(SRC)):
        return LIB
    tmp = f"{LIB}.{os.getpid()}.tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle build failed\n{' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        L.oracle_lap_apply.argtypes = [I64, P, P, P, P, I64, P, ctypes.c_int]
        L.oracle_lap_apply.restype = None
        L.oracle_triad.argtypes = [I64, P, P, P, ctypes.c_double, ctypes.c_int]
        L.oracle_triad.restype = None
        _lib = L
    return _lib


def default_threads() -> int:
    """Threads for the oracle's loops: OMP_NUM_THREADS if set, else the CPUs
    this process may run on."""
    v = os.environ.get("OMP_NUM_THREADS")
    if v and v.isdigit() and int(v) > 0:
        return int(v)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1
