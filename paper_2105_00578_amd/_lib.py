"""ctypes binding of libsphynx.so (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(PKG, "libsphynx.so")

OK, NOT_CONVERGED = 0, 1
UNIT, F32, F64 = 0, 1, 2
COMBINATORIAL, GENERALIZED, NORMALIZED = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI, PRECOND_CHEBYSHEV, PRECOND_GMRES = 0, 1, 2, 3
FP64, MIXED = 0, 1
INIT_RANDOM, INIT_PIECEWISE, INIT_USER = 0, 1, 2
SKIP_VALIDATE = 1


class SphynxError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"sphynx error {code}: {message}")
        self.code = code


class _Options(C.Structure):
    _fields_ = [("problem", C.c_int), ("precond", C.c_int), ("cheb_degree", C.c_int),
                ("cheb_ratio", C.c_double), ("precision", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("init", C.c_int), ("seed", C.c_uint64),
                ("locking", C.c_int), ("drop_tol", C.c_double), ("promote_window", C.c_int),
                ("reorder", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("restarts", C.c_int),
                ("graph_regular", C.c_int), ("max_degree", C.c_int64),
                ("avg_degree", C.c_double), ("rho", C.c_double * 32),
                ("ms_total", C.c_double), ("ms_setup", C.c_double), ("ms_spmm", C.c_double),
                ("ms_precond", C.c_double), ("ms_gram", C.c_double), ("ms_rr", C.c_double),
                ("ms_update", C.c_double), ("ms_split", C.c_double),
                ("ms_quality", C.c_double), ("spmm_calls", C.c_int64),
                ("precond_calls", C.c_int64), ("gb_spmm", C.c_double),
                ("gb_precond", C.c_double), ("precond_cols", C.c_int64),
                ("promoted", C.c_int32), ("col_index_bytes", C.c_int32)]


def _load():
    if not os.path.exists(library_path):
        raise ImportError(
            f"{library_path} is missing: build it with `python -m paper_2105_00578_amd.build` "
            "(there is no fallback implementation)")
    L = C.CDLL(library_path)
    vp, i64, i32p = C.c_void_p, C.c_int64, C.POINTER(C.c_int32)
    dp = C.POINTER(C.c_double)
    sig = {
        "sphx_status_string": (C.c_char_p, [C.c_int]),
        "sphx_create": (C.c_int, [C.POINTER(vp), C.c_int, vp]),
        "sphx_destroy": (C.c_int, [vp]),
        "sphx_set_stream": (C.c_int, [vp, vp]),
        "sphx_last_error": (C.c_char_p, [vp]),
        "sphx_set_timing": (C.c_int, [vp, C.c_int]),
        "sphx_num_eigenvectors": (C.c_int, [C.c_int]),
        "sphx_options_default": (None, [C.POINTER(_Options), C.c_int, C.c_int]),
        "sphx_graph_create": (C.c_int, [vp, i64, i64, vp, C.c_int, vp, vp, C.c_int, vp,
                                        C.c_uint32, C.POINTER(vp)]),
        "sphx_graph_destroy": (C.c_int, [vp]),
        "sphx_graph_info": (C.c_int, [vp, vp, C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                      dp]),
        "sphx_workspace_size": (C.c_int, [vp, vp, C.c_int, C.POINTER(_Options),
                                          C.POINTER(C.c_size_t)]),
        "sphx_set_workspace": (C.c_int, [vp, vp, C.c_size_t]),
        "sphx_workspace_owned": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "sphx_backward_info": (C.c_int, [vp, C.POINTER(C.c_int), dp]),
        "sphx_workspace_release": (C.c_int, [vp]),
        "sphx_quality_noalloc": (C.c_int, [vp, vp, vp, C.c_int, dp, dp, dp,
                                           C.POINTER(C.c_int64)]),
        "sphx_laplacian_apply": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int, vp, vp]),
        "sphx_poly_roots": (C.c_int, [vp, vp, C.c_int, C.c_int, vp, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int)]),
        "sphx_poly_apply": (C.c_int, [vp, vp, C.c_int, C.c_int, C.POINTER(C.c_double),
                                      C.c_int, C.c_int, vp, vp]),
        "sphx_precond_apply": (C.c_int, [vp, vp, C.POINTER(_Options), C.c_int, C.c_int, vp,
                                         vp]),
        "sphx_eigensolve": (C.c_int, [vp, vp, C.c_int, C.POINTER(_Options), vp, dp, vp,
                                      C.POINTER(_Stats)]),
        "sphx_split": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, vp]),
        "sphx_quality": (C.c_int, [vp, vp, vp, C.c_int, dp, dp, dp, C.POINTER(C.c_int64)]),
        "sphx_refine": (C.c_int, [vp, vp, C.c_int, vp, C.c_double, C.c_int, dp, dp,
                                  C.POINTER(C.c_int), C.POINTER(C.c_int64)]),
        "sphx_partition": (C.c_int, [vp, vp, C.c_int, C.POINTER(_Options), vp, dp, vp, vp,
                                     dp, dp, C.POINTER(_Stats)]),
        "sphx_eig_backward": (C.c_int, [vp, vp, C.c_int, C.c_int, dp, vp, dp, vp, C.c_double,
                                        C.c_int, vp]),
        "sphx_block_gram": (C.c_int, [vp, i64, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp,
                                      C.c_int, i32p, C.c_int, C.c_int, vp, dp, dp]),
        "sphx_rayleigh_ritz": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_double, dp, dp,
                                         dp, dp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


class _LazyLib:
    """Loads libsphynx.so on first use (so that the build step can import this
    package before the library exists); raises ImportError if it is missing."""

    _L = None

    def __getattr__(self, name):
        if _LazyLib._L is None:
            _LazyLib._L = _load()
        return getattr(_LazyLib._L, name)


lib = _LazyLib()


def status_string(code: int) -> str:
    return lib.sphx_status_string(code).decode()


def num_eigenvectors(K: int) -> int:
    """Eq. 4: d = floor(log2 K) + 1."""
    return lib.sphx_num_eigenvectors(K)


@dataclasses.dataclass
class Options:
    problem: int = COMBINATORIAL
    precond: int = PRECOND_JACOBI
    cheb_degree: int = 25
    cheb_ratio: float = 1000.0
    precision: int = FP64
    tol: float = 1e-3
    max_iter: int = 10000
    init: int = INIT_RANDOM
    seed: int = 0x5EED
    locking: int = 1
    drop_tol: float = 0.0
    promote_window: int = 0
    reorder: int = 1

    def _c(self) -> _Options:
        return _Options(**dataclasses.asdict(self))


def options_default(graph_is_regular: bool, precond: int = PRECOND_JACOBI, **overrides) -> Options:
    """Defaults of Sec. 6.3.1 from the library, with keyword overrides."""
    o = _Options()
    lib.sphx_options_default(C.byref(o), 1 if graph_is_regular else 0, precond)
    opts = Options(**{f: getattr(o, f) for f, _ in _Options._fields_})
    for k, v in overrides.items():
        if not hasattr(opts, k):
            raise TypeError(f"unknown option {k}")
        setattr(opts, k, v)
    return opts


@dataclasses.dataclass
class Stats:
    iterations: int
    converged: int
    restarts: int
    graph_regular: int
    max_degree: int
    avg_degree: float
    rho: list
    ms_total: float
    phases_ms: dict
    spmm_calls: int
    precond_calls: int
    gb_spmm: float
    gb_precond: float
    precond_cols: int
    promoted: int
    col_index_bytes: int


def _stats(s: _Stats, nev: int) -> Stats:
    phases = {k: getattr(s, "ms_" + k) for k in
              ("setup", "spmm", "precond", "gram", "rr", "update", "split", "quality")}
    return Stats(s.iterations, s.converged, s.restarts, s.graph_regular, s.max_degree,
                 s.avg_degree, list(s.rho[: min(nev, 32)]), s.ms_total, phases,
                 s.spmm_calls, s.precond_calls, s.gb_spmm, s.gb_precond, s.precond_cols,
                 s.promoted, s.col_index_bytes)


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Handle:
    """Library handle on a device, ordered on PyTorch's current stream."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = device
        self.h = C.c_void_p()
        self._check(lib.sphx_create(C.byref(self.h), device,
                                    C.c_void_p(torch.cuda.current_stream(device).cuda_stream)))
        self._ws = None

    def sync_stream(self):
        torch = _torch()
        lib.sphx_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, code: int, allow_warn: bool = False) -> int:
        if code < 0 or (code > 0 and not allow_warn):
            msg = ""
            if self.h:
                msg = lib.sphx_last_error(self.h).decode()
            raise SphynxError(code, f"{status_string(code)}: {msg}")
        return code

    def set_timing(self, on: bool):
        self._check(lib.sphx_set_timing(self.h, 1 if on else 0))

    def close(self):
        if self.h:
            lib.sphx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """Device CSR graph (borrowed tensors are kept referenced here)."""

    def __init__(self, h: Handle, rowptr, col, w=None, vwgt=None, validate: bool = True):
        torch = _torch()
        dev = torch.device("cuda", h.device)
        self.rowptr = rowptr.to(dev)
        self.col = col.to(dev, torch.int32).contiguous()
        self.w = None if w is None else w.to(dev).contiguous()
        self.vwgt = None if vwgt is None else vwgt.to(dev, torch.int32).contiguous()
        if self.rowptr.dtype not in (torch.int32, torch.int64):
            self.rowptr = self.rowptr.to(torch.int64)
        self.rowptr = self.rowptr.contiguous()
        self.n = self.rowptr.numel() - 1
        self.nnz = self.col.numel()
        wdt = UNIT
        if self.w is not None:
            wdt = {torch.float32: F32, torch.float64: F64}.get(self.w.dtype)
            if wdt is None:
                raise TypeError("edge weights must be float32 or float64")
        self.wdt = wdt
        self.h = h
        self.g = C.c_void_p()
        h._check(lib.sphx_graph_create(
            h.h, self.n, self.nnz, C.c_void_p(_ptr(self.rowptr)),
            1 if self.rowptr.dtype == torch.int64 else 0, C.c_void_p(_ptr(self.col)),
            C.c_void_p(_ptr(self.w)), wdt, C.c_void_p(_ptr(self.vwgt)),
            0 if validate else SKIP_VALIDATE, C.byref(self.g)))

    def info(self):
        _attach_workspace(self.h, self, 1, Options())
        reg = C.c_int()
        mx = C.c_int64()
        avg = C.c_double()
        self.h._check(lib.sphx_graph_info(self.h.h, self.g, C.byref(reg), C.byref(mx),
                                          C.byref(avg)))
        return bool(reg.value), mx.value, avg.value

    def close(self):
        if self.g:
            lib.sphx_graph_destroy(self.g)
            self.g = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dtype_code(t):
    torch = _torch()
    return {torch.float32: F32, torch.float64: F64}[t.dtype]


def workspace_size(h: Handle, g: Graph, nev: int, opts: Options) -> int:
    b = C.c_size_t()
    o = opts._c()
    h._check(lib.sphx_workspace_size(h.h, g.g, nev, C.byref(o), C.byref(b)))
    return b.value


def set_workspace(h: Handle, buf) -> None:
    """Hand the library a device byte tensor as workspace (kept referenced)."""
    h._ws = buf
    h._check(lib.sphx_set_workspace(h.h, C.c_void_p(_ptr(buf)),
                                    0 if buf is None else buf.numel() * buf.element_size()))


def workspace_owned(h: Handle) -> int:
    """Device bytes the handle owns as its own cached workspace."""
    b = C.c_size_t()
    h._check(lib.sphx_workspace_owned(h.h, C.byref(b)))
    return b.value


def workspace_release(h: Handle) -> None:
    """Free the handle's own cached workspace."""
    h._check(lib.sphx_workspace_release(h.h))


def _attach_workspace(h: Handle, g: Graph, nev: int, opts: Options) -> None:
    """Size the workspace for (g, nev, opts) and give the library a PyTorch
    byte buffer at least that large, so the call allocates no device memory
    of its own (the buffer grows, never shrinks, and stays with the handle)."""
    need = workspace_size(h, g, nev, opts)
    have = 0 if h._ws is None else h._ws.numel()
    if have < need:
        torch = _torch()
        set_workspace(h, torch.empty(need, dtype=torch.uint8, device=g.col.device))


def laplacian_apply(h: Handle, g: Graph, X, out=None, problem: int = COMBINATORIAL):
    """Y = L X for an n x m block (float32 or float64): L_C, or L_N for the
    normalized problem."""
    torch = _torch()
    X = X.contiguous()
    Y = torch.empty_like(X) if out is None else out
    m = 1 if X.dim() == 1 else X.shape[1]
    _attach_workspace(h, g, m, Options(problem=problem, precision=MIXED))
    h._check(lib.sphx_laplacian_apply(h.h, g.g, problem, m, _dtype_code(X),
                                      C.c_void_p(_ptr(X)), C.c_void_p(_ptr(Y))))
    return Y


def poly_roots(h: Handle, g: Graph, problem: int, degree: int, b):
    """Roots (Leja order) of the GMRES residual polynomial from start vector b
    (float64 device vector of length n)."""
    import numpy as np
    b = b.to(_torch().float64).contiguous()
    roots = (C.c_double * (degree + 1))()
    nr = C.c_int()
    h._check(lib.sphx_poly_roots(h.h, g.g, problem, degree, C.c_void_p(_ptr(b)), roots,
                                 C.byref(nr)))
    return np.array(roots[: nr.value])


def poly_apply(h: Handle, g: Graph, problem: int, roots, R, out=None):
    """H = p(A) R for the GMRES polynomial with the given roots."""
    torch = _torch()
    R = R.contiguous()
    H = torch.empty_like(R) if out is None else out
    m = 1 if R.dim() == 1 else R.shape[1]
    rr = (C.c_double * len(roots))(*[float(x) for x in roots])
    h._check(lib.sphx_poly_apply(h.h, g.g, problem, len(roots), rr, m, _dtype_code(R),
                                 C.c_void_p(_ptr(R)), C.c_void_p(_ptr(H))))
    return H


def precond_apply(h: Handle, g: Graph, opts: Options, R, out=None):
    torch = _torch()
    R = R.contiguous()
    H = torch.empty_like(R) if out is None else out
    m = 1 if R.dim() == 1 else R.shape[1]
    o = opts._c()
    _attach_workspace(h, g, m, opts)
    h._check(lib.sphx_precond_apply(h.h, g.g, C.byref(o), m, _dtype_code(R),
                                    C.c_void_p(_ptr(R)), C.c_void_p(_ptr(H))))
    return H


def _vec_dtype(opts: Options):
    torch = _torch()
    return torch.float32 if opts.precision == MIXED else torch.float64


def eigensolve(h: Handle, g: Graph, nev: int, opts: Options, X0=None, out=None,
               allow_not_converged: bool = False):
    """nev smallest eigenpairs: (eigvals float64[nev] on host, V device n x nev, Stats)."""
    torch = _torch()
    dt = _vec_dtype(opts)
    V = torch.empty((g.n, nev), dtype=dt, device=g.col.device) if out is None else out
    if X0 is not None:
        X0 = X0.to(g.col.device, dt).contiguous()
    lam = (C.c_double * nev)()
    st = _Stats()
    o = opts._c()
    _attach_workspace(h, g, nev, opts)
    code = lib.sphx_eigensolve(h.h, g.g, nev, C.byref(o), C.c_void_p(_ptr(X0)), lam,
                               C.c_void_p(_ptr(V)), C.byref(st))
    h._check(code, allow_warn=allow_not_converged)
    return list(lam), V, _stats(st, nev)


def split(h: Handle, g: Graph, coords, K: int, ld: Optional[int] = None, ncoord=None):
    """Part vector (int32[n]) from coordinates (n x ncoord block, row stride ld)."""
    torch = _torch()
    if coords.dim() == 1:
        coords = coords[:, None]
    ld = coords.stride(0) if ld is None else ld
    ncoord = coords.shape[1] if ncoord is None else ncoord
    part = torch.empty(g.n, dtype=torch.int32, device=g.col.device)
    h._check(lib.sphx_split(h.h, g.g, C.c_void_p(_ptr(coords)), ld, ncoord,
                            _dtype_code(coords), K, C.c_void_p(_ptr(part))))
    return part


def quality(h: Handle, g: Graph, part, K: int):
    """(cut, cut2x, imbalance, part_weights) -- Eq. 1 and max/avg part weight."""
    cut = C.c_double()
    cut2 = C.c_double()
    imb = C.c_double()
    pw = (C.c_int64 * K)()
    part = part.contiguous()
    h._check(lib.sphx_quality(h.h, g.g, C.c_void_p(_ptr(part)), K, C.byref(cut),
                              C.byref(cut2), C.byref(imb), pw))
    return cut.value, cut2.value, imb.value, list(pw)


def quality_noalloc(h: Handle, g: Graph, part, K: int):
    """As `quality`, through the entry point that allocates nothing (fixed
    device scratch, K <= 65536)."""
    cut = C.c_double()
    cut2 = C.c_double()
    imb = C.c_double()
    pw = (C.c_int64 * K)()
    part = part.contiguous()
    h._check(lib.sphx_quality_noalloc(h.h, g.g, C.c_void_p(_ptr(part)), K, C.byref(cut),
                                      C.byref(cut2), C.byref(imb), pw))
    return cut.value, cut2.value, imb.value, list(pw)


def refine(h: Handle, g: Graph, part, K: int, eps: float = 0.01, max_passes: int = 8):
    """Greedy refinement of the device int32 part vector, in place:
    (cut, imbalance, passes kept, accepted moves)."""
    torch = _torch()
    if part.dtype != torch.int32 or not part.is_contiguous():
        raise ValueError("part must be a contiguous int32 tensor (refined in place)")
    cut = C.c_double()
    imb = C.c_double()
    passes = C.c_int()
    moves = C.c_int64()
    h._check(lib.sphx_refine(h.h, g.g, K, C.c_void_p(_ptr(part)), float(eps), int(max_passes),
                             C.byref(cut), C.byref(imb), C.byref(passes), C.byref(moves)))
    return cut.value, imb.value, passes.value, moves.value


def partition(h: Handle, g: Graph, K: int, opts: Options, X0=None,
              allow_not_converged: bool = False):
    """Algorithm 2: (eigvals, V, part, cut, imbalance, Stats)."""
    torch = _torch()
    d = num_eigenvectors(K)
    dt = _vec_dtype(opts)
    V = torch.empty((g.n, d), dtype=dt, device=g.col.device)
    part = torch.empty(g.n, dtype=torch.int32, device=g.col.device)
    if X0 is not None:
        X0 = X0.to(g.col.device, dt).contiguous()
    lam = (C.c_double * d)()
    cut = C.c_double()
    imb = C.c_double()
    st = _Stats()
    o = opts._c()
    _attach_workspace(h, g, d, opts)
    code = lib.sphx_partition(h.h, g.g, K, C.byref(o), C.c_void_p(_ptr(X0)), lam,
                              C.c_void_p(_ptr(V)), C.c_void_p(_ptr(part)), C.byref(cut),
                              C.byref(imb), C.byref(st))
    h._check(code, allow_warn=allow_not_converged)
    return list(lam), V, part, cut.value, imb.value, _stats(st, d)


def eig_backward(h: Handle, g: Graph, problem: int, eigvals, V, g_vals=None, g_vecs=None,
                 cg_tol: float = 1e-12, cg_max_iter: int = 20000,
                 allow_not_converged: bool = False):
    """d loss / d w per CSR entry (float64 device tensor)."""
    torch = _torch()
    nev = V.shape[1]
    V = V.to(torch.float64).contiguous()
    lam = (C.c_double * nev)(*[float(x) for x in eigvals])
    gl = None
    if g_vals is not None:
        gl = (C.c_double * nev)(*[float(x) for x in g_vals])
    if g_vecs is not None:
        g_vecs = g_vecs.to(V.device, torch.float64).contiguous()
    grad = torch.empty(g.nnz, dtype=torch.float64, device=g.col.device)
    _attach_workspace(h, g, nev, Options(problem=problem))
    code = lib.sphx_eig_backward(h.h, g.g, problem, nev, lam, C.c_void_p(_ptr(V)), gl,
                                 C.c_void_p(_ptr(g_vecs)), cg_tol, cg_max_iter,
                                 C.c_void_p(_ptr(grad)))
    h._check(code, allow_warn=allow_not_converged)
    return grad


def backward_info(h: Handle):
    """(CG steps, largest final relative residual) of the last eig_backward."""
    it = C.c_int()
    rr = C.c_double()
    h._check(lib.sphx_backward_info(h.h, C.byref(it), C.byref(rr)))
    return it.value, rr.value


def block_gram(h: Handle, X, LX, H=None, LH=None, P=None, LP=None, act=(), bdiag=None):
    """Test hook: (GA, GB) of S = [X, H_a, P_a] as numpy w x w arrays."""
    import numpy as np
    n, m = X.shape
    act = list(act)
    use_h = H is not None
    use_p = P is not None
    w = m + len(act) * (int(use_h) + int(use_p))
    GA = np.zeros((w, w))
    GB = np.zeros((w, w))
    acts = (C.c_int32 * max(1, len(act)))(*act)
    dp = C.POINTER(C.c_double)
    h._check(lib.sphx_block_gram(
        h.h, n, m, _dtype_code(X), C.c_void_p(_ptr(X)), C.c_void_p(_ptr(LX)),
        C.c_void_p(_ptr(H)), C.c_void_p(_ptr(LH)), C.c_void_p(_ptr(P)), C.c_void_p(_ptr(LP)),
        len(act), acts, int(use_h), int(use_p), C.c_void_p(_ptr(bdiag)),
        GA.ctypes.data_as(dp), GB.ctypes.data_as(dp)))
    return GA, GB


def rayleigh_ritz(h: Handle, m: int, GA, GB, p_begin=None, drop_tol: float = 1e-14):
    """Test hook: (Y, theta, kept, breakdown) of the pencil (GA, GB)."""
    import numpy as np
    w = GA.shape[0]
    GA = np.ascontiguousarray(GA, dtype=np.float64)
    GB = np.ascontiguousarray(GB, dtype=np.float64)
    Y = np.zeros((w, m))
    th = np.zeros(m)
    kept = C.c_int()
    bd = C.c_int()
    dp = C.POINTER(C.c_double)
    h._check(lib.sphx_rayleigh_ritz(h.h, m, w, w if p_begin is None else p_begin, drop_tol,
                                    GA.ctypes.data_as(dp), GB.ctypes.data_as(dp),
                                    Y.ctypes.data_as(dp), th.ctypes.data_as(dp),
                                    C.byref(kept), C.byref(bd)))
    return Y, th, kept.value, bd.value
