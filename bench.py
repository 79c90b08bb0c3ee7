#!/usr/bin/env python3
"""Benchmark of the spectral-partitioning hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 3D 7-point
grid 128^3 (2,097,152 vertices, 6,242,304 unit edges), combinatorial
Laplacian, K = 64 parts (d = 7 eigenvectors), LOBPCG with a degree-25
Chebyshev preconditioner, residual tolerance 1e-3 (the paper's default for
regular graphs), random start.  One step = one full partition (setup, LOBPCG,
embedding, split, cut and imbalance) with the graph resident in HBM.

Metric: Laplacian SpMM HBM GB/s and time to the K-way eigenvectors in mixed
precision (FP32 SpMM / preconditioner / updates, FP64 Gram and
Rayleigh-Ritz) vs all-FP64 at the same residual tolerance.  `value` is the
GB/s of the dominant kernel (the fused Chebyshev-step Laplacian product):
algorithmic bytes of all its launches (over the int32 CSR the caller
passes) divided by their summed durations, measured with events that each
launch's dispatch stamps on the library's stream, in an instrumented pass of
`--steps` partitions after the timed ones.  The timed steps, and the time to
eigenvectors (the eigensolver alone, `--steps` calls, median), run without
those per-launch events, as the library does by default.  On this
grid the kernels read the column indices as int16 offsets from the row
(`roofline.col_index_bytes_read`), so the bytes they move are fewer than the
algorithmic count; `roofline.traffic` gives the measured bytes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --workload NAME      (another configuration; adjoint-rmat18
                                      and adjoint-king512 time EigFn forward and
                                      backward on the differentiation workloads)
       python bench.py --repartition        (also: greedy refinement and a
                                      warm-started repartition)
       python bench.py --only-mixed --steps 1 --warmup 0 --no-cpu-baseline
                                      (one mixed partition, for counter runs)
       python bench.py --copy-probe BYTES   (one plain device copy of BYTES,
                                      the calibration of the byte counters)

`roofline.traffic` is the HBM bytes per launch of the dominant kernel from
the FETCH_SIZE / WRITE_SIZE counter runs summarised in profiles/, scaled by
the counters' reading for a plain copy of known size; it is reported only
while the kernel source is the one the counters were taken on (checked by
hash), else null.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Laplacian SpMM HBM GB/s; time to K-way eigvecs FP32 vs FP64 at equal residual"
HBM_PEAK_GBS = 8000.0


def _path_eigval(n, k):
    """Path graph P_n: eigenvalue 2 - 2 cos(pi k / n)."""
    import numpy as np
    return 2.0 - 2.0 * np.cos(np.pi * k / n)


def _grid_eigvec(side, ks):
    """Tensor product of path eigenvectors cos(pi k (i + 1/2) / n) on the
    side^3 grid (vertex numbering x fastest)."""
    import numpy as np
    i = np.arange(side)
    v = np.ones(1)
    for k in ks:
        v = np.multiply.outer(v, np.cos(np.pi * k * (i + 0.5) / side))
    return v.ravel()


def closed_form_check(lam, V, side):
    """Eigenvalue relative errors and subspace angle against the closed-form
    spectrum of the side^3 grid (sums of path eigenvalues, tensor vectors)."""
    import numpy as np
    m = len(lam)
    ks = [(a, b, c) for a in range(3) for b in range(3) for c in range(3)]
    val = {k: sum(_path_eigval(side, q) for q in k) for k in ks}
    ks = sorted(ks, key=lambda k: val[k])
    exact = np.array([val[k] for k in ks[:m + 1]])
    rel = [abs(lam[k] - exact[k]) / exact[k] for k in range(1, m)]
    trivial = abs(lam[0]) / exact[1]
    # exact invariant subspace of the m smallest (the block ends at a gap)
    ks = ks[:m]
    E = np.stack([_grid_eigvec(side, k) for k in ks], axis=1)
    # sine of the largest principal angle between span(V) and span(E)
    qv, _ = np.linalg.qr(V.astype(np.float64))
    qe, _ = np.linalg.qr(E)
    smin = np.linalg.svd(qv.T @ qe, compute_uv=False).min()
    sin = float(np.sqrt(max(0.0, 1.0 - smin * smin)))
    return max(rel), trivial, sin, float(exact[m] - exact[m - 1])


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_triad_gbs(threads, n=1 << 26, reps=5):
    """STREAM-style triad a = b + s c on the host cores (the oracle's C
    loop), best of reps: 24 bytes per element."""
    import numpy as np
    from oracle import _native
    lib = _native.lib()
    a = np.empty(n)
    b = np.ones(n)
    c = np.ones(n)
    best = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        lib.oracle_triad(n, a.ctypes.data, b.ctypes.data, c.ctypes.data, 0.5, threads)
        dt = time.perf_counter() - t0
        best = max(best, 24.0 * n / dt / 1e9)
    return best


def cpu_baseline(g, m, gpu_fp64_iterations, opts, budget_s=20.0):
    """The oracle's LOBPCG (Algorithm 1 in FP64 with its C/OpenMP Laplacian
    product and the same Chebyshev preconditioner: degree 25, ratio, tol) on
    all host cores, from an N(0,1) start block, for a bounded number of
    iterations (about budget_s); reported as the oracle's product rate in the
    metric's unit, with the time per iteration and the time to eigenvectors
    it implies at the GPU's FP64 iteration count."""
    import numpy as np
    import graphgen
    from oracle import _native, eigen, laplacian as lap, precond
    threads = _native.default_threads()
    op0 = lap.operator(g.rowptr, g.col, g.w, lap.COMBINATORIAL, fast=True)
    stat = {"bytes": 0.0, "secs": 0.0, "calls": 0}
    nnz = float(g.nnz)

    def op(Z):
        t0 = time.perf_counter()
        Y = op0(Z)
        stat["secs"] += time.perf_counter() - t0
        k = 1 if Z.ndim == 1 else Z.shape[1]
        stat["bytes"] += 4.0 * (g.n + 1) + 4.0 * nnz + 2.0 * g.n * k * 8
        stat["calls"] += 1
        return Y

    deg = lap.degrees_fast(g.rowptr, g.col, g.w)
    hi = precond.gershgorin_bound(deg, lap.COMBINATORIAL)
    pre = lambda R: precond.chebyshev(g.rowptr, g.col, g.w, R, opts.cheb_degree,  # noqa: E731
                                      hi / opts.cheb_ratio, hi, op=op)
    X0 = graphgen.normal_block(g.n, m, 2)
    # iterations that fit the budget: one untimed probe iteration sizes it
    t0 = time.perf_counter()
    eigen.lobpcg(g.rowptr, g.col, g.w, lap.COMBINATORIAL, X0, pre, opts.tol, maxiter=1,
                 op=op, bd=np.ones(g.n))
    per_it = time.perf_counter() - t0
    its = max(2, min(gpu_fp64_iterations, int(budget_s / max(per_it, 1e-3))))
    stat.update(bytes=0.0, secs=0.0, calls=0)
    t0 = time.perf_counter()
    _, _, done, rho = eigen.lobpcg(g.rowptr, g.col, g.w, lap.COMBINATORIAL, X0, pre, opts.tol,
                                   maxiter=its, op=op, bd=np.ones(g.n))
    dt = time.perf_counter() - t0
    # the final explicit residual product inside lobpcg is one more call
    per_iter = dt / max(done, 1)
    return {
        "value": round(stat["bytes"] / stat["secs"] / 1e9, 3), "unit": "GB/s",
        "cores": threads, "kind": "oracle",
        "sample": (f"{done} LOBPCG iterations of the oracle (FP64, C/OpenMP Laplacian product, "
                   f"Chebyshev degree {opts.cheb_degree}, ratio {opts.cheb_ratio:g}) on the "
                   f"128^3 7-point grid with d = {m}, {threads} threads, {dt:.1f} s; value = "
                   f"its Laplacian-product rate over {stat['calls']} products"),
        "seconds_per_iteration": round(per_iter, 3),
        "est_time_to_eigvecs_s": round(per_iter * gpu_fp64_iterations, 1),
        "est_basis": f"{gpu_fp64_iterations} iterations (the GPU FP64 solve's count)",
        "converged_in_sample": bool(np.all(rho <= opts.tol)),
        "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
        "host_triad_gbs": round(host_triad_gbs(threads), 1),
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cheb_step_grid7_128_traffic.md")
KERNEL_SOURCES = ["paper_2105_00578_amd/csrc/spmm_vec.hip", "paper_2105_00578_amd/csrc/kernels.h",
                  "paper_2105_00578_amd/csrc/common.h"]


def kernel_hash():
    import hashlib
    h = hashlib.sha1()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """Counter-derived HBM bytes per launch of the Chebyshev step, if the
    committed counter summary was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("<!-- traffic:"):
                rec = json.loads(line[len("<!-- traffic:"):].rsplit("-->", 1)[0])
                if rec.get("kernel_src_sha1") == kernel_hash():
                    return rec
    return None


def copy_probe(nbytes):
    """One plain elementwise copy of nbytes on the GPU (reads and writes
    nbytes once each): the calibration kernel of the byte counters."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    y = x * 1.0
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "check": float(y[-1].item())}), flush=True)


# Workloads.  The default is the configuration the headline metric is quoted
# on; the others are the remaining configurations of the path, the paper's
# Brick3D meshes (Table of preconditioner results, K = 24, Jacobi) and the
# normalized problem on the power-law graph.
WORKLOADS = {
    "grid7_128": dict(graph="grid7_128", K=64, precond="cheb", side=128,
                      desc="3D 7-point grid 128^3, combinatorial Laplacian, K=64 (d=7), "
                           "LOBPCG + Chebyshev degree 25, tol 1e-3"),
    "rmat22": dict(graph="rmat22", K=16, precond="jacobi",
                   desc="R-MAT scale 22 (LCC), generalized Laplacian, K=16 (d=5), "
                        "LOBPCG + Jacobi, tol 1e-2, piecewise-constant start"),
    "rmat22-cheb": dict(graph="rmat22", K=16, precond="cheb",
                        desc="R-MAT scale 22 (LCC), normalized Laplacian, K=16 (d=5), "
                             "LOBPCG + Chebyshev degree 25, tol 1e-2, piecewise-constant start"),
    "brick96lr": dict(graph="brick96lr", K=256, precond="jacobi",
                      desc="3D 27-point 96^3 + 1% long-range edges, weights U[0.5,1.5) FP32, "
                           "combinatorial, K=256 (d=9), LOBPCG + Jacobi, tol 1e-3"),
    "brick100": dict(graph="brick100", K=24, precond="jacobi",
                     desc="Galeri Brick3D 27-point 100^3, combinatorial, K=24 (d=5), "
                          "LOBPCG + Jacobi, tol 1e-3 (the paper's preconditioner table)"),
    "brick200": dict(graph="brick200", K=24, precond="jacobi",
                     desc="Galeri Brick3D 27-point 200^3, combinatorial, K=24 (d=5), "
                          "LOBPCG + Jacobi, tol 1e-3"),
    "brick400": dict(graph="brick400", K=24, precond="jacobi",
                     desc="Galeri Brick3D 27-point 400^3, combinatorial, K=24 (d=5), "
                          "LOBPCG + Jacobi, tol 1e-3 (the paper's preconditioner table)"),
    "brick400-cheb": dict(graph="brick400", K=24, precond="cheb",
                          desc="Galeri Brick3D 27-point 400^3, combinatorial, K=24 (d=5), "
                               "LOBPCG + Chebyshev degree 25, tol 1e-3"),
    "brick100-cheb": dict(graph="brick100", K=24, precond="cheb",
                          desc="Galeri Brick3D 27-point 100^3, combinatorial, K=24 (d=5), "
                               "LOBPCG + Chebyshev degree 25, tol 1e-3"),
    "grid7_128-gmres": dict(graph="grid7_128", K=64, precond="gmres",
                            desc="3D 7-point grid 128^3, combinatorial Laplacian, K=64 (d=7), "
                                 "LOBPCG + GMRES polynomial degree 25, tol 1e-3"),
    "brick100-gmres": dict(graph="brick100", K=24, precond="gmres",
                           desc="Galeri Brick3D 27-point 100^3, combinatorial, K=24 (d=5), "
                                "LOBPCG + GMRES polynomial degree 25, tol 1e-3"),
    "rmat22-gmres": dict(graph="rmat22", K=16, precond="gmres",
                         desc="R-MAT scale 22 (LCC), normalized Laplacian, K=16 (d=5), "
                              "LOBPCG + GMRES polynomial degree 25, tol 1e-2, piecewise start"),
}


def run(args):
    import numpy as np
    import torch

    import graphgen
    import paper_2105_00578_amd as sx

    wl = WORKLOADS[args.workload]
    headline = args.workload == "grid7_128"
    g = graphgen.config_graph(wl["graph"], scale_down=args.scale_down)
    dev = torch.device("cuda", 0)
    h = sx.Handle(0)
    rp = g.rowptr.astype(np.int64 if g.rowptr[-1] >= 2 ** 31 else np.int32)
    wt = None if g.w is None else torch.from_numpy(g.w).to(dev)
    G = sx.Graph(h, torch.from_numpy(rp).to(dev), torch.from_numpy(g.col).to(dev), wt,
                 validate=True)
    reg, _, _ = G.info()
    K = wl["K"]
    d = sx.num_eigenvectors(K)
    pc = {"cheb": sx.PRECOND_CHEBYSHEV, "gmres": sx.PRECOND_GMRES,
          "jacobi": sx.PRECOND_JACOBI}[wl["precond"]]
    base = dict(cheb_degree=25, cheb_ratio=args.cheb_ratio, seed=12345)
    opts = {
        "mixed": sx.options_default(reg, pc, precision=sx.MIXED, **base),
        "fp64": sx.options_default(reg, pc, precision=sx.FP64, **base),
    }
    results = {}
    last = {}
    for name in (("mixed",) if args.only_mixed else ("mixed", "fp64")):
        o = opts[name]
        # timed steps and the time to eigenvectors without per-launch events
        # (the library's default); kernel durations from an instrumented pass
        h.set_timing(False)
        for _ in range(args.warmup):
            sx.partition(h, G, K, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = []
        for _ in range(args.steps):
            outs.append(sx.partition(h, G, K, o))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps * 1e3
        lam, V, part, cut, imb, st = outs[-1]
        last[name] = outs[-1]
        if args.no_instrumented:
            # one pass only (very large meshes): the partition's own device
            # time stands for the time to eigenvectors (it also holds the
            # split and cut, about 1 % of it) and phase times are not taken
            eig_ms = [s[5].ms_total for s in outs]
            sts = [s[5] for s in outs]
        else:
            eig_ms = [sx.eigensolve(h, G, d, o)[2].ms_total for _ in range(args.steps)]
            h.set_timing(True)
            sts = [sx.partition(h, G, K, o)[5] for _ in range(args.steps)]
            h.set_timing(False)
        gbp = sum(s.gb_precond for s in sts)
        msp = sum(s.phases_ms["precond"] for s in sts)
        gbs = sum(s.gb_spmm for s in sts)
        mss = sum(s.phases_ms["spmm"] for s in sts)
        r = dict(
            ms_per_step=dt, time_to_eigvecs_ms=float(np.median(eig_ms)),
            iterations=st.iterations, promoted=int(st.promoted), rho_max=max(st.rho[:d]),
            cut=cut, imbalance=imb,
            cheb_gbs=gbp / (msp * 1e-3) if msp > 0 else 0.0,
            cheb_avg_us=msp / max(1, sum(s.precond_calls for s in sts)) * 1e3,
            cheb_calls=sum(s.precond_calls for s in sts),
            avg_active_cols=sum(s.precond_cols for s in sts) / max(1, sum(s.iterations for s in sts)),
            col_index_bytes=st.col_index_bytes,
            spmm_gbs=gbs / (mss * 1e-3) if mss > 0 else 0.0,
            spmm_calls=sum(s.spmm_calls for s in sts),
            phases_ms={k: round(v / 1.0, 3) for k, v in sts[-1].phases_ms.items()},
            lam=lam)
        if headline:
            relerr, trivial, sin, gap = closed_form_check(lam, V.cpu().numpy(), wl["side"] // args.scale_down)
            r.update(eig_relerr_max=relerr, trivial_rel=trivial, subspace_sin=sin)
        results[name] = r
    mx = results["mixed"]
    f64 = results.get("fp64", mx)
    cheb = pc in (sx.PRECOND_CHEBYSHEV, sx.PRECOND_GMRES)
    value = mx["cheb_gbs"] if cheb else mx["spmm_gbs"]
    tr = measured_traffic() if headline else None
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mx["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{wl['desc']} (n={g.n}, nnz={g.nnz}); FP32 SpMM/updates with FP64 Gram "
                        f"and Rayleigh-Ritz vs all-FP64",
            "n": g.n, "nnz": int(g.nnz), "K": K, "nev": d,
            "problem": ["combinatorial", "generalized", "normalized"][opts["mixed"].problem],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(value, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(value / HBM_PEAK_GBS, 4),
            "traffic": None if tr is None else tr["bytes_per_launch"],
            "kernel": (("Chebyshev-step" if pc == sx.PRECOND_CHEBYSHEV else "GMRES-polynomial-step")
                       + " Laplacian product (FP32)" if cheb else
                       "Laplacian products with the fused residual / Jacobi epilogue (FP32)"),
            "avg_launch_us": round(mx["cheb_avg_us"], 3) if cheb else None,
            "launches": mx["cheb_calls"] if cheb else mx["spmm_calls"],
            "avg_active_cols": round(mx["avg_active_cols"], 3),
            # the kernel reads this many bytes per column index (2: int16
            # offsets from the row); `achieved` counts 4, the int32 CSR input
            "col_index_bytes_read": mx["col_index_bytes"],
        },
        "time_to_eigvecs_ms": {"mixed": round(mx["time_to_eigvecs_ms"], 3),
                               "fp64": round(f64["time_to_eigvecs_ms"], 3)},
        "speedup_mixed_vs_fp64": round(f64["time_to_eigvecs_ms"] / mx["time_to_eigvecs_ms"], 3),
        "ms_per_step_fp64": round(f64["ms_per_step"], 3),
        "spmm_gbs_fp64": round(f64["cheb_gbs"] if cheb else f64["spmm_gbs"], 2),
        "iterations": {"mixed": mx["iterations"], "fp64": f64["iterations"]},
        "promoted": mx["promoted"],
        "rho_max": {"mixed": mx["rho_max"], "fp64": f64["rho_max"]},
        "cut": {"mixed": mx["cut"], "fp64": f64["cut"]},
        "imbalance": {"mixed": mx["imbalance"], "fp64": f64["imbalance"]},
        "phase_ms_last_step": {"mixed": mx["phases_ms"], "fp64": f64["phases_ms"]},
    }
    if headline:
        line["config"]["cheb_ratio"] = args.cheb_ratio
        line["eig_relerr_max_vs_closed_form"] = {"mixed": mx["eig_relerr_max"],
                                                 "fp64": f64["eig_relerr_max"]}
        line["subspace_sin_vs_closed_form"] = {"mixed": mx["subspace_sin"],
                                               "fp64": f64["subspace_sin"]}
    if args.repartition:
        line["repartition"] = repartition(h, G, g, K, opts["mixed"], last["mixed"], dev)
    if headline and not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(g, d, f64["iterations"], opts["fp64"])
    return line


ADJOINT_WORKLOADS = {
    "adjoint-rmat18": dict(graph="rmat18", precond="jacobi",
                           desc="R-MAT scale 18 (LCC), weights U[0.5,1.5) FP64, generalized, "
                                "7 eigenpairs (tol 1e-10), loss = sum lambda_1..4 + "
                                "||V_1..4 - V_target||^2"),
    "adjoint-king512": dict(graph="king512", precond="cheb",
                            desc="9-point grid 512^2, weights U[0.5,1.5) FP64, generalized, "
                                 "7 eigenpairs (tol 5e-10), loss = sum lambda_1..4 + "
                                 "||V_1..4 - V_target||^2"),
}


def run_adjoint(args):
    """The differentiation workloads: EigFn forward (FP64 eigensolve) and the
    hand-written backward (adjoint kernels + projected CG), timed per step."""
    import numpy as np
    import torch

    import graphgen
    import paper_2105_00578_amd as sx

    wl = ADJOINT_WORKLOADS[args.workload]
    g = graphgen.config_graph(wl["graph"])
    dev = torch.device("cuda", 0)
    h = sx.Handle(0)
    rp = torch.from_numpy(g.rowptr.astype(np.int32)).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    w0 = torch.from_numpy(g.w).to(dev)
    target = torch.from_numpy(graphgen.normal_block(g.n, 4, 3) / np.sqrt(g.n)).to(dev)
    pre = sx.PRECOND_CHEBYSHEV if wl["precond"] == "cheb" else sx.PRECOND_JACOBI
    opts = sx.Options(problem=sx.GENERALIZED, precond=pre, precision=sx.FP64,
                      tol=5e-10 if wl["graph"] == "king512" else 1e-10, max_iter=20000)
    r = torch.from_numpy(np.repeat(np.arange(g.n), np.diff(g.rowptr))).to(dev)
    bd = torch.zeros(g.n, dtype=torch.float64, device=dev).index_add_(0, r, w0)
    fwd, bwd, cg = [], [], []
    for step in range(args.warmup + args.steps):
        wt = w0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, V = sx.EigFn.apply(wt, h, rp, col, 7, opts, None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Vs = V[:, 1:5]
        sign = torch.sign(((Vs * bd[:, None]) * target).sum(0)).detach()
        loss = lam[1:5].sum() + ((Vs * sign - target) ** 2).sum()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if step >= args.warmup:
            fwd.append((t1 - t0) * 1e3)
            bwd.append((t3 - t2) * 1e3)
            cg.append(sx.backward_info(h))
    return {
        "workload": args.workload, "config": f"{wl['desc']} (n={g.n}, nnz={g.nnz})",
        "steps": args.steps, "warmup": args.warmup,
        "forward_ms": round(float(np.median(fwd)), 3),
        "backward_ms": round(float(np.median(bwd)), 3),
        "cg_steps": cg[-1][0], "cg_rel_residual": cg[-1][1],
        "data": "synthetic", "dtype": "f64",
    }


def repartition(h, G, g, K, o, out, dev):
    """Greedy refinement of the timed mixed partition (eps = 1 %), and a
    warm-started repartition after the edge weights drift by up to 1 %: the
    previous eigenvectors as the initial block against a cold start."""
    import copy

    import numpy as np
    import torch

    import graphgen
    import paper_2105_00578_amd as sx

    lam, V, part, cut0, imb0, st = out
    times = []
    for rep in range(2):                       # the first call warms the kernels up
        p = part.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cut, imb, kept, moves = sx.refine(h, G, p, K, eps=0.01)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    res = {"refine": {"eps": 0.01, "ms": round(times[-1], 3), "cut_before": cut0,
                      "cut_after": cut, "imbalance_after": imb, "passes_kept": kept,
                      "moves": moves}}
    g1 = graphgen.perturb_weights(g, 0.01, 1, dtype=np.float32)
    rp = g1.rowptr.astype(np.int64 if g1.rowptr[-1] >= 2 ** 31 else np.int32)
    G1 = sx.Graph(h, torch.from_numpy(rp).to(dev), torch.from_numpy(g1.col).to(dev),
                  torch.from_numpy(g1.w).to(dev))
    warm = copy.copy(o)
    warm.init = sx.INIT_USER
    row = {}
    for name, oo, X0 in (("cold", o, None), ("warm", warm, V)):
        sx.partition(h, G1, K, oo, X0=X0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sx.partition(h, G1, K, oo, X0=X0)
        torch.cuda.synchronize()
        row[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 3),
                     "iterations": r[5].iterations, "cut": r[3]}
    res["warm_start"] = {"weight_drift": 0.01, **row}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cheb-ratio", type=float, default=1000.0)
    ap.add_argument("--scale-down", type=int, default=1, help="shrink the grid (tests only)")
    ap.add_argument("--only-mixed", action="store_true",
                    help="time only the mixed-precision partition (counter runs)")
    ap.add_argument("--workload", default="grid7_128",
                    choices=sorted(WORKLOADS) + sorted(ADJOINT_WORKLOADS),
                    help="configuration to time (default: the headline 128^3 grid)")
    ap.add_argument("--repartition", action="store_true",
                    help="also time the greedy refinement of the partition and a "
                         "warm-started repartition after a 1 %% weight drift")
    ap.add_argument("--no-instrumented", action="store_true",
                    help="skip the separate eigensolve and per-launch-event passes "
                         "(for the largest meshes); GB/s fields are then 0")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="run one plain device copy of this many bytes and exit")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build has no "
              "multi-GPU path; the whole graph is the one-GPU share.", file=sys.stderr)
        sys.exit(2)
    line = run_adjoint(args) if args.workload in ADJOINT_WORKLOADS else run(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
