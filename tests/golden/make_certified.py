"""Write the certified eigenpair fixtures tests/golden/certified_<name>.json.

Calls only the seeded generators (graphgen) and the oracle (oracle.certify):
no value here comes from the GPU path.  Each workload is solved from two
independent random start blocks; both runs are stored, and the tests require
that they agree (support for the ordering assumption of oracle.certify).

    python tests/golden/make_certified.py [name ...]

Names: rmat22 (R-MAT scale 22 LCC, generalized, K = 16 -> d = 5),
brick96lr (27-point 96^3 + 1 % long-range edges, weights U[0.5, 1.5),
combinatorial, K = 256 -> d = 9), king512 (9-point 512^2, weights U[0.5, 1.5),
generalized, d = 7), rmat18 (R-MAT scale 18 LCC, weights U[0.5, 1.5),
generalized, d = 7) and brick100 (the paper's Brick3D 27-point 100^3 mesh,
unit weights, combinatorial, K = 24 -> d = 5).  Runtimes on 8 host cores: minutes (king512, rmat18) to
tens of minutes (rmat22, brick96lr).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
from oracle import certify, laplacian as lap  # noqa: E402

WORKLOADS = {
    # name: (problem, d, preconditioner of the oracle's own solve)
    "rmat22": (lap.GENERALIZED, 5, "jacobi"),
    "brick96lr": (lap.COMBINATORIAL, 9, "chebyshev"),
    "king512": (lap.GENERALIZED, 7, "chebyshev"),
    "rmat18": (lap.GENERALIZED, 7, "jacobi"),
    "brick100": (lap.COMBINATORIAL, 5, "chebyshev"),
}
SEEDS = (7, 8)
GUARDS = 4
TOL = 1e-10
GUARD_TOL = 1e-8
# a leading block of k columns counts as separated when the certified lower
# bound of lambda_k exceeds theta_{k-1} by this fraction of theta_k
GAP_REL = 0.02


def graph_digest(g) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g.rowptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(g.col, dtype=np.int32).tobytes())
    if g.w is not None:
        h.update(np.ascontiguousarray(g.w, dtype=np.float64).tobytes())
    return h.hexdigest()


def run(name: str) -> dict:
    problem, d, prec = WORKLOADS[name]
    t0 = time.time()
    g = graphgen.config_graph(name)
    print(f"{name}: n={g.n} nnz={g.nnz} built in {time.time() - t0:.1f} s", flush=True)
    runs = []
    for seed in SEEDS:
        r = certify.certified_eigenpairs(g.rowptr, g.col, g.w, problem, d,
                                         guards=GUARDS, tol=TOL, guard_tol=GUARD_TOL,
                                         seed=seed, prec=prec, log=print)
        runs.append(r)
        print(f"  seed {seed}: theta {r['theta']}", flush=True)
    r0 = runs[0]
    th, eps = r0["theta"], r0["eps"]
    lam_lo = th - eps                      # Weinstein, under the ordering assumption
    gapped = [k for k in range(2, d + 1)
              if lam_lo[k] - th[k - 1] >= GAP_REL * th[k]]
    out = {
        "name": name,
        "recipe": graphgen.CONFIGS[name],
        "n": int(g.n), "nnz": int(g.nnz), "sha256": graph_digest(g),
        "problem": {lap.COMBINATORIAL: "combinatorial", lap.GENERALIZED: "generalized",
                    lap.NORMALIZED: "normalized"}[problem],
        "d": d, "guards": GUARDS, "tol": TOL, "guard_tol": GUARD_TOL, "oracle_precond": prec,
        "theta": th.tolist(), "eps": eps.tolist(), "lam_lo": lam_lo.tolist(),
        "delta": r0["delta"], "eig_bound": r0["eig_bound"], "sin_bound": r0["sin_bound"],
        "gapped_blocks": gapped,
        "runs": [{"seed": s, "theta": r["theta"].tolist(), "eps": r["eps"].tolist(),
                  "iterations": r["iterations"], "seconds": round(r["seconds"], 1)}
                 for s, r in zip(SEEDS, runs)],
    }
    path = os.path.join(HERE, f"certified_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} ({time.time() - t0:.0f} s)", flush=True)
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    for nm in names:
        run(nm)
