"""Writes the full-size FGMRES fixtures of tests/golden/ from the oracle alone.

For each workload below the oracle assembles the hierarchy (oracle.problems),
factors every patch (oracle.relax / oracle.lu), runs restarted FGMRES(30)
right-preconditioned by its phMG V-cycle (oracle.fgmres, oracle.multigrid) to
a relative residual of 1e-8 from x = 0 -- the solver of Section 4 -- and
stores what a GPU run can be checked against without re-running the oracle:

  iters, converged, relres        FGMRES counts and the true relative residual
  history                         |g_{j+1}| / ||r_0|| per inner iteration
  margin                          min_j | history_j / rtol - 1 |
  norm2, norminf                  norms of the solution with its pressure
                                  mean removed (the constant-pressure kernel)
  idx, val                        a seeded sample of that solution's entries

Nothing here imports the GPU package.  Run from the repository root:
    OMP_NUM_THREADS=1 python tests/golden/make_fullsize_golden.py cfg2
(one workload per process; cfg3 also runs with k=3, and cfg3_bumps solves 4 of
the 16 Gaussian-bump right-hand sides, columns 0, 5, 10 and 15).  Each run takes minutes to an hour of CPU.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fgmres as ofgmres  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
from oracle import problems as oproblems  # noqa: E402

NSAMPLE = 2048
RTOL = 1e-8

JOBS = {
    # name: (workload, k, forcing, columns)
    "cfg2": ("cfg2", None, "mms", [0]),
    "cfg3": ("cfg3", 4, "mms", [0]),
    "cfg3_k3": ("cfg3", 3, "mms", [0]),
    "cfg3_bumps": ("cfg3", 4, "bumps", [0, 5, 10, 15]),
    "cfg4": ("cfg4", None, "mms", [0]),
}


def normalise(x: np.ndarray, nfu: int, dim: int = 2) -> np.ndarray:
    y = np.array(x, copy=True)
    y[dim * nfu:] -= y[dim * nfu:].mean()
    return y


def run(job: str) -> str:
    name, k, forcing, cols = JOBS[job]
    t0 = time.perf_counter()
    kw = dict(forcing=forcing)
    if forcing == "bumps":
        kw["nrhs"] = 16
    levels, discs, opts, b = oproblems.build(name, k=k, **kw)
    omg.setup(levels, opts)
    t_setup = time.perf_counter() - t0
    K0 = levels[0].K
    n = K0.shape[0]
    nfu = discs[0].nfu
    out = {"workload": name, "k": k if k is not None else discs[0].k, "forcing": forcing, "rtol": RTOL,
           "restart": 30, "n": int(n), "nfu": int(nfu), "levels_n": [int(L.n) for L in levels],
           "lambda_max": [float(L.lmax) for L in levels[:-1]] if opts.smoother == "chebyshev" else None,
           "oracle_setup_s": round(t_setup, 1), "columns": []}
    rng = np.random.default_rng(20240707)
    idx = np.sort(rng.choice(n, size=min(NSAMPLE, n), replace=False))
    out["idx"] = idx.tolist()
    B = b if b.ndim == 2 else b[None, :]
    for c in cols:
        t1 = time.perf_counter()
        res = ofgmres.fgmres(lambda v: K0 @ v, lambda v: omg.vcycle(levels, opts, v), B[c], rtol=RTOL,
                             restart=30, maxit=1000)
        x = normalise(res.x, nfu)
        hist = np.asarray(res.history)
        out["columns"].append({
            "column": c, "iters": res.iters, "converged": bool(res.converged), "relres": float(res.relres),
            "history": [float(h) for h in hist], "margin": float(np.min(np.abs(hist / RTOL - 1.0))),
            "norm2": float(np.linalg.norm(x)), "norminf": float(np.abs(x).max()),
            "b_norm2": float(np.linalg.norm(B[c])), "val": [float(v) for v in x[idx]],
            "oracle_solve_s": round(time.perf_counter() - t1, 1)})
        print(f"{job} column {c}: {res.iters} iterations, relres {res.relres:.3e}, "
              f"{time.perf_counter() - t1:.0f} s", flush=True)
    path = os.path.join(HERE, f"fgmres_{job}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0, separators=(",", ":"))
        f.write("\n")
    return path


if __name__ == "__main__":
    for job in sys.argv[1:] or ["cfg2"]:
        print(run(job), flush=True)
