#!/usr/bin/env python3
"""Benchmark of the Vanka-star / phMG / FGMRES hot path on one MI355X.

Workload (default, "cfg3"): Taylor-Hood P4/P3 Stokes on the structured 128 x 128
unit-square mesh (670 467 free DoFs), direct p-coarsening to P2/P1 on the same
mesh, then P2/P1 on 64^2 ... 8^2 and a dense coarse solve; Vanka-star patches of
18-141 DoFs; nu = 2 Chebyshev steps of the additive Schwarz smoother; 16 seeded
Gaussian-bump forcings (homogeneous Dirichlet data) solved together.  Synthetic
inputs stand in for the paper's cavity / step problems.

One timed step = the whole hot path on the resident hierarchy for one batch of
16 right-hand sides: relaxation set-up (patch extraction + patch inversion on
every level, coarse inverse, Chebyshev eigenvalue estimates) followed by
FGMRES(30) to a relative residual of 1e-8 from x = 0 for all 16 systems
(lockstep, MFMA block patch solves), FP64.

Printed: one JSON line.  `value` is the achieved HBM bandwidth of the level-0
patch solve in FP64 -- the method's bytes per launch (the symmetric patch
inverse's m(m+1)/2 words, DoF index, gathered residual, staged result) divided
by the mean launch duration from HIP events on the library's stream -- the
"Vanka patch-apply HBM GB/s" half of the metric; the "time-to-1e-8, mixed vs
FP64" half is the step time for FP64, FP32 and BF16 patch inverses, each with
its error against the FP64 oracle's stored solutions (tests/golden/).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Vanka patch-apply HBM GB/s; phMG-FGMRES time-to-1e-8, mixed vs FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6      # dense FP64 MFMA peak of MI355X
GOLDEN = os.path.join(ROOT, "tests", "golden")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "patch_apply_traffic.json")
# the patch solve's source: the kernel and the shared header with its layout helpers and reductions
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2407_07253_amd", "csrc", f) for f in ("patch_apply.hip", "phmg_internal.h")]
PRECS = ("f64", "f32", "bf16")
ES = {"f64": 8, "f32": 4, "bf16": 2}

WORKLOADS = {
    "cfg3": "TH P4/P3 2D structured 128x128 (670467 DoFs); phMG direct P4/P3 -> P2/P1 -> 4 h-levels; "
            "Vanka-star patches 18-141 DoFs; 16 seeded Gaussian-bump right-hand sides",
    "cfg2": "TH P4/P3 2D, Delaunay 64 seeded pts + corners, 3 refinements (170483 DoFs); phMG direct "
            "P4/P3 -> P2/P1 -> 3 h-levels; Vanka-star patches 64-210 DoFs",
    "cfg4": "SV P4/P3disc 2D on the Alfeld split of a jittered 16x16 mesh refined twice (637954 DoFs)",
    "cfg1": "TH P2/P1 2D, structured 8x8 (531 DoFs); hMG 2 levels; nu=2, omega=0.5",
}


def _fmt(v):
    return float(f"{v:.6g}") if isinstance(v, float) else v


# --------------------------------------------------------------------------
# byte and flop counts
# --------------------------------------------------------------------------
def patch_sizes(fl):
    import numpy as np
    return np.diff(np.asarray(fl.patch_ptr)).astype(np.int64)


def method_apply_bytes(m, es: int, sym: bool) -> int:
    """Method bytes of one patch-solve launch: the patch inverse's words read once (m(m+1)/2 for the
    symmetric inverse of a symmetric level, m^2 otherwise), per slot the DoF index (4 B), the gathered
    residual (8 B) and the staged result (8 B), per patch order + ptr + offset (20 B)."""
    words = int((m * (m + 1) // 2).sum()) if sym else int((m * m).sum())
    return es * words + 20 * int(m.sum()) + 20 * len(m)


def layout_apply_bytes(m, es: int, sym: bool) -> int:
    """Bytes the kernel's stored layout streams: general m^2 words; symmetric strips of 16 rows hold the
    strictly lower part of the strip (height padded to the 16-byte row group V = 16 / es) and the diagonal
    block from row floor(c / G) G down in column c (G = V for float64 / float32, 16 for bfloat16)."""
    import numpy as np
    if not sym:
        return method_apply_bytes(m, es, False)
    V = 16 // es
    G = V if V < 8 else 16
    m = np.asarray(m, dtype=np.int64)
    ns = (m + 15) // 16
    h = m - (ns - 1) * 16
    hp = (h + V - 1) // V * V

    def diag(hh, hpp):                       # stored entries of a diagonal block of hh columns, height hpp
        c = np.arange(16)
        g = c // G * G
        return np.where(c[None, :] < np.asarray(hh)[:, None], np.asarray(hpp)[:, None] - g[None, :], 0).sum(axis=1)

    full = int(diag(np.array([16]), np.array([16]))[0])
    words = 128 * (ns - 1) * (ns - 2) + full * (ns - 1) + 16 * hp * (ns - 1) + diag(h, hp)
    return es * int(words.sum()) + 20 * int(m.sum()) + 20 * len(m)


def method_block_bytes(m, es: int, sym: bool, nrhs: int = 16) -> int:
    """Method bytes of one 16-system block patch solve: factor words once for all systems, per slot the
    index and the gathered and staged 16-wide rows (2 x 8 x 16 B)."""
    words = int((m * (m + 1) // 2).sum()) if sym else int((m * m).sum())
    return es * words + (4 + 16 * nrhs) * int(m.sum()) + 20 * len(m)


def kernel_source_sha() -> str:
    """SHA-256 over the patch solve's source files, in order."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def traffic_entry(workload: str, prec: str):
    """Counter-measured HBM bytes per launch from the committed rocprofv3 summary, when it covers this
    workload and the kernel source is unchanged."""
    try:
        d = json.load(open(TRAFFIC_FILE))
        if d.get("kernel_source_sha256") != kernel_source_sha():
            return None
        return float(d["per_launch_bytes"][workload][prec])
    except Exception:
        return None


def golden(job: str):
    path = os.path.join(GOLDEN, f"fgmres_{job}.json")
    return json.load(open(path)) if os.path.exists(path) else None


def oracle_error(x, g, column: int):
    """Relative error of a solution against the FP64 oracle's stored sample (pressure mean removed)."""
    import numpy as np
    col = next(c for c in g["columns"] if c["column"] == column)
    y = np.array(x, dtype=np.float64, copy=True)
    y[2 * g["nfu"]:] -= y[2 * g["nfu"]:].mean()
    idx = np.asarray(g["idx"])
    val = np.asarray(col["val"])
    return float(np.abs(y[idx] - val).max() / np.abs(val).max())


# --------------------------------------------------------------------------
# CPU baseline: the oracle on the host
# --------------------------------------------------------------------------
def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(workload: str, sweeps_per_cycle: int, iters: int, budget_s: float = 20.0) -> dict:
    """The plain FP64 oracle on a bounded sample of the level-0 patches of the workload.

    The oracle assembles level 0 and builds its patches (untimed), then on every stride-th patch
    times its set-up (patch extraction + LU with partial pivoting) and its share of a relaxation
    sweep (LU solve of the gathered residual), and times one residual K x.  Per-patch figures are
    scaled to all patches: one level-0 sweep = residual + all patch solves; set-up = all
    extractions + LUs; FGMRES = iterations x the level-0 sweeps of one cycle (lower levels not
    counted: a lower bound, labelled as extrapolated).  BLAS threads are set to all host cores; the
    oracle's per-patch work is sequential Python over small arrays, so one core does the work."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.discretization import assemble_stokes
    from oracle.lu import lu_factor, lu_solve
    from oracle.patches import vanka_star_patches
    from oracle.problems import level_specs
    from oracle.relax import extract_patch

    nproc = os.cpu_count() or 1
    with threadpool_limits(limits=nproc):
        meshes = synth.config_mesh_hierarchy(workload)[::-1]
        specs, _ = level_specs(workload)
        mi, k, kind = specs[0]
        d = assemble_stokes(meshes[mi], k, kind)
        patches = vanka_star_patches(d)
        K = d.K
        rng = np.random.default_rng(0)
        x = rng.standard_normal(d.n)
        t0 = time.perf_counter()
        reps = 0
        while reps < 3 or time.perf_counter() - t0 < 1.0:
            r = x - K @ x
            reps += 1
        t_res = (time.perf_counter() - t0) / reps
        stride = max(1, len(patches) // 400)
        sample = patches[::stride]
        t0 = time.perf_counter()
        facs = [lu_factor(extract_patch(K, S)) for S in sample]
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        passes = 0
        while True:
            for S, (LU, piv) in zip(sample, facs):
                lu_solve(LU, piv, r[S])
            passes += 1
            if time.perf_counter() - t0 > budget_s or passes >= 200:
                break
        t_solve = (time.perf_counter() - t0) / passes
    m = np.array([len(S) for S in sample], dtype=np.int64)
    mall = np.array([len(S) for S in patches], dtype=np.int64)
    scale = len(patches) / len(sample)
    sweep_s = t_res + t_solve * scale
    return {
        "value": method_apply_bytes(m, 8, False) / t_solve / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{workload} level 0: the oracle's LU solve of the gathered residual on {len(sample)} of the "
                  f"{len(patches)} patches (every {stride}th), {passes} passes; value = method bytes of those "
                  f"solves (8 m^2 + 20 m + 20 per patch: the oracle stores full LU factors) / time",
        "cpu_model": cpu_model(),
        "nproc": nproc,
        "blas_threads": nproc,
        "level0_sweep_s": _fmt(sweep_s),
        "level0_sweep_s_note": "residual K x timed in full + patch solves scaled from the sample by patch count",
        "setup_s": _fmt(t_setup * scale),
        "setup_s_note": "extraction + LU of the sampled patches scaled by patch count",
        "fgmres_s_extrapolated": _fmt(iters * sweeps_per_cycle * sweep_s),
        "fgmres_s_note": f"{iters} iterations x {sweeps_per_cycle} level-0 sweeps per cycle (lower levels not "
                         f"counted: a lower bound)",
        "level0_patches": len(patches),
        "level0_sum_m2": int((mall * mall).sum()),
    }


# --------------------------------------------------------------------------
# GPU legs
# --------------------------------------------------------------------------
def make_hierarchy(workload: str, k=None, forcing: str = "mms", nrhs: int = 1):
    from paper_2407_07253_amd import frontend
    from paper_2407_07253_amd._lib import Hierarchy
    t0 = time.perf_counter()
    fh = frontend.build_hierarchy(workload, k=k, forcing=forcing, nrhs=nrhs)
    return fh, Hierarchy.from_frontend(fh), time.perf_counter() - t0


def set_precision(H, fh, prec: str):
    for l in range(len(fh.levels) - 1):
        H.set_precision(l, prec)


def apply_leg(H, fh, prec: str, reps: int, workload: str) -> dict:
    """Level-0 single-system patch solve: HIP events on the library's stream around `reps` sweeps."""
    import torch
    set_precision(H, fh, prec)
    H.setup()
    n0 = fh.levels[0].n
    b = torch.ones(n0, dtype=torch.float64, device="cuda")
    xs = torch.zeros_like(b)
    for _ in range(3):
        H.relax_apply(0, b, xs, 1)
    H.profile(["patch_apply", "spmv", "scatter"])
    H.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        H.relax_apply(0, b, xs, 1)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / reps
    ms, cnt = H.profile_read("patch_apply", 0)
    ms_sp, c_sp = H.profile_read("spmv", 0)
    ms_sc, c_sc = H.profile_read("scatter", 0)
    H.profile([])
    info = H.level_info(0)
    sym = info["symmetric_storage"]
    m = patch_sizes(fh.levels[0])
    avg = ms / max(cnt, 1)
    mb = method_apply_bytes(m, ES[prec], sym)
    lb = layout_apply_bytes(m, ES[prec], sym)
    return {"avg_ms": avg, "launches": cnt, "sym": sym, "method_bytes": mb, "layout_bytes": lb,
            "gbps": mb / (avg * 1e-3) / 1e9, "layout_gbps": lb / (avg * 1e-3) / 1e9, "sweep_wall_ms": wall,
            "spmv_ms": ms_sp / max(c_sp, 1), "scatter_ms": ms_sc / max(c_sc, 1),
            "traffic": traffic_entry(workload, prec), "shape": info["apply_variant"]}


def factor_leg(H, fh) -> dict:
    """Level-0 patch inversion alone (set-up of level 0), HIP events on the level's stream."""
    import numpy as np
    import torch
    set_precision(H, fh, "f64")
    H.setup()
    H.profile(["factor"])
    H.profile_reset()
    for _ in range(3):
        H.setup(0)
    torch.cuda.synchronize()
    ms, cnt = H.profile_read("factor", 0)
    H.profile([])
    m = patch_sizes(fh.levels[0]).astype(np.float64)
    avg = ms / max(cnt, 1)
    lu = 2.0 / 3.0 * float((m ** 3).sum())
    gj = 2.0 * float((m ** 3).sum())
    return {"avg_ms": avg, "launches": cnt, "lu_flops": lu, "gj_flops": gj,
            "tflops": lu / (avg * 1e-3) / 1e12, "gj_tflops": gj / (avg * 1e-3) / 1e12}


def block_apply_leg(H, fh, prec: str, B) -> dict:
    import torch
    Xr = torch.zeros_like(B)
    for _ in range(3):
        H.relax_apply_batched(0, B, Xr, 1)
    H.profile(["patch_apply", "spmv", "scatter"])
    H.profile_reset()
    for _ in range(10):
        H.relax_apply_batched(0, B, Xr, 1)
    ms, cnt = H.profile_read("patch_apply", 0)
    ms_sp, c_sp = H.profile_read("spmv", 0)
    ms_sc, c_sc = H.profile_read("scatter", 0)
    H.profile([])
    m = patch_sizes(fh.levels[0])
    info = H.level_info(0)
    avg = ms / max(cnt, 1)
    mb = method_block_bytes(m, ES[prec], info["symmetric_storage"])
    return {"block_apply_ms": _fmt(avg), "block_apply_gbps": _fmt(mb / (avg * 1e-3) / 1e9),
            "block_apply_method_bytes": mb, "spmm_ms": _fmt(ms_sp / max(c_sp, 1)),
            "block_scatter_ms": _fmt(ms_sc / max(c_sc, 1)), "block_variant": info["block_variant"]}


def single_solve_leg(H, fh, prec: str, b, g, column: int) -> dict:
    """Set-up + FGMRES to 1e-8 of one system: split, iterations, true residual, error vs the oracle."""
    import numpy as np
    import torch
    set_precision(H, fh, prec)
    H.setup()
    x = torch.zeros_like(b)
    H.fgmres(b, x, rtol=1e-8)                       # first use: graph capture
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    H.setup()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    x.zero_()
    its, rr, conv = H.fgmres(b, x, rtol=1e-8)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    r = torch.empty_like(b)
    H.residual(0, b, x, r)
    out = {"time_to_1e-8_ms": _fmt((t3 - t1) * 1e3), "setup_ms": _fmt((t2 - t1) * 1e3),
           "solve_ms": _fmt((t3 - t2) * 1e3), "iters": its, "converged": bool(conv),
           "true_relres": _fmt(float(torch.linalg.norm(r) / torch.linalg.norm(b)))}
    if g is not None:
        out["err_vs_fp64_oracle"] = _fmt(oracle_error(x.cpu().numpy(), g, column))
        out["oracle_iters"] = next(c for c in g["columns"] if c["column"] == column)["iters"]
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--phase", default="all", choices=["all", "apply", "setup", "block", "step"],
                    help="apply: only the repeated level-0 relaxation sweeps; setup: only the relaxation set-up, "
                         "repeated; block: only the 16-system level-0 sweeps; step: only the timed steps of the "
                         "first precision of --prec (for profiler runs)")
    ap.add_argument("--prec", default="f64,f32,bf16", help="precisions of the apply / block phases")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the P3/P2 and cfg2 legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="apply phase: also run 3 plain device copies of 256 MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (multi-GPU sharding of the patch "
              "relaxation is a design note, not implemented)", file=sys.stderr)
        return 2
    precs = [p for p in args.prec.split(",") if p]
    for p in precs:
        if p not in PRECS:
            ap.error(f"unknown precision {p!r}")

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    batched = args.workload == "cfg3"
    fh, H, t_build = make_hierarchy(args.workload, forcing="bumps" if batched else "mms", nrhs=16 if batched else 1)
    nl = len(fh.levels)
    infos = [H.level_info(l) for l in range(nl)]
    print(f"# workload {args.workload}: levels n={[i['n'] for i in infos]} host build {t_build:.1f}s",
          file=sys.stderr, flush=True)
    B = torch.tensor(fh.b, device=dev)                    # (16, n) or (1, n)
    X = torch.zeros_like(B)

    if args.phase == "setup":
        H.setup()
        torch.cuda.synchronize()
        H.profile(["extract", "factor"])
        H.profile_reset()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            H.setup()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
        levels = []
        for l in range(nl):
            fms, fc = H.profile_read("factor", l)
            ems, ec = H.profile_read("extract", l)
            info = H.level_info(l)
            d = {"level": l, "n": info["n"], "factor_ms": _fmt(fms / max(fc, 1)), "extract_ms": _fmt(ems / max(ec, 1))}
            if info["npatch"]:
                m = patch_sizes(fh.levels[l]).astype(np.float64)
                d["lu_gflop"] = _fmt(2.0 / 3.0 * float((m ** 3).sum()) / 1e9)
                d["lu_tflops"] = _fmt(2.0 / 3.0 * float((m ** 3).sum()) / (fms / max(fc, 1) * 1e-3) / 1e12)
            levels.append(d)
        H.profile([])
        print(json.dumps({"phase": "setup", "workload": args.workload, "setup_ms": _fmt(wall), "levels": levels}),
              flush=True)
        H.close()
        return 0
    if args.phase == "apply":
        legs = {p: {k: _fmt(v) for k, v in apply_leg(H, fh, p, args.apply_reps, args.workload).items()} for p in precs}
        if args.calibrate_copy:
            src = torch.ones(1 << 25, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            legs["copy_bytes_each_way"] = src.numel() * 8
        print(json.dumps({"phase": "apply", "workload": args.workload, "apply": legs}), flush=True)
        H.close()
        return 0
    if args.phase == "block":
        legs = {}
        for p in precs:
            set_precision(H, fh, p)
            H.setup()
            legs[p] = block_apply_leg(H, fh, p, B)
        print(json.dumps({"phase": "block", "workload": args.workload, "block": legs}), flush=True)
        H.close()
        return 0

    # ---- the timed step: set-up + FGMRES of the whole batch, per precision
    def step():
        H.setup()
        X.zero_()
        if batched:
            return H.fgmres_batched(B, X, rtol=1e-8, restart=30, maxit=1000)
        its, rr, conv = H.fgmres(B[0], X[0], rtol=1e-8, restart=30, maxit=1000)
        return [its], [rr], conv

    g_batch = golden("cfg3_bumps") if batched else golden(args.workload)
    legs = {}
    if args.phase == "step":
        set_precision(H, fh, precs[0])
        H.setup()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = step()
        torch.cuda.synchronize()
        print(json.dumps({"phase": "step", "workload": args.workload, "prec": precs[0],
                          "ms_per_step": _fmt((time.perf_counter() - t0) * 1e3 / max(args.steps, 1)),
                          "iters": res[0]}), flush=True)
        H.close()
        return 0
    for prec in PRECS:
        set_precision(H, fh, prec)
        H.setup()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        for _ in range(args.steps):
            res = step()
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
        # split of one step
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        H.setup()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        X.zero_()
        its, rr, conv = (H.fgmres_batched(B, X, rtol=1e-8) if batched else step())
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        r = torch.empty(fh.levels[0].n, dtype=torch.float64, device=dev)
        true_rel = 0.0
        for c in range(B.shape[0]):
            H.residual(0, B[c].contiguous(), X[c].contiguous(), r)
            true_rel = max(true_rel, float(torch.linalg.norm(r) / torch.linalg.norm(B[c])))
        leg = {"ms_per_step": _fmt(ms_step), "setup_ms": _fmt((t2 - t1) * 1e3), "solve_ms": _fmt((t3 - t2) * 1e3),
               "iters_min": min(its), "iters_max": max(its), "converged": bool(conv),
               "true_relres_max": _fmt(true_rel)}
        if g_batch is not None:
            Xh = X.cpu().numpy()
            errs = {str(c["column"]): _fmt(oracle_error(Xh[c["column"]], g_batch, c["column"]))
                    for c in g_batch["columns"] if c["column"] < B.shape[0]}
            leg["err_vs_fp64_oracle"] = errs
            leg["oracle_iters"] = {str(c["column"]): c["iters"] for c in g_batch["columns"] if c["column"] < B.shape[0]}
        if batched:
            leg.update(block_apply_leg(H, fh, prec, B))
        legs[prec] = leg
    # one system at a time (FP64), for the batching gain
    if batched:
        set_precision(H, fh, "f64")
        H.setup()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for c in range(B.shape[0]):
            x1 = torch.zeros(fh.levels[0].n, dtype=torch.float64, device=dev)
            H.fgmres(B[c].contiguous(), x1, rtol=1e-8)
        torch.cuda.synchronize()
        one_by_one = (time.perf_counter() - t1) * 1e3
    # single-system legs of the metric's workload (bump column 0) and the patch-solve kernels
    single = {p: single_solve_leg(H, fh, p, B[0].contiguous(), g_batch, 0) for p in PRECS}
    ap = {p: apply_leg(H, fh, p, args.apply_reps, args.workload) for p in PRECS}
    gj = factor_leg(H, fh)
    variants = {p: ap[p]["shape"] for p in PRECS}
    lambdas = [round(H.level_info(l)["lambda_max"], 6) for l in range(nl - 1)]
    H.close()

    extra = {}
    if not args.no_extra and batched:
        print("# extra legs: cfg3 P3/P2, cfg2, cfg4 ...", file=sys.stderr, flush=True)
        for name, wl, k, job in (("cfg3_P3P2", "cfg3", 3, "cfg3_k3"), ("cfg2", "cfg2", None, "cfg2"),
                                 ("cfg4", "cfg4", None, "cfg4")):
            fx, Hx, tb = make_hierarchy(wl, k=k)
            bx = torch.tensor(fx.b[0], device=dev)
            gx = golden(job)
            e = {"workload": WORKLOADS[wl] if wl != "cfg3" else
                 "TH P3/P2 2D structured 128x128 (359427 DoFs); phMG direct P3/P2 -> P2/P1 -> 4 h-levels; MMS forcing",
                 "levels_n": [L.n for L in fx.levels], "host_build_s": round(tb, 2)}
            for p in PRECS:
                e[p] = single_solve_leg(Hx, fx, p, bx, gx, 0)
                a = apply_leg(Hx, fx, p, args.apply_reps, wl)
                e[p]["patch_apply_gbps"] = _fmt(a["gbps"])
                e[p]["patch_apply_layout_gbps"] = _fmt(a["layout_gbps"])
                e[p]["patch_apply_ms"] = _fmt(a["avg_ms"])
            e["setup_roofline_lu_tflops"] = _fmt(factor_leg(Hx, fx)["tflops"])
            Hx.close()
            extra[name] = e

    m0 = patch_sizes(fh.levels[0])
    a64 = ap["f64"]
    result = {
        "metric": METRIC,
        "value": round(a64["gbps"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(legs["f64"]["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {WORKLOADS[args.workload]}",
            "levels_n": [i["n"] for i in infos],
            "level0_patches": infos[0]["npatch"],
            "level0_sum_m2": infos[0]["sum_m2"],
            "level0_max_m": infos[0]["max_m"],
            "level0_layout": "symmetric strips" if a64["sym"] else "general",
            "rhs_per_step": int(B.shape[0]),
            "step": "relax_setup (extract + patch inversion, all levels, coarse inverse, eigenvalue estimates) + "
                    + ("FGMRES(30) to 1e-8 from x=0 of all 16 systems together" if batched else
                       "FGMRES(30) to 1e-8 from x=0"),
            "smoother": fh.opts.get("smoother", "richardson"),
            "lambda_max": lambdas,
            "apply_kernel_shape": variants,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("patch_apply_sym_kernel<double>" if a64["sym"] else "patch_apply_kernel<double>") + " (level 0)",
            "achieved": round(a64["gbps"], 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(a64["gbps"] / HBM_PEAK_GBS, 4),
            "traffic": a64["traffic"],
            "bytes_per_launch": a64["method_bytes"],
            "bytes_counted": "method: 8 sum m(m+1)/2 (symmetric patch inverses) + 20 sum m + 20 npatch",
            "layout_bytes_per_launch": a64["layout_bytes"],
            "layout_gbps": round(a64["layout_gbps"], 2),
            "avg_launch_ms": round(a64["avg_ms"], 5),
            "launches": a64["launches"],
        },
        "setup_roofline": {
            "bound": "mfma",
            "kernel": "level-0 patch inversion alone (gj_reg_kernel: Gauss-Jordan, matrix in MFMA f64 registers)",
            "achieved": round(gj["tflops"], 3),
            "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(gj["tflops"] / FP64_MFMA_PEAK_TFLOPS, 4),
            "flops_counted": "LU: 2/3 sum m^3 per launch",
            "flops_per_launch": gj["lu_flops"],
            "executed_gj_flops_per_launch": gj["gj_flops"],
            "executed_gj_tflops": round(gj["gj_tflops"], 3),
            "avg_launch_ms": round(gj["avg_ms"], 4),
            "launches": gj["launches"],
        },
        "time_to_1e-8": legs,
        "single_system_time_to_1e-8": single,
        "patch_apply_gbps": {p: round(ap[p]["gbps"], 2) for p in PRECS},
        "patch_apply_ms": {p: round(ap[p]["avg_ms"], 5) for p in PRECS},
        "sweep_level0": {p: {"wall_ms": round(ap[p]["sweep_wall_ms"], 4), "spmv_ms": round(ap[p]["spmv_ms"], 4),
                             "scatter_ms": round(ap[p]["scatter_ms"], 4)} for p in PRECS},
    }
    if batched:
        result["f64_one_system_at_a_time_solve_ms"] = _fmt(one_by_one)
    if extra:
        result["extra"] = extra
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        sw = 2 * (fh.opts.get("nu_p", 2))
        result["cpu_baseline"] = cpu_baseline(args.workload, sw, single["f64"]["iters"])
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
