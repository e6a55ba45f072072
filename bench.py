#!/usr/bin/env python3
"""Benchmark of the Vanka-star / phMG / FGMRES hot path on one MI355X.

Workload (default): Taylor-Hood P4/P3 Stokes on a Delaunay mesh of 64 seeded
points plus the corners refined 3 times (170 483 free DoFs), direct
p-coarsening to P2/P1 on the same mesh, then 3 coarser P2/P1 h-levels and a
dense coarse solve; Vanka-star patches of 64-210 DoFs; nu = 2, omega = 0.5,
FGMRES(30) to a relative residual of 1e-8.  Synthetic manufactured-solution
data stand in for the paper's cavity / step problems.

One timed step = the whole hot path on the resident hierarchy: relaxation
set-up (patch extraction + patch factorisation on every level, coarse
factorisation) followed by the FGMRES solve from x = 0.

Printed: one JSON line.  ``value`` is the achieved HBM bandwidth of the
level-0 batched patch-solve kernel in float64 (algorithmic bytes per launch
divided by its mean duration, HIP events on the library's stream), i.e. the
"Vanka patch-apply HBM GB/s" half of the metric; the "time-to-1e-8" half is
reported for float64 and for float32 / bfloat16 patch inverses ("mixed") next
to it.  ``setup_roofline`` gives the level-0 patch inversion (set-up) against
the FP64 MFMA peak, timed the same way.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "patch_apply_cfg2_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2407_07253_amd", "csrc", "patch_apply.hip")

WORKLOADS = {
    "cfg2": "TH P4/P3 2D, Delaunay 64 seeded pts + corners, 3 refinements (170483 DoFs); phMG direct "
            "P4/P3 -> P2/P1 -> 3 h-levels; Vanka-star patches 64-210 DoFs; FP64",
    "cfg1": "TH P2/P1 2D, structured 8x8 (531 DoFs); hMG 2 levels; nu=2, omega=0.5",
    "cfg4": "SV P4/P3disc 2D on the Alfeld split of a jittered 16x16 mesh refined twice (637954 DoFs)",
    "cfg3": "TH P4/P3 2D structured 128x128 (670467 DoFs); phMG direct",
}


def factor_elements(patch_ptr, sym: bool) -> int:
    """Factor words one launch of the patch solve reads: sum m^2 in the general layout; in the
    symmetric strip layout the strictly lower part of every 16-row strip plus its full 16 x 16
    diagonal block, i.e. 128 (ns - 1) ns + h m per patch (ns strips, h rows in the last one;
    padding rows not counted)."""
    import numpy as np

    m = np.diff(np.asarray(patch_ptr)).astype(np.int64)
    if not sym:
        return int((m * m).sum())
    ns = (m + 15) // 16
    h = m - (ns - 1) * 16
    return int((128 * (ns - 1) * ns + h * m).sum())


def apply_bytes(info: dict, elem_bytes: int, felems: int) -> int:
    """Algorithmic bytes of one launch of the batched patch solve on a level:
    factor words s_f * felems, patch DoF indices 4 sum m, gathered residual
    8 sum m, staged y written 8 sum m, per patch order + ptr + offset 20 B."""
    return elem_bytes * felems + 20 * info["sum_m"] + 20 * info["npatch"]


def sweep_bytes(info: dict, elem_bytes: int, felems: int) -> int:
    """Compulsory bytes of one full relaxation sweep on a level (SpMV + apply + scatter)."""
    n, nnz, sm = info["n"], info["nnz"], info["sum_m"]
    spmv = 12 * nnz + 4 * (n + 1) + 8 * n * 3           # CSR + x, b read, r written
    scatter = 8 * sm + 4 * sm + 8 * sm + 4 * (n + 1) + 16 * n   # Y, slots, weights, ptr, x r/w
    return spmv + apply_bytes(info, elem_bytes, felems) + scatter


def traffic_entry(prec: str, workload: str):
    """Counter-measured HBM bytes per launch from the committed rocprofv3 summary, if it covers this
    workload and the kernel source is unchanged."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        d = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if d.get("workload") != workload or d.get("kernel_source_sha256") != sha:
            return None
        if prec not in d.get("per_launch_bytes", {}):
            return None
        return float(d["per_launch_bytes"][prec])
    except Exception:
        return None


def cpu_baseline(workload: str, budget_s: float = 12.0):
    """The oracle's patch solve (LU forward/back substitution) on a bounded sample of level-0 patches."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.discretization import assemble_stokes
    from oracle.lu import lu_factor, lu_solve
    from oracle.patches import vanka_star_patches
    from oracle.problems import level_specs

    meshes = synth.config_mesh_hierarchy(workload)[::-1]
    specs, _ = level_specs(workload)
    mi, k, kind = specs[0]
    with threadpool_limits(limits=1):
        d = assemble_stokes(meshes[mi], k, kind)
        patches = vanka_star_patches(d)
        stride = max(1, len(patches) // 200)
        sample = patches[::stride]
        K = d.K
        facs = [lu_factor(K[S][:, S].toarray()) for S in sample]
        rng = np.random.default_rng(0)
        r = rng.standard_normal(d.n)
        nbytes = sum(8 * len(S) ** 2 + 20 * len(S) + 20 for S in sample)
        t0 = time.perf_counter()
        passes = 0
        while True:
            for S, (LU, piv) in zip(sample, facs):
                lu_solve(LU, piv, r[S])
            passes += 1
            if time.perf_counter() - t0 > budget_s or passes >= 400:
                break
        dt = time.perf_counter() - t0
    return {
        "value": nbytes * passes / dt / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle LU forward/back substitution on {len(sample)} of the {len(patches)} level-0 patches "
                  f"(every {stride}th), {passes} passes, algorithmic bytes of the LU solve 8 m^2 + 20 m + 20 per patch "
                  f"(the GPU's symmetric strip layout streams about 0.56 of the factor words), "
                  f"BLAS limited to 1 thread; host {platform.processor() or platform.machine()}, "
                  f"nproc {os.cpu_count()}",
    }


def batched_leg(nrhs: int = 16) -> dict:
    """16 right-hand sides solved together (block path): TH P4/P3 on the structured 128x128 mesh,
    seeded Gaussian-bump forcings; FP64 vs FP32 vs BF16 patch inverses (MFMA block products),
    FP64 FGMRES per column to 1e-8.  Also the same 16 systems solved one after another (FP64)."""
    import torch

    from paper_2407_07253_amd import frontend
    from paper_2407_07253_amd._lib import Hierarchy

    t0 = time.perf_counter()
    fh = frontend.build_hierarchy("cfg3", forcing="bumps", nrhs=nrhs)
    t_build = time.perf_counter() - t0
    H = Hierarchy.from_frontend(fh)
    nl = len(fh.levels)
    n0 = fh.levels[0].n
    B = torch.tensor(fh.b, device="cuda")
    out = {"workload": "cfg3: " + WORKLOADS["cfg3"] + f"; {nrhs} seeded Gaussian-bump right-hand sides",
           "levels_n": [L.n for L in fh.levels], "host_build_s": round(t_build, 2)}
    info0 = H.level_info(0)
    for prec in ("f64", "f32", "bf16"):
        for l in range(nl - 1):
            H.set_precision(l, prec)
        H.setup()
        X = torch.zeros_like(B)
        H.fgmres_batched(B, X, rtol=1e-8)                  # first use: block autotune + graph capture
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        H.setup()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        X.zero_()
        its, rr, conv = H.fgmres_batched(B, X, rtol=1e-8)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        r = torch.empty(n0, dtype=torch.float64, device="cuda")
        true_rel = 0.0
        for c in range(nrhs):
            H.residual(0, B[c].contiguous(), X[c].contiguous(), r)
            true_rel = max(true_rel, float(torch.linalg.norm(r) / torch.linalg.norm(B[c])))
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
        eb = {"f64": 8, "f32": 4, "bf16": 2}[prec]
        # the block path streams the general layout (a general copy on symmetric levels)
        fel = factor_elements(fh.levels[0].patch_ptr, False)
        # factor words once for all columns + per slot: index 4 B, gathered row and staged row 2 x 16 x 8 B
        byt = eb * fel + info0["sum_m"] * (4 + 2 * 8 * 16) + 20 * info0["npatch"]
        avg = ms / max(cnt, 1)
        out[prec] = {"setup_ms": _fmt((t2 - t1) * 1e3), "solve_ms": _fmt((t3 - t2) * 1e3),
                     "time_to_1e-8_ms": _fmt((t3 - t1) * 1e3), "iters_min": min(its), "iters_max": max(its),
                     "converged": bool(conv), "true_relres_max": _fmt(true_rel),
                     "block_apply_ms": _fmt(avg), "block_apply_gbps": _fmt(byt / (avg * 1e-3) / 1e9),
                     "block_apply_bytes": byt, "spmm_ms": _fmt(ms_sp / max(c_sp, 1)),
                     "block_scatter_ms": _fmt(ms_sc / max(c_sc, 1)),
                     "block_variant": H.level_info(0)["block_variant"]}
    for l in range(nl - 1):
        H.set_precision(l, "f64")
    H.setup()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for c in range(nrhs):
        x1 = torch.zeros(n0, dtype=torch.float64, device="cuda")
        H.fgmres(B[c].contiguous(), x1, rtol=1e-8)
    torch.cuda.synchronize()
    out["f64_one_by_one_solve_ms"] = _fmt((time.perf_counter() - t1) * 1e3)
    H.close()
    return out


def _fmt(v):
    return float(f"{v:.6g}") if isinstance(v, float) else v


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--phase", default="all", choices=["all", "apply", "setup"],
                    help="apply: only the repeated level-0 relaxation sweeps; setup: only the relaxation "
                         "set-up, repeated (both for counter runs)")
    ap.add_argument("--mixed", default="f32,bf16",
                    help="comma-separated reduced precisions of the patch inverses to time next to f64 ('none': skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 16-right-hand-side batched leg (TH P4/P3 on the structured 128x128 mesh)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="apply phase: also run 3 plain device copies of 256 MiB (counter calibration)")
    args = ap.parse_args()

    mixed = [] if args.mixed == "none" else [p for p in args.mixed.split(",") if p]
    for p in mixed:
        if p not in ("f32", "bf16"):
            ap.error(f"unknown precision {p!r} in --mixed")
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (multi-GPU sharding of the patch "
              "relaxation is a design note, not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2407_07253_amd import frontend
    from paper_2407_07253_amd._lib import Hierarchy

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_build = time.perf_counter()
    fh = frontend.build_hierarchy(args.workload)
    t_build = time.perf_counter() - t_build
    H = Hierarchy.from_frontend(fh)
    nl = len(fh.levels)
    infos = [H.level_info(l) for l in range(nl)]
    b = torch.tensor(fh.b[0], device=dev)
    x = torch.zeros_like(b)
    print(f"# workload {args.workload}: levels n={[i['n'] for i in infos]} host build {t_build:.1f}s", file=sys.stderr,
          flush=True)

    def step():
        H.setup()
        x.zero_()
        return H.fgmres(b, x, rtol=1e-8, restart=30, maxit=1000)

    def timed_legs(prec: str):
        for l in range(nl - 1):
            H.set_precision(l, prec)
        H.setup()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = None
        for _ in range(args.steps):
            its = step()
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
        # split of one step: setup vs solve
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        H.setup()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x.zero_()
        its2 = H.fgmres(b, x, rtol=1e-8)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        r = torch.empty_like(b)
        H.residual(0, b, x, r)
        relres = float(torch.linalg.norm(r) / torch.linalg.norm(b))
        return dict(ms_per_step=ms_step, setup_ms=(t2 - t1) * 1e3, solve_ms=(t3 - t2) * 1e3, iters=its2[0],
                    converged=bool(its2[2]), true_relres=relres)

    def apply_leg(prec: str):
        for l in range(nl - 1):
            H.set_precision(l, prec)
        H.setup()
        xs = torch.zeros_like(b)
        for _ in range(3):
            H.relax_apply(0, b, xs, 1)
        H.profile(["patch_apply", "spmv", "scatter"])
        H.profile_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.apply_reps):
            H.relax_apply(0, b, xs, 1)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / args.apply_reps
        ms, cnt = H.profile_read("patch_apply", 0)
        ms_spmv, c_spmv = H.profile_read("spmv", 0)
        ms_sc, c_sc = H.profile_read("scatter", 0)
        H.profile([])
        eb = {"f64": 8, "f32": 4, "bf16": 2}[prec]
        sym = H.level_info(0)["symmetric_storage"]
        fel = factor_elements(fh.levels[0].patch_ptr, sym)
        per = apply_bytes(infos[0], eb, fel)
        avg = ms / max(cnt, 1)
        return dict(avg_ms=avg, launches=cnt, bytes_per_launch=per, gbps=per / (avg * 1e-3) / 1e9,
                    sym=sym, factor_elements=fel,
                    sweep_wall_ms=wall, sweep_bytes=sweep_bytes(infos[0], eb, fel),
                    sweep_gbps=sweep_bytes(infos[0], eb, fel) / (wall * 1e-3) / 1e9,
                    spmv_ms=ms_spmv / max(c_spmv, 1), scatter_ms=ms_sc / max(c_sc, 1))

    if args.phase == "setup":
        # patch extraction + Gauss-Jordan inversion on every level, and the coarse inverse;
        # algorithmic flops of inverting an m x m patch: 2 m^3 (LU 2m^3/3 + the rest of the inverse)
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
                flops = 2.0 * float(np.sum(np.diff(fh.levels[l].patch_ptr).astype(np.float64) ** 3))
                d["factor_gflop"] = _fmt(flops / 1e9)
                d["factor_tflops"] = _fmt(flops / (fms / max(fc, 1) * 1e-3) / 1e12)
            levels.append(d)
        H.profile([])
        print(json.dumps({"phase": "setup", "workload": args.workload, "setup_ms": _fmt(wall), "levels": levels}),
              flush=True)
        H.close()
        return 0

    if args.phase == "apply":
        legs = {p: apply_leg(p) for p in ["f64"] + mixed}
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

    def factor_leg():
        # level-0 patch inversion alone (set-up of level 0 only), HIP events on the level's
        # stream; algorithmic flops of inverting an m x m patch: 2 m^3
        H.profile(["factor"])
        H.profile_reset()
        for _ in range(3):
            H.setup(0)
        torch.cuda.synchronize()
        ms, cnt = H.profile_read("factor", 0)
        H.profile([])
        flops = 2.0 * float(np.sum(np.diff(fh.levels[0].patch_ptr).astype(np.float64) ** 3))
        avg = ms / max(cnt, 1)
        return dict(avg_ms=avg, launches=cnt, flops=flops, tflops=flops / (avg * 1e-3) / 1e12)

    f64 = timed_legs("f64")
    ap64 = apply_leg("f64")
    gj64 = factor_leg()
    variants = {"f64": [H.level_info(l)["apply_variant"] for l in range(nl - 1)]}
    lambdas = [round(H.level_info(l)["lambda_max"], 6) for l in range(nl - 1)]
    out_mixed, ap_mixed = {}, {}
    for prec in mixed:
        out_mixed[prec] = timed_legs(prec)
        ap_mixed[prec] = apply_leg(prec)
        variants[prec] = [H.level_info(l)["apply_variant"] for l in range(nl - 1)]
    H.close()

    traffic = traffic_entry("f64", args.workload)
    result = {
        "metric": METRIC,
        "value": round(ap64["gbps"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 4),
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
            "level0_layout": "symmetric strips" if ap64["sym"] else "general",
            "level0_factor_elements": ap64["factor_elements"],
            "level0_max_m": infos[0]["max_m"],
            "step": "relax_setup (extract + patch inversion, all levels) + FGMRES(30) to 1e-8 from x=0",
            "smoother": fh.opts.get("smoother", "richardson"),
            "lambda_max": lambdas,
            "apply_kernel_shape": variants,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("patch_apply_sym_kernel<double>" if ap64["sym"] else "patch_apply_kernel<double>")
                      + " (level 0)",
            "achieved": round(ap64["gbps"], 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(ap64["gbps"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": ap64["bytes_per_launch"],
            "avg_launch_ms": round(ap64["avg_ms"], 5),
            "launches": ap64["launches"],
        },
        "setup_roofline": {
            "bound": "mfma",
            "kernel": "gj_kernel (level-0 patch inversion alone, FP64 MFMA 16x16x4 trailing updates)",
            "achieved": round(gj64["tflops"], 3),
            "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(gj64["tflops"] / FP64_MFMA_PEAK_TFLOPS, 4),
            "flops_per_launch": gj64["flops"],
            "avg_launch_ms": round(gj64["avg_ms"], 4),
            "launches": gj64["launches"],
        },
        "time_to_1e-8": {"f64": {k: _fmt(v) for k, v in f64.items()}},
        "sweep_level0": {"f64": {"wall_ms": round(ap64["sweep_wall_ms"], 4), "gbps": round(ap64["sweep_gbps"], 1),
                                 "spmv_ms": round(ap64["spmv_ms"], 4), "scatter_ms": round(ap64["scatter_ms"], 4)}},
    }
    result["patch_apply_gbps"] = {"f64": round(ap64["gbps"], 2)}
    for prec in mixed:
        result["time_to_1e-8"][prec] = {k: _fmt(v) for k, v in out_mixed[prec].items()}
        result["patch_apply_gbps"][prec] = round(ap_mixed[prec]["gbps"], 2)
        result["sweep_level0"][prec] = {"wall_ms": round(ap_mixed[prec]["sweep_wall_ms"], 4),
                                        "gbps": round(ap_mixed[prec]["sweep_gbps"], 1)}
    if not args.no_batched:
        print("# batched leg (cfg3, 16 right-hand sides) ...", file=sys.stderr, flush=True)
        result["batched_16rhs"] = batched_leg()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.workload if args.workload != "cfg3" else "cfg2")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
