#!/usr/bin/env python3
"""Benchmark: Gamma v = F solves per second at 1M cells, relres 1e-8, on one GPU.

One step is one pass of the whole hot path over the 1M-cell workload with all
inputs already resident in HBM: collide -> assemble_gamma -> build_tree ->
factor_tree -> pcg_solve (tree preconditioner, FP64, relres 1e-8).  The
workload: jittered FCC ball of 1,000,000 spheres (nearest-neighbour spacing
1.9, jitter N(0, 0.05^2)), radii U[0.95, 1.05], forces N(0, 1), seed 0.

Prints ONE JSON line.  Besides the headline value it carries:
  roofline      the CG's block-CSR product (the dominant kernel): algorithmic
                bytes per launch / its average launch time, measured with HIP
                events on the library's stream inside the timed region;
  cpu_baseline  the FP64 CPU oracle timed on this host's cores on a bounded
                sample of the same workload (setup + a fixed number of CG
                iterations, extrapolated to the GPU's iteration count);
  extra         phase times, block-Jacobi PCG and FP32-inner refinement on the
                same system (iterations and solve time), for comparison.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def spmv_bytes(n: int, nnzb: int, val_bytes: int = 48) -> int:
    """Algorithmic bytes of one block-CSR product y = Gamma x as the library
    stores Gamma: every block's 6 distinct entries (the blocks are symmetric,
    48 B in FP64) and its column index once, the row pointers once, x once,
    y once."""
    return nnzb * (val_bytes + 4) + 4 * (n + 1) + 24 * n + 24 * n


def cpu_baseline(c, gpu_iters: int, sample_iters: int = 10):
    """Oracle on this host: full setup at the full size, then `sample_iters` CG
    iterations; the solve time is extrapolated to the GPU's iteration count."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    g = O.collide(c["pos"], c["radius"])
    A = O.assemble(g)
    t = O.build_tree(g)
    f = O.tree_factor(g, t)
    t1 = time.perf_counter()
    O.pcg(A, c["force"], "tree", f, fixed_iters=sample_iters)
    t2 = time.perf_counter()
    per_iter = (t2 - t1) / sample_iters
    est = (t1 - t0) + per_iter * gpu_iters
    return {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"1M-cell workload: collide+assemble+Prim+root+TreeLDLT in full ({t1 - t0:.1f} s) "
                      f"plus {sample_iters} tree-PCG iterations ({t2 - t1:.1f} s), "
                      f"extrapolated to {gpu_iters} iterations; single-threaded C, -O2",
            "setup_s": t1 - t0, "per_iter_s": per_iter}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--schedule", default="contract", choices=["contract", "level"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--kernel-only", choices=["spmv"], default=None,
                    help="build the system once, then run only the named kernel (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2410_04512_amd as P
    from workloads import sphere_cluster

    torch.cuda.set_device(0)
    c = sphere_cluster(args.n, 0)
    dev = lambda a: torch.as_tensor(a).to("cuda")  # noqa: E731
    pos, R, F = dev(c["pos"]), dev(c["radius"]), dev(c["force"])
    ctx = P.Context()
    g, A, T, M = P.Graph(ctx), P.Bsr(ctx), P.Tree(ctx), P.Prec(ctx)
    v = torch.zeros_like(F)
    info = {}

    def step():
        nonlocal info
        ctx.collide(pos, R, 32, g)
        ctx.assemble_gamma(g, 1.0, 0.1, 1e-3, A)
        ctx.build_tree(g, T)
        ctx.factor_tree(g, T, 1.0, 0.1, 1e-3, args.schedule, M)
        _, info = ctx.pcg_solve(A, M, F, v, rtol=1e-8)

    if args.kernel_only == "spmv":
        # counter-run mode: a plain copy of known size (calibrates FETCH_SIZE /
        # WRITE_SIZE), then the block-CSR product alone, 20 times
        ctx.collide(pos, R, 32, g)
        ctx.assemble_gamma(g, 1.0, 0.1, 1e-3, A)
        n, _ = g.size()
        _, nnzb = A.size()
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 512 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        x = torch.ones_like(F)
        y = torch.empty_like(F)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            ctx.spmv(A, x, y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        print(json.dumps({"kernel": "k_spmv_sym", "copy_bytes": 2 * src.numel() * 8, "api_call_avg_ms": ms,
                          "bytes_per_launch": spmv_bytes(n, nnzb),
                          "note": "api_call_avg_ms includes the two permutations of sgp_spmv; the kernel alone is in the trace"}), flush=True)
        ctx.close()
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_timing(True)
    phase = {k: 0.0 for k in ("collide", "assemble", "build_tree", "factor", "solve")}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        for k, val in ctx.phase_times().items():
            phase[k] += val
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    spmv_ms, spmv_launches = ctx.kernel_stats()
    ctx.kernel_timing(False)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    n, m = g.size()
    _, nnzb = A.size()
    nt, n_roots, max_depth = T.size()
    avg_spmv_ms = spmv_ms / max(spmv_launches, 1)
    bytes_spmv = spmv_bytes(n, nnzb)
    achieved = bytes_spmv / (avg_spmv_ms * 1e-3) / 1e9
    out = {
        "metric": "Gamma v=F solves/s @1M cells, relres 1e-8 (tree-PCG, FP64)",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"jittered FCC ball, {n} spheres, seed 0; step = collide+assemble+tree+factor+tree-PCG",
                   "n_cells": n, "contacts": m, "nnzb": nnzb, "tree_depth": max_depth, "trees": n_roots,
                   "schedule": args.schedule, "elim_steps": M.steps(), "cg_iters": info.get("iters"),
                   "relres_true": info.get("relres_true")},
        "roofline": {"bound": "hbm", "kernel": "k_spmv (block-CSR product in CG)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bytes_spmv, "avg_launch_ms": avg_spmv_ms,
                     "launches": spmv_launches},
        "phase_ms": {k: v_ / args.steps for k, v_ in phase.items()},
    }
    if not args.no_extra:
        ex = {}
        MJ = ctx.make_jacobi(A)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, ij = ctx.pcg_solve(A, MJ, F, torch.zeros_like(F), rtol=1e-8)
        torch.cuda.synchronize()
        ex["jacobi_pcg"] = {"iters": ij["iters"], "solve_ms": 1e3 * (time.perf_counter() - ta)}
        ta = time.perf_counter()
        _, it = ctx.pcg_solve(A, M, F, torch.zeros_like(F), rtol=1e-8)
        torch.cuda.synchronize()
        ex["tree_pcg"] = {"iters": it["iters"], "solve_ms": 1e3 * (time.perf_counter() - ta)}
        ta = time.perf_counter()
        _, ii = ctx.pcg_solve(A, M, F, torch.zeros_like(F), rtol=1e-8, precision="f32ir", inner_rtol=1e-4)
        torch.cuda.synchronize()
        ex["tree_pcg_f32ir"] = {"iters": ii["iters"], "outer": ii["outer_iters"], "relres": ii["relres_rec"],
                                "solve_ms": 1e3 * (time.perf_counter() - ta)}
        out["extra"] = ex
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, int(info.get("iters") or 170))
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
