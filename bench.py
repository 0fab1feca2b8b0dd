#!/usr/bin/env python3
"""Benchmark of the layered-media linearized Poisson-Boltzmann FMM on one MI355X.

Workload (default): three layers, interfaces z = 0 and -1.2, eps = (1, 2, 4),
lambda = (1.2, 1.5, 2.0), 1e6 charges per layer (3e6 total) uniform in unit
cubes, q ~ U[-1, 1], p = 10, leaf cap 50.  A step is one lpb_evaluate of the
whole method (3 free-space and 16 reaction FMMs, component sum) on charges
already resident in HBM; tree and operators are built before the timed region.

value = charges/sec of the mixed-precision form (FP32 bulk, FP64 Bessel and
operator generation).  The plain FP64 GPU path is timed beside it
(fp64_value) and the mixed result's per-layer relative l2 error against it is
reported (rel_err_vs_fp64, gate 1e-6).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# peaks (MI355X, published): HBM 8 TB/s; vector FP32 157.3 TFLOP/s; vector FP64 78.6 TFLOP/s
PEAK_FP32 = 157.3
PEAK_FP64 = 78.6
# algorithmic flops per unit of work of each stage
FLOPS_PER_P2P_PAIR = 20.0


def err2_per_layer(a, b, layer):
    return [float(np.linalg.norm(a[layer == l] - b[layer == l]) / np.linalg.norm(b[layer == l])) for l in range(3)]


def time_context(lpb, torch, prob, p, leaf_cap, precision, steps, warmup):
    dev = torch.device("cuda:0")
    t = {k: torch.tensor(getattr(prob, k), dtype=torch.float64, device=dev) for k in ("x", "y", "z", "q")}
    ctx = lpb.Context(p=p, leaf_cap=leaf_cap, precision=precision, timing=1,
                      stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_layers(prob.eps, prob.lam, prob.d)
    t0 = time.perf_counter()
    ctx.build_tree(t["x"], t["y"], t["z"])
    t_build = time.perf_counter() - t0
    phi = torch.empty_like(t["q"])
    for _ in range(max(1, warmup)):          # the first call also generates the operators
        ctx.evaluate(t["q"], phi)
    torch.cuda.synchronize()
    st0 = ctx.stats()
    stage = {k: 0.0 for k in st0["t_stage_ms"]}
    evals = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.evaluate(t["q"], phi)
        s = ctx.stats()
        evals.append(s["t_eval_ms"])
        for k, v in s["t_stage_ms"].items():
            stage[k] += v / steps
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    out = phi.cpu().numpy()
    stats = ctx.stats()
    ctx.close()
    return {"wall_s": wall, "eval_ms": float(np.mean(evals)), "stage_ms": stage, "stats": stats,
            "t_build_s": t_build, "phi": out}


def cpu_baseline(per_layer, p, leaf_cap):
    """The oracle FMM (plain C, FP64, all host threads) on a bounded sample."""
    import oracle
    from paper_2002_01334_amd import inputs

    prob = inputs.three_layer(per_layer, seed=0)
    ly = oracle.Layers(prob.eps, prob.lam, prob.d)
    # the host share of one GPU is at most 16 threads, whatever the machine reports
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    oracle.fmm(ly, prob.x, prob.y, prob.z, prob.q, p, leaf_cap=leaf_cap, nthreads=cores)
    dt = time.perf_counter() - t0
    return {"value": prob.n / dt, "unit": "charges/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle CPU FMM (FP64, OpenMP) on {prob.n} charges ({per_layer}/layer, same recipe, p={p}, "
                      f"leaf cap {leaf_cap}); {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--per-layer", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--leaf-cap", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-sample-per-layer", type=int, default=200_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path would shard by "
              "assigning independent FMMs to GPUs, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2002_01334_amd import inputs, lpb

    lpb.load()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n * 8} bytes read, {n * 8} bytes written", file=sys.stderr, flush=True)
        del src, dst
    prob = inputs.three_layer(args.per_layer, seed=0)
    print(f"[bench] workload: 3 layers, {prob.n} charges, p={args.p}", file=sys.stderr, flush=True)
    mixed = time_context(lpb, torch, prob, args.p, args.leaf_cap, lpb.LPB_MIXED, args.steps, args.warmup)
    print(f"[bench] mixed: {mixed['eval_ms']:.2f} ms/eval, stages {mixed['stage_ms']}", file=sys.stderr, flush=True)
    fp64 = time_context(lpb, torch, prob, args.p, args.leaf_cap, lpb.LPB_FP64, args.fp64_steps, 1)
    print(f"[bench] fp64: {fp64['eval_ms']:.2f} ms/eval, stages {fp64['stage_ms']}", file=sys.stderr, flush=True)
    rel = err2_per_layer(mixed["phi"], fp64["phi"], prob.layer)

    st = mixed["stats"]
    K = (args.p + 1) ** 2
    stage = mixed["stage_ms"]
    # dominant kernel and its algorithmic work per launch
    work = {
        "m2l_tile": (2.0 * K * K * st["n_m2l_tile_pairs"], "mfma", "2K^2 flops per V-list pair (real-form dense product)"),
        "p2p_free": (FLOPS_PER_P2P_PAIR * (st["n_p2p_pairs"] - st["n_react_p2p_pairs"]), "alu",
                     "20 flops per charge pair"),
    }
    dom = max(work, key=lambda k: stage.get(k, 0.0))
    flops, bound, per = work[dom]
    achieved = flops / (stage[dom] * 1e-3) / 1e12
    roof = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32, "traffic": None,
            "work": f"{flops:.4g} algorithmic flops per launch ({per})"}
    fp64_roof = {"kernel": "m2l_tile", "achieved": 2.0 * K * K * st["n_m2l_tile_pairs"] / (fp64["stage_ms"]["m2l_tile"] * 1e-3) / 1e12,
                 "peak": PEAK_FP64, "unit": "TFLOP/s"}
    fp64_roof["frac"] = fp64_roof["achieved"] / PEAK_FP64

    ms = mixed["eval_ms"]
    line = {
        "metric": "charges/sec (3-layer potential, p=10): mixed-batched vs FP64 at <=1e-6 rel err",
        "value": prob.n / (ms * 1e-3),
        "unit": "charges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"3-layer medium eps=(1,2,4) lambda=(1.2,1.5,2.0) d=(0,-1.2), "
                               f"{args.per_layer}/layer uniform unit cubes, q~U[-1,1], seed 0",
                   "charges": prob.n, "p": args.p, "leaf_cap": args.leaf_cap, "precision": "mixed"},
        "fp64_value": prob.n / (fp64["eval_ms"] * 1e-3),
        "fp64_ms_per_step": fp64["eval_ms"],
        "speedup_vs_fp64": fp64["eval_ms"] / ms,
        "rel_err_vs_fp64": max(rel),
        "rel_err_vs_fp64_per_layer": rel,
        "wall_ms_per_step": mixed["wall_s"] * 1e3,
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "fp64_stage_ms": {k: round(v, 4) for k, v in fp64["stage_ms"].items()},
        "setup": {"tree_build_s": mixed["t_build_s"], "opgen_ms": st["t_opgen_ms"], "n_m2l_pairs": st["n_m2l_pairs"],
                  "n_p2p_pairs": st["n_p2p_pairs"], "n_operators": st["n_operators"], "max_depth": st["max_depth"]},
        "roofline": roof,
        "fp64_roofline": fp64_roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_per_layer, args.p, args.leaf_cap)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
