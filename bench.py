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

Other workloads (--workload): clustered (1e5 charges per layer, half of them
Gaussian with sigma 0.1 about the cube centre; default p = 6), interface (1e5
per layer, half in tight clusters next to the interfaces; default p = 6), batch (256
independent systems of uneven sizes and random media evaluated by one batched
call; default p = 8) and paper (the paper's own test problem: eps = (1, 8.6,
20.5), lambda = (1.2, 0.5, 2.1), charges uniform in the three P_4-shaped
bodies, --charges total, default 2,861,288, the largest count of its timing
table; default p = 5, the table's order; the table's 36-core CPU time for the
same count is quoted as context).  --p overrides the order (e.g. 15 on the
default workload); --adaptive evaluates on adaptive trees (W- and X-lists).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# peaks (MI355X, published): HBM 8 TB/s; matrix cores FP32 157.3 TFLOP/s, FP64 78.6 TFLOP/s.
# Vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s for FP32 without
# packed instructions (the library is built with packed FP32 disabled; the published 157.3 counts them)
# and for FP64.
PEAK_FP32 = 157.3
PEAK_FP64 = 78.6
PEAK_VALU = 78.6
PEAK_HBM_GBS = 8000.0
# algorithmic work per unit of each stage: 20 flops per near-field charge pair (distance, rsqrt, exp2,
# product, sum); about 8K flops per charge and expansion in P2M and L2P (Bessel and solid-harmonic
# recurrences and the K coefficients); 2K^2 flops per real-form dense K x K product
FLOPS_PER_P2P_PAIR = 20.0
# the paper's timing table (Table 1), 36 cores: N -> (free-space s, reaction s)
PAPER_TABLE1 = {618_256: (2.042, 1.639), 1_128_556: (4.308, 4.459), 1_862_568: (14.94, 6.104),
                2_861_288: (15.21, 7.673)}


def err2_per_layer(a, b, layer):
    return [float(np.linalg.norm(a[layer == l] - b[layer == l]) / np.linalg.norm(b[layer == l])) for l in range(3)]


def _time_evals(ctx, torch, run, steps, warmup):
    """warmup untimed calls (the first also generates the operators), then
    `steps` timed calls; per-call and per-stage times from the library's HIP
    events on its stream, wall time around the whole loop."""
    for _ in range(max(1, warmup)):
        run()
    torch.cuda.synchronize()
    stage = {k: 0.0 for k in ctx.stats()["t_stage_ms"]}
    evals = []
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
        s = ctx.stats()
        evals.append(s["t_eval_ms"])
        for k, v in s["t_stage_ms"].items():
            stage[k] += v / steps
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return float(np.mean(evals)), stage, wall


def _run_contexts(lpb, torch, setup, run_one, p, leaf_cap, precision, steps, warmup, stage_steps, adaptive=0):
    """The timed evaluations use the captured passes (graph = 1, autotuned
    schedules, no per-stage events); a second context launches the passes one
    by one with events between stages for the stage breakdown."""
    stream = torch.cuda.current_stream().cuda_stream
    ctx = lpb.Context(p=p, leaf_cap=leaf_cap, precision=precision, timing=0, graph=1, autotune=1, stream=stream,
                      adaptive=adaptive)
    t_build = setup(ctx)
    ms, _, wall = _time_evals(ctx, torch, lambda: run_one(ctx), steps, warmup)
    out = run_one(ctx)
    stats = ctx.stats()
    ctx.close()
    ctx = lpb.Context(p=p, leaf_cap=leaf_cap, precision=precision, timing=1, graph=0, autotune=0, stream=stream,
                      adaptive=adaptive)
    setup(ctx)
    ms_eager, stage, _ = _time_evals(ctx, torch, lambda: run_one(ctx), stage_steps, 1)
    ctx.close()
    return {"wall_s": wall, "eval_ms": ms, "eval_ms_eager": ms_eager, "stage_ms": stage, "stats": stats,
            "t_build_s": t_build, "phi": out}


def time_context(lpb, torch, prob, p, leaf_cap, precision, steps, warmup, stage_steps=3, adaptive=0):
    dev = torch.device("cuda:0")
    t = {k: torch.tensor(getattr(prob, k), dtype=torch.float64, device=dev) for k in ("x", "y", "z", "q")}
    phi = torch.empty_like(t["q"])

    def setup(ctx):
        ctx.set_layers(prob.eps, prob.lam, prob.d)
        t0 = time.perf_counter()
        ctx.build_tree(t["x"], t["y"], t["z"])
        return time.perf_counter() - t0

    def run_one(ctx):
        ctx.evaluate(t["q"], phi)
        return phi

    r = _run_contexts(lpb, torch, setup, run_one, p, leaf_cap, precision, steps, warmup, stage_steps, adaptive)
    r["phi"] = r["phi"].cpu().numpy()
    return r


def time_batch(lpb, torch, probs, p, leaf_cap, precision, steps, warmup, stage_steps=2):
    dev = torch.device("cuda:0")
    ts = [{k: torch.tensor(getattr(pr, k), dtype=torch.float64, device=dev) for k in ("x", "y", "z", "q")}
          for pr in probs]
    outs = [torch.empty_like(t["q"]) for t in ts]
    qs = [t["q"] for t in ts]

    def setup(ctx):
        ctx.set_systems([pr.eps for pr in probs], [pr.lam for pr in probs], [pr.d for pr in probs])
        t0 = time.perf_counter()
        ctx.build_trees([t["x"] for t in ts], [t["y"] for t in ts], [t["z"] for t in ts])
        return time.perf_counter() - t0

    def run_one(ctx):
        ctx.evaluate_batch(qs, outs)
        return outs

    r = _run_contexts(lpb, torch, setup, run_one, p, leaf_cap, precision, steps, warmup, stage_steps)
    r["phi"] = [o.cpu().numpy() for o in r["phi"]]
    return r


def shrink(prob, k):
    """Every k-th charge of a problem (same recipe, 1/k of the density)."""
    import dataclasses

    return dataclasses.replace(prob, **{f: getattr(prob, f)[::k].copy() for f in ("x", "y", "z", "q", "layer")})


def cpu_baseline(probs, p, leaf_cap, what, cores=None, adaptive=False):
    """The oracle FMM (plain C, FP64, OpenMP) on a bounded sample of the
    workload.  Its cost is linear in the number of charges at a fixed leaf
    occupancy (the tree deepens with N), so charges/s carries over to the
    full-size workload of the same recipe."""
    import oracle

    # the host share of one GPU is at most 16 threads, whatever the machine reports
    if cores is None:
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
    n = 0
    t0 = time.perf_counter()
    for prob in probs:
        ly = oracle.Layers(prob.eps, prob.lam, prob.d)
        oracle.fmm(ly, prob.x, prob.y, prob.z, prob.q, p, leaf_cap=leaf_cap, nthreads=cores, adaptive=adaptive)
        n += prob.n
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "charges/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle CPU FMM (FP64, OpenMP) on {what}: {n} charges, p={p}, leaf cap {leaf_cap}; {dt:.1f} s"}


def kernel_sources_sha():
    """sha256 over the evaluation kernels' sources (csrc/*.hip and *.h, sorted)."""
    d = os.path.join(ROOT, "paper_2002_01334_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def kernel_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if the kernels' sources are unchanged since it was taken."""
    prof = os.path.join(ROOT, "profiles", "hbm_traffic_3layer_3e6_p10.md")
    try:
        text = open(prof).read()
        blk = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blk.get("source_sha256") != kernel_sources_sha():
        return None
    for k in blk.get("kernels", []):
        if k["stage"] == kernel:
            return k["bytes_per_launch"]
    return None


def stage_work(st, p, precision_mixed=True):
    """Algorithmic work of every stage of one evaluation: (flops, bytes,
    flop peak in TFLOP/s, unit "mfma" or "alu", description).  The tiled M2L counts one product per
    (target box, reflection orbit) in its orbit form (mixed precision, 5 <= p
    <= 15), one per V-list pair otherwise."""
    K = (p + 1) ** 2
    fb = 4 if precision_mixed else 8
    mfma = PEAK_FP32 if precision_mixed else PEAK_FP64
    orbit_form = precision_mixed and 5 <= p <= 15
    tile_units = 56 * 64 * st["n_m2l_tiles"] if orbit_form else st["n_m2l_tile_pairs"]
    list_pairs = st["n_m2l_pairs"] - st["n_m2l_tile_pairs"]
    return {
        "m2l_tile": (2.0 * K * K * tile_units, 0.0, mfma, "mfma",
                     "2K^2 flops per (target box, reflection orbit) product" if orbit_form
                     else "2K^2 flops per V-list pair (real-form dense product)"),
        "m2l_list": (2.0 * K * K * list_pairs, float(st["n_m2l_list_ops"]) * K * K * fb, mfma, "mfma",
                     "2K^2 flops per untiled V-list pair; each distinct operator (K^2 reals) read once"),
        "p2p_free": (FLOPS_PER_P2P_PAIR * (st["n_p2p_pairs"] - st["n_react_p2p_pairs"]), 0.0, PEAK_VALU, "alu",
                     "20 flops per near-field charge pair"),
        "p2m": (8.0 * K * st["n_p2m_points"], 0.0, PEAK_VALU, "alu", "8K flops per charge expansion"),
        "l2p": (8.0 * K * st["n_l2p_points"], 0.0, PEAK_VALU, "alu", "8K flops per charge evaluation"),
        "m2m": (2.0 * K * K * st["n_m2m_links"], 0.0, mfma, "mfma", "2K^2 flops per child link"),
        "l2l": (2.0 * K * K * st["n_l2l_links"], 0.0, mfma, "mfma", "2K^2 flops per child link"),
    }


def roofline(st, stage_ms, p, precision_mixed=True, traffic_ok=False):
    """Per-stage roofline fractions and the object of the stage that takes
    the most time: the ideal time of a stage is the larger of its flops at the
    flop peak of its unit and its bytes at the HBM peak; frac = ideal /
    measured; `achieved` is given in the unit of the binding resource."""
    work = stage_work(st, p, precision_mixed)
    per = {}
    for k, (fl, by, peak, unit, what) in work.items():
        t = stage_ms.get(k, 0.0)
        if t <= 0.0 or (fl == 0.0 and by == 0.0):
            continue
        t_fl = fl / (peak * 1e12)
        t_by = by / (PEAK_HBM_GBS * 1e9)
        per[k] = {"ms": t, "frac": max(t_fl, t_by) / (t * 1e-3), "bound": "hbm" if t_by > t_fl else unit}
    dom = max(per, key=lambda k: per[k]["ms"])
    fl, by, peak, _, what = work[dom]
    t = stage_ms[dom] * 1e-3
    if per[dom]["bound"] == "hbm":
        obj = {"kernel": dom, "bound": "hbm", "achieved": by / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        obj = {"kernel": dom, "bound": per[dom]["bound"], "achieved": fl / t / 1e12, "peak": peak, "unit": "TFLOP/s"}
    obj["frac"] = obj["achieved"] / obj["peak"]
    obj["traffic"] = kernel_traffic(dom) if traffic_ok else None
    obj["work"] = f"{fl:.4g} algorithmic flops" + (f" and {by:.4g} bytes" if by else "") + f" per launch ({what})"
    obj["stages"] = {k: {"frac": round(v["frac"], 4), "bound": v["bound"]} for k, v in per.items()}
    return obj


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("uniform", "clustered", "interface", "batch", "paper"), default="uniform",
                    help="uniform: 1e6 charges per layer in unit cubes (default); clustered: 1e5 per layer, half "
                         "Gaussian (sigma 0.1); batch: 256 independent systems of uneven sizes; paper: the paper's "
                         "test problem (P_4-shaped bodies, its media)")
    ap.add_argument("--per-layer", type=int, default=None)
    ap.add_argument("--charges", type=int, default=2_861_288, help="total charges of the paper workload")
    ap.add_argument("--systems", type=int, default=256)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--leaf-cap", type=int, default=50)
    ap.add_argument("--adaptive", action="store_true",
                    help="adaptive trees with W- and X-lists (lpb_options.adaptive = 1; the oracle sample too)")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=None, help="charges per layer of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path would shard by "
              "assigning independent FMMs (and systems of a batch) to GPUs and summing the output slots with "
              "one reduce", file=sys.stderr)
        sys.exit(2)
    wl = args.workload
    p = args.p if args.p is not None else {"uniform": 10, "clustered": 6, "interface": 6, "batch": 8, "paper": 5}[wl]
    per_layer = args.per_layer if args.per_layer is not None else {"uniform": 1_000_000, "clustered": 100_000,
                                                                   "interface": 100_000, "batch": 0, "paper": 0}[wl]
    ad = 1 if args.adaptive else 0

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

    if wl == "batch":
        probs = [inputs.batch_system(k) for k in range(args.systems)]
        ntot = sum(pr.n for pr in probs)
        desc = (f"{args.systems} independent 3-layer systems (system k: seed 1000+k, N log-uniform in [1e3,5e4], "
                f"eps~U[1,80], lambda~U[0.5,3], middle thickness~U[0.8,2]), one batched evaluation")
        print(f"[bench] workload: {args.systems} systems, {ntot} charges, p={p}", file=sys.stderr, flush=True)
        mixed = time_batch(lpb, torch, probs, p, args.leaf_cap, lpb.LPB_MIXED, args.steps, args.warmup)
        print(f"[bench] mixed: {mixed['eval_ms']:.2f} ms/eval, stages {mixed['stage_ms']}", file=sys.stderr, flush=True)
        fp64 = time_batch(lpb, torch, probs, p, args.leaf_cap, lpb.LPB_FP64, args.fp64_steps, 1)
        print(f"[bench] fp64: {fp64['eval_ms']:.2f} ms/eval, stages {fp64['stage_ms']}", file=sys.stderr, flush=True)
        rel = [max(err2_per_layer(a, b, pr.layer)) for a, b, pr in zip(mixed["phi"], fp64["phi"], probs)]
        rel_layers = None
        sample = []
        for pr in probs:
            if sum(x.n for x in sample) >= (args.cpu_sample or 300_000):
                break
            sample.append(pr)
        sample_what = f"the first {len(sample)} systems of the batch"
    else:
        clustered = wl == "clustered"
        if wl == "interface":
            prob = inputs.three_layer_interface_clusters(per_layer, seed=0)
            desc = (f"3-layer medium eps=(1,2,4) lambda=(1.2,1.5,2.0) d=(0,-1.2), {per_layer}/layer, half uniform "
                    "in the layer's slab (0.02 from the interfaces), half Gaussian (sigma 0.04) next to an interface, "
                    "q~U[-1,1], seed 0")
        elif wl == "paper":
            prob = inputs.paper_domains(args.charges, seed=0)
            counts = "+".join(str(int((prob.layer == l).sum())) for l in range(3))
            desc = (f"the paper's test problem: eps=(1,8.6,20.5) lambda=(1.2,0.5,2.1) d=(0,-1.2), {counts} charges "
                    "uniform in the P_4-shaped bodies (a=0.1,0.15,0.05; centres z=0.6,-0.6,-1.8), q~U[-1,1], seed 0")
        else:
            prob = inputs.three_layer(per_layer, seed=0, clustered_fraction=0.5 if clustered else 0.0, sigma=0.1)
            desc = (f"3-layer medium eps=(1,2,4) lambda=(1.2,1.5,2.0) d=(0,-1.2), {per_layer}/layer "
                    + ("50% uniform + 50% Gaussian (sigma 0.1) in unit cubes" if clustered else "uniform unit cubes")
                    + ", q~U[-1,1], seed 0")
        ntot = prob.n
        print(f"[bench] workload: 3 layers, {ntot} charges, p={p}", file=sys.stderr, flush=True)
        mixed = time_context(lpb, torch, prob, p, args.leaf_cap, lpb.LPB_MIXED, args.steps, args.warmup, adaptive=ad)
        print(f"[bench] mixed: {mixed['eval_ms']:.2f} ms/eval, stages {mixed['stage_ms']}", file=sys.stderr, flush=True)
        fp64 = time_context(lpb, torch, prob, p, args.leaf_cap, lpb.LPB_FP64, args.fp64_steps, 1, adaptive=ad)
        print(f"[bench] fp64: {fp64['eval_ms']:.2f} ms/eval, stages {fp64['stage_ms']}", file=sys.stderr, flush=True)
        rel_layers = err2_per_layer(mixed["phi"], fp64["phi"], prob.layer)
        rel = rel_layers
        cs = args.cpu_sample or (200_000 if not clustered else 100_000)
        if wl == "paper":
            sample = [inputs.paper_domains(3 * cs, seed=0)]
            sample_what = f"the same recipe at {3 * cs} charges"
        elif wl == "interface":
            sample = [inputs.three_layer_interface_clusters(cs, seed=0)]
            sample_what = f"the same recipe at {cs} charges per layer"
        else:
            sample = [inputs.three_layer(cs, seed=0, clustered_fraction=0.5 if clustered else 0.0, sigma=0.1)]
            sample_what = f"the same recipe at {cs} charges per layer"

    st = mixed["stats"]
    headline = wl == "uniform" and per_layer == 1_000_000 and p == 10
    roof = roofline(st, mixed["stage_ms"], p, True, traffic_ok=headline)
    fp64_roof = roofline(fp64["stats"], fp64["stage_ms"], p, False)
    fp64_roof.pop("traffic", None)

    ms = mixed["eval_ms"]
    line = {
        "metric": f"charges/sec (3-layer potential, p={p}): mixed-batched vs FP64 at <=1e-6 rel err",
        "value": ntot / (ms * 1e-3),
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
        "config": {"workload": desc, "charges": ntot, "p": p, "leaf_cap": args.leaf_cap, "precision": "mixed",
                   "tree": "adaptive" if ad else "uniform"},
        "fp64_value": ntot / (fp64["eval_ms"] * 1e-3),
        "fp64_ms_per_step": fp64["eval_ms"],
        "speedup_vs_fp64": fp64["eval_ms"] / ms,
        "rel_err_vs_fp64": max(rel),
        "wall_ms_per_step": mixed["wall_s"] * 1e3,
        "eager_ms_per_step": mixed["eval_ms_eager"],
        "schedules": {"tile": st["tile_schedule"], "batch": st["batch_schedule"], "tune_ms": st["t_tune_ms"]},
        "stage_ms": {k: round(v, 4) for k, v in mixed["stage_ms"].items()},
        "fp64_stage_ms": {k: round(v, 4) for k, v in fp64["stage_ms"].items()},
        "setup": {"tree_build_s": mixed["t_build_s"], "opgen_ms": st["t_opgen_ms"], "n_m2l_pairs": st["n_m2l_pairs"],
                  "n_w_pairs": st["n_w_pairs"], "n_x_pairs": st["n_x_pairs"], "n_point_ops": st["n_point_ops"],
                  "n_p2p_pairs": st["n_p2p_pairs"], "n_operators": st["n_operators"],
                  "operator_bytes": st["operator_bytes"], "max_depth": st["max_depth"]},
        "roofline": roof,
        "fp64_roofline": fp64_roof,
    }
    if rel_layers is not None:
        line["rel_err_vs_fp64_per_layer"] = rel_layers
    if wl == "paper" and ntot in PAPER_TABLE1:
        free_s, react_s = PAPER_TABLE1[ntot]
        line["paper_context"] = {
            "what": "the paper's timing table, 36 cores of 2x Xeon E5-2699 v4 (DASHMM, CPU), same N and p = 5; "
                    "other hardware, context only",
            "free_s": free_s, "reaction_s": react_s, "charges_per_s": ntot / (free_s + react_s)}
    gate = max(rel) <= 1e-6
    line["gate"] = {"rel_err_max": max(rel), "bar": 1e-6, "pass": bool(gate)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sample, p, args.leaf_cap, sample_what, adaptive=bool(ad))
        if wl != "batch":
            # the same oracle on one host core, on a tenth of the sample
            small = [shrink(pr, 10) for pr in sample]
            line["cpu_baseline_1core"] = cpu_baseline(small, p, args.leaf_cap, sample_what + " (every 10th charge)",
                                                      cores=1, adaptive=bool(ad))
    print(json.dumps(line), flush=True)
    if not gate:
        print(f"[bench] mixed-precision error {max(rel):.3e} above the 1e-6 bar", file=sys.stderr, flush=True)
        sys.exit(3)


if __name__ == "__main__":
    main()
