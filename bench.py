"""Benchmark of one FMM evaluation of v and s (the whole hot path) on one GPU.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A step is one pass of the whole path over the synthetic input, already
resident in device memory: plan (Morton keys, sort, octree, interaction lists,
operator tables) + execute (P2M, M2M, M2L/L2L, L2P, P2P) for N elements.
Prints ONE JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.

Roofline: the dominant kernel is the downward pass (M2L + L2L, one launch per
level); its time comes from HIP events recorded by the library on the execute
stream during the timed steps.  Algorithmic work per M2L translation (RCR,
both potentials, real-packed):
    F(p) = 2 [2 F_roty + 2 F_rotz + F_coax] + 6 p^2,
    F_roty = 2p(4p^2-1)/3, F_rotz = 3p(p-1), F_coax = 2p(2p^2+1)/3
(25,472 flop at p = 12), times the number of M2L translations.
CPU baseline: the FP64 oracle (direct-mode translations) on the same input:
full upward pass plus the downward pass and near field of a seeded sample of
leaves; the full-job time is projected from the per-translation and per-pair
rates of the sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "vortex elements/s (v + stretching) at rel err 1e-6; FP32-MFMA vs FP64 speedup"
PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def f_m2l(p: int) -> int:
    f_roty = 2 * p * (4 * p * p - 1) // 3
    f_rotz = 3 * p * (p - 1)
    f_coax = 2 * p * (2 * p * p + 1) // 3
    return 2 * (2 * f_roty + 2 * f_rotz + f_coax) + 6 * p * p


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, n_leaves=64):
    import oracle
    import workloads
    x, w, a, p, d = cfg["x"], cfg["w"], cfg["a"], cfg["p"], cfg["depth"]
    samp = workloads.sample_targets(x.shape[0], n_leaves, seed=99)
    t0 = time.perf_counter()
    _, _, st = oracle.fmm(x, w, a, p, d, sample=samp)
    wall = time.perf_counter() - t0
    _, m2l_tot, pairs_tot = oracle.tree_counts(x, d)
    t_down = st["t_down"] * m2l_tot / max(st["n_m2l"], 1)
    t_near = st["t_near"] * pairs_tot / max(st["n_p2p_pairs"], 1)
    t_job = st["t_tree"] + st["t_up"] + t_down + t_near
    return {
        "value": x.shape[0] / t_job, "unit": "elements/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": (f"FP64 oracle (direct O(p^4) translations) on the same {x.shape[0]}-element input: full tree + "
                   f"upward pass, downward pass + near field for the {len(set(samp.tolist()))} leaves of "
                   f"{n_leaves} seeded elements ({st['n_m2l']} M2L, {st['n_p2p_pairs']} pairs); full-job time "
                   f"projected from the per-translation and per-pair rates: {t_job:.1f} s "
                   f"(sample wall {wall:.1f} s)"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube1m_fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1201_5430_amd as lhf
    import workloads
    if not os.path.exists(lhf.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    cfg = workloads.make(args.workload)
    prec = lhf.FP64 if cfg["precision"] == "fp64" else lhf.FP32
    dt = torch.float64 if prec == lhf.FP64 else torch.float32
    n, p, d, a = cfg["n"], cfg["p"], cfg["depth"], cfg["a"]
    log(f"bench: workload {args.workload} N={n} p={p} depth={d} precision={cfg['precision']}")
    xt = torch.from_numpy(cfg["x"]).to(device="cuda", dtype=dt)
    wt = torch.from_numpy(cfg["w"]).to(device="cuda", dtype=dt)
    v = torch.empty_like(wt)
    s = torch.empty_like(wt)

    def step(profile=False):
        plan = lhf.Plan(xt, a, p=p, depth=d, precision=prec)
        if profile:
            plan.profile_begin(1)
        plan.execute(wt, v, s)
        ph = None
        if profile:
            ph, _ = plan.profile_end()
        st = plan.stats()
        plan.close()
        return ph, st

    for k in range(args.warmup):
        step()
        log(f"bench: warmup {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    phases = {k: 0.0 for k in lhf.PHASES}
    t0 = time.perf_counter()
    for k in range(args.steps):
        ph, st = step(profile=True)
        for kk in phases:
            phases[kk] += ph[kk]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"bench: {args.steps} timed steps done")
    ms_step = (t1 - t0) * 1e3 / args.steps
    ph_step = {k: vv / args.steps for k, vv in phases.items()}
    exec_ms = sum(ph_step.values())

    # dominant kernel: downward pass (M2L + L2L), one launch per level 2..d
    launches = sum(1 for l in range(2, d + 1) if st["boxes"][l] > 0)
    flops = st["n_m2l"] * f_m2l(p)
    down_s = ph_step["down"] * 1e-3
    achieved = flops / down_s / 1e12
    peak = PEAK_FP64_TFLOPS if prec == lhf.FP64 else PEAK_FP32_MFMA_TFLOPS
    out = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == lhf.FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "depth": d, "precision": cfg["precision"],
                   "distribution": "uniform in [0,1)^3, omega ~ N(0,1)^3, Gaussian core a = 0.5 N^(-1/3)",
                   "step": "plan (keys, sort, octree, lists, tables) + execute (P2M, M2M, M2L/L2L, L2P, P2P)"},
        "execute_ms": exec_ms,
        "plan_ms": ms_step - exec_ms,
        "execute_only_elements_per_s": n / (exec_ms * 1e-3),
        "phases_ms": ph_step,
        "counts": {"m2l": st["n_m2l"], "p2p_pairs": st["n_p2p_pairs"], "boxes": st["boxes"]},
        "roofline": {
            "kernel": "k_down (M2L + L2L, one launch per level)",
            "bound": "alu" if prec == lhf.FP64 else "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "launches_per_step": launches,
            "avg_launch_ms": ph_step["down"] / launches,
            "flop_per_launch": flops / launches,
            "flop_per_m2l": f_m2l(p),
        },
    }
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (sampled) ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
