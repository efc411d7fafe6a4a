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
PEAK_FP32_VALU_TFLOPS = 78.6  # non-packed FP32 FMA, same unit count as FP64
PEAK_HBM_GBS = 8000.0


def f_m2l(p: int) -> int:
    f_roty = 2 * p * (4 * p * p - 1) // 3
    f_rotz = 3 * p * (p - 1)
    f_coax = 2 * p * (2 * p * p + 1) // 3
    return 2 * (2 * f_roty + 2 * f_rotz + f_coax) + 6 * p * p


# the M2L kernel the library runs for the cube workloads (FP64 p = 12, FP32 p = 10)
M2L_KERNEL = {0: "k_m2l_half", 1: "k_m2l_half"}  # by lhf_precision (FP64 = 0, FP32 = 1)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(which):
    """HBM bytes per M2L launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary,
    or None when the kernel's source changed after the counters were taken"""
    import hashlib
    import re
    try:
        md = open(os.path.join(ROOT, "profiles", "m2l_cube1m_hbm.md")).read()
        js = json.loads(re.search(r"```json\n(.*?)\n```", md, re.S).group(1))[which]
        src = open(os.path.join(ROOT, "paper_1201_5430_amd", "csrc", js["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest()[:16] != js["source_sha256_prefix"]:
            return None
        return js["bytes_per_launch"]
    except Exception:
        return None


def accuracy(cfg, v, s, n_targets=1000):
    """relative L2 error of v and s against the oracle's split-kernel direct sum on sampled
    targets (the paper measures on 1000 random source points); oracle leg of the benchmark"""
    import numpy as np
    import oracle
    import workloads
    x, w, a, d = cfg["x"], cfg["w"], cfg["a"], cfg["depth"]
    if cfg.get("precision") == "fp32":
        x = x.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
        a = float(np.float32(a))
    tg = workloads.sample_targets(x.shape[0], n_targets, seed=1000)
    vd, sd = oracle.direct(x, w, a, mode=oracle.DIRECT_SPLIT, depth=d, targets=tg)
    ev = float(np.linalg.norm(v[tg] - vd) / np.linalg.norm(vd))
    es = float(np.linalg.norm(s[tg] - sd) / np.linalg.norm(sd))
    return {"rel_l2_v": ev, "rel_l2_s": es, "targets": int(len(tg)),
            "reference": "split-kernel direct sum (Gaussian core between adjacent leaves, singular beyond), FP64 oracle"}


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


def run_batch(lhf, torch, steps, warmup, with_accuracy):
    """256 independent systems (sizes log-uniform in [1024, 65536]) in one batch: per-system
    depth from the measured cost model, all depth groups replayed as one HIP graph"""
    import numpy as np
    import workloads
    cfg = workloads.CONFIGS["batch256_fp32"]
    sizes, systems = workloads.batched(cfg["n_systems"], cfg["seed"])
    p, ns = cfg["p"], len(sizes)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = np.concatenate([sx for sx, _ in systems])
    w = np.concatenate([sw for _, sw in systems])
    a = np.array([workloads.core_radius(int(k)) for k in sizes])
    n = int(off[-1])
    log(f"bench: batch of {ns} systems, N = {n}, p = {p}, FP32")
    xt = torch.from_numpy(x).to(device="cuda", dtype=torch.float32)
    wt = torch.from_numpy(w).to(device="cuda", dtype=torch.float32)
    v = torch.empty_like(wt)
    s = torch.empty_like(wt)
    t0 = time.perf_counter()
    tune = lhf.autotune(p, lhf.FP32)
    t_tune = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = lhf.Batch(xt, off, a, p=p, precision=lhf.FP32, tune=tune)
    torch.cuda.synchronize()
    t_plan_cold = time.perf_counter() - t0
    # a plan rebuilt every step takes its device blocks from the blocks the previous one
    # released: the per-step plan cost is the mean over a few rebuilds
    n_rebuild = max(1, min(steps, 3))
    t0 = time.perf_counter()
    for _ in range(n_rebuild):
        B.close()
        B = lhf.Batch(xt, off, a, p=p, precision=lhf.FP32, tune=tune)
    torch.cuda.synchronize()
    t_plan = (time.perf_counter() - t0) / n_rebuild
    info = B.info()
    for _ in range(max(warmup, 1)):
        B.execute(wt, v, s, graph=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        B.execute(wt, v, s, graph=True)
    ev1.record()
    torch.cuda.synchronize()
    ms_exec = ev0.elapsed_time(ev1) / steps
    log(f"bench: batch graph {ms_exec:.3f} ms per execute")
    # the same systems as separate single-system plans, executed one after another
    plans = []
    for k in range(ns):
        i0, i1 = int(off[k]), int(off[k + 1])
        plans.append((lhf.Plan(xt[i0:i1], float(a[k]), p=p, depth=int(info["depths"][k]), precision=lhf.FP32),
                      i0, i1))
    vs, ss = torch.empty_like(wt), torch.empty_like(wt)
    for pl, i0, i1 in plans:
        pl.execute(wt[i0:i1], vs[i0:i1], ss[i0:i1])
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        for pl, i0, i1 in plans:
            pl.execute(wt[i0:i1], vs[i0:i1], ss[i0:i1])
    ev1.record()
    torch.cuda.synchronize()
    ms_sep = ev0.elapsed_time(ev1) / steps
    for pl, _, _ in plans:
        pl.close()
    depths, counts = np.unique(info["depths"], return_counts=True)
    res = {
        "workload": "batch256_fp32", "n_systems": ns, "n": n, "p": p,
        "sizes": {"min": int(sizes.min()), "median": int(np.median(sizes)), "max": int(sizes.max())},
        "depth_groups": {int(dd): int(c) for dd, c in zip(depths, counts)},
        "core_split_warning": bool(B.warn_core_split),
        "tune": {"t_box_ns": tune.t_box_ns, "t_pair_ns": tune.t_pair_ns, "seconds": t_tune},
        "plan_ms": t_plan * 1e3,
        "plan_first_ms": t_plan_cold * 1e3,
        "execute_ms": ms_exec,
        "elements_per_s": n / ((t_plan * 1e3 + ms_exec) * 1e-3),
        "execute_only_elements_per_s": n / (ms_exec * 1e-3),
        "mean_system_execute_us": ms_exec * 1e3 / ns,
        "separate_plans_execute_ms": ms_sep,
        "graph_speedup_vs_separate_plans": ms_sep / ms_exec,
        "counts": {"m2l": info["n_m2l"], "p2p_pairs": info["n_p2p_pairs"]},
    }
    if with_accuracy:
        import oracle
        vh, sh = v.double().cpu().numpy(), s.double().cpu().numpy()
        errs = []
        order = np.argsort(sizes)
        for k in (int(order[0]), int(order[ns // 2]), int(order[-1])):
            i0, i1 = int(off[k]), int(off[k + 1])
            xk = x[i0:i1].astype(np.float32).astype(np.float64)
            wk = w[i0:i1].astype(np.float32).astype(np.float64)
            tg = workloads.sample_targets(i1 - i0, 200, seed=2000 + k)
            vd, sd = oracle.direct(xk, wk, float(np.float32(a[k])), mode=oracle.DIRECT_SPLIT,
                                   depth=int(info["depths"][k]), targets=tg)
            errs.append({"system": k, "n": i1 - i0, "depth": int(info["depths"][k]),
                         "rel_l2_v": float(np.linalg.norm(vh[i0:i1][tg] - vd) / np.linalg.norm(vd)),
                         "rel_l2_s": float(np.linalg.norm(sh[i0:i1][tg] - sd) / np.linalg.norm(sd))})
        res["accuracy_sampled_systems"] = errs
    B.close()
    return res


def run_ring(lhf, torch, steps, warmup, with_accuracy):
    """clustered workload: 4,194,304 elements on a vortex ring + 10% background, adaptive octree
    (<= 64 per leaf, deepest level 8), p = 16; the FP32 path timed per step (plan + execute),
    the FP64 path on the same input for the speedup"""
    import numpy as np
    import workloads
    cfg = workloads.CONFIGS["ring4m_fp32"]
    n, p, mx, depth = cfg["n"], cfg["p"], cfg["max_per_leaf"], 8
    x, w = workloads.vortex_ring(n, cfg["seed"])
    a = workloads.core_radius(n)
    log(f"bench: ring N={n} p={p} adaptive <= {mx}/leaf")
    res = {"workload": "ring4m_fp32", "n": n, "p": p, "max_per_leaf": mx, "max_level": depth,
           "distribution": "vortex ring R0 = 0.3, Gaussian cross-section sigma = 0.05, + 10% uniform background"}
    outs = {}
    for prec, name, k_steps in ((lhf.FP32, "fp32", steps), (lhf.FP64, "fp64", max(1, min(steps, 2)))):
        dt = torch.float32 if prec == lhf.FP32 else torch.float64
        xt = torch.from_numpy(x).to(device="cuda", dtype=dt)
        wt = torch.from_numpy(w).to(device="cuda", dtype=dt)
        v, s = torch.empty_like(wt), torch.empty_like(wt)
        for _ in range(warmup if prec == lhf.FP32 else 1):
            pl = lhf.Plan(xt, a, p=p, depth=depth, precision=prec, max_per_leaf=mx)
            pl.execute(wt, v, s)
            pl.close()
        torch.cuda.synchronize()
        phases = {k: 0.0 for k in lhf.PHASES}
        t0 = time.perf_counter()
        for _ in range(k_steps):
            pl = lhf.Plan(xt, a, p=p, depth=depth, precision=prec, max_per_leaf=mx)
            pl.profile_begin(1)
            pl.execute(wt, v, s)
            ph, _ = pl.profile_end()
            st = pl.stats()
            pl.close()
            for kk in phases:
                phases[kk] += ph[kk] / k_steps
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / k_steps
        exec_ms = sum(vv for kk, vv in phases.items() if kk != "m2l")
        log(f"bench: ring {name} {ms:.1f} ms per step")
        res[name] = {"ms_per_step": ms, "elements_per_s": n / (ms * 1e-3), "execute_ms": exec_ms,
                     "execute_only_elements_per_s": n / (exec_ms * 1e-3), "phases_ms": phases, "steps": k_steps,
                     "m2l_achieved_tflops": st["n_m2l"] * f_m2l(p) / (phases["m2l"] * 1e-3) / 1e12}
        res["counts"] = {"boxes": st["boxes"], "leaves": st["n_leaves"], "m2l": st["n_m2l"],
                         "u_pairs": st["n_p2p_pairs"], "wx_pairs": st["n_wx_pairs"]}
        outs[name] = (v.double().cpu().numpy(), s.double().cpu().numpy())
        del xt, wt, v, s
    res["speedup_fp32_vs_fp64"] = res["fp64"]["ms_per_step"] / res["fp32"]["ms_per_step"]
    if with_accuracy:
        import oracle
        tg = workloads.sample_targets(n, 200, seed=3000)
        xr = x.astype(np.float32).astype(np.float64)
        wr = w.astype(np.float32).astype(np.float64)
        vd, sd = oracle.direct_adaptive(xr, wr, float(np.float32(a)), mx, depth, targets=tg)
        vd64, sd64 = oracle.direct_adaptive(x, w, a, mx, depth, targets=tg)
        acc = {}
        for name, (vv, ss) in outs.items():
            rv, rs = (vd, sd) if name == "fp32" else (vd64, sd64)
            acc[name] = {"rel_l2_v": float(np.linalg.norm(vv[tg] - rv) / np.linalg.norm(rv)),
                         "rel_l2_s": float(np.linalg.norm(ss[tg] - rs) / np.linalg.norm(rs))}
        res["accuracy_vs_direct_sum"] = dict(acc, targets=int(len(tg)),
                                             reference="adaptive split-kernel direct sum, FP64 oracle")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube1m_fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 run on the same input")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-system batched run")
    ap.add_argument("--no-ring", action="store_true", help="skip the clustered (vortex ring, adaptive) run")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="only copy a buffer of this many MiB on the device (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(see the sharding design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calib_copy:
        nbytes = args.calib_copy << 20
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": nbytes}), flush=True)
        return

    import paper_1201_5430_amd as lhf
    import workloads
    if not os.path.exists(lhf.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    def run(name, steps, warmup):
        cfg = workloads.make(name)
        prec = lhf.FP64 if cfg["precision"] == "fp64" else lhf.FP32
        dt = torch.float64 if prec == lhf.FP64 else torch.float32
        n, p, d, a = cfg["n"], cfg["p"], cfg["depth"], cfg["a"]
        log(f"bench: workload {name} N={n} p={p} depth={d} precision={cfg['precision']}")
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

        for k in range(warmup):
            step()
            log(f"bench: {name} warmup {k + 1}/{warmup} done")
        torch.cuda.synchronize()
        phases = {k: 0.0 for k in lhf.PHASES}
        t0 = time.perf_counter()
        for k in range(steps):
            ph, st = step(profile=True)
            for kk in phases:
                phases[kk] += ph[kk]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        log(f"bench: {name} {steps} timed steps done")
        ms_step = (t1 - t0) * 1e3 / steps
        ph_step = {k: vv / steps for k, vv in phases.items()}
        exec_ms = sum(vv for kk, vv in ph_step.items() if kk != "m2l")  # m2l is part of "down"
        launches = sum(1 for l in range(2, d + 1) if st["boxes"][l] > 0)
        flops = st["n_m2l"] * f_m2l(p)
        achieved = flops / (ph_step["m2l"] * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if prec == lhf.FP64 else PEAK_FP32_MFMA_TFLOPS
        return dict(cfg=cfg, prec=prec, n=n, p=p, d=d, ms_step=ms_step, ph_step=ph_step, exec_ms=exec_ms,
                    st=st, launches=launches, flops=flops, achieved=achieved, peak=peak,
                    v=v.double().cpu().numpy(), s=s.double().cpu().numpy())

    r = run(args.workload, args.steps, args.warmup)
    cfg, prec, n, p, d = r["cfg"], r["prec"], r["n"], r["p"], r["d"]
    out = {
        "metric": METRIC,
        "value": n / (r["ms_step"] * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == lhf.FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "depth": d, "precision": cfg["precision"],
                   "distribution": "uniform in [0,1)^3, omega ~ N(0,1)^3, Gaussian core a = 0.5 N^(-1/3)",
                   "step": "plan (keys, sort, octree, lists, tables) + execute (P2M, M2M, M2L/L2L, L2P, P2P)"},
        "execute_ms": r["exec_ms"],
        "plan_ms": r["ms_step"] - r["exec_ms"],
        "execute_only_elements_per_s": n / (r["exec_ms"] * 1e-3),
        "phases_ms": r["ph_step"],
        "counts": {"m2l": r["st"]["n_m2l"], "p2p_pairs": r["st"]["n_p2p_pairs"], "boxes": r["st"]["boxes"]},
        "roofline": {
            "kernel": M2L_KERNEL[prec] + " (batched M2L), one launch per level 2..d",
            "bound": "alu",
            "achieved": r["achieved"],
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": r["achieved"] / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic("fp64" if prec == lhf.FP64 else "fp32"),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)",
            "launches_per_step": r["launches"],
            "avg_launch_ms": r["ph_step"]["m2l"] / r["launches"],
            "flop_per_launch": r["flops"] / r["launches"],
            "flop_per_m2l": f_m2l(p),
        },
    }
    r32 = None
    if args.workload == "cube1m_fp64" and not args.no_fp32:
        # the mixed-precision path on the same input (FP32 elements and expansions, p = 10)
        r32 = run("cube1m_fp32", args.steps, args.warmup)
        out["fp32"] = {
            "workload": "cube1m_fp32", "p": r32["p"], "ms_per_step": r32["ms_step"],
            "elements_per_s": r32["n"] / (r32["ms_step"] * 1e-3),
            "execute_only_elements_per_s": r32["n"] / (r32["exec_ms"] * 1e-3),
            "speedup_vs_fp64": r["ms_step"] / r32["ms_step"],
            "phases_ms": r32["ph_step"],
            "m2l_achieved_tflops": r32["achieved"],
            "m2l_frac_of_fp32_vector_peak": r32["achieved"] / PEAK_FP32_VALU_TFLOPS,
        }
    if args.workload == "cube1m_fp64" and not args.no_batch:
        out["batch"] = run_batch(lhf, torch, args.steps, args.warmup, not args.no_cpu_baseline)
    if args.workload == "cube1m_fp64" and not args.no_ring:
        out["ring"] = run_ring(lhf, torch, args.steps, args.warmup, not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (sampled) ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
        log("bench: accuracy against the oracle's direct sum on 1000 sampled targets ...")
        out["cpu_baseline"]["accuracy_fp64_path"] = accuracy(cfg, r["v"], r["s"])
        if r32 is not None:
            out["cpu_baseline"]["accuracy_fp32_path"] = accuracy(r32["cfg"], r32["v"], r32["s"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
