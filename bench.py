"""Benchmark of one FMM evaluation of v and s (the whole hot path) on one GPU.

    python bench.py [--steps K] [--warmup W] [--p P] [--legs ring16,wx,scalar,filament,cube,batch]
                    [--no-cpu-baseline] [--calib-copy MIB]

A step is one pass of the whole path over the synthetic input, already resident
in device memory: plan (Morton keys, sort, octree, interaction lists, operator
tables) + execute (P2M, M2M, M2L/L2L, L2P, P2P) for N elements.  Prints ONE JSON
line.  Only one GPU is used: --gpus above 1 exits.

Headline: the clustered workload (4,194,304 elements on a vortex ring with 10%
uniform background, adaptive octree of at most 64 elements per leaf down to level
8) in FP64 at the smallest order p whose relative L2 errors of v and s against the
split-kernel direct sum are both <= 1e-6 (p = 23 by the error-vs-order sweep; the
run measures the errors it reaches on 4096 seeded targets with the oracle).  The
other legs are labelled sections of the same line: the same ring at p = 16 in FP32
and FP64 (the precision speedup), the ring in FP64 at p = 16 with the W/X lists by
M2P / P2L instead of direct sums, the scalar harmonic FMM against the vortex FMM on
the 2^20-element cube (the paper's comparison), the 2^20-element uniform cube (FP64
p = 12, FP32 p = 10) and the batch of 256 systems.

Roofline: per phase (gather, P2M, M2M, M2L + L2L, L2P, P2P) the algorithmic work
(flop and compulsory HBM bytes, counted in roofline_work()) against the MI355X
peaks, T_roof = sum over phases of max(flop / peak, bytes / 8 TB/s), and the
aggregate T_roof / T_meas.  The dominant kernel (the batched M2L) is reported in
the 'roofline' object: algorithmic flop per launch over its average launch time,
measured with HIP events the library records on the execute stream.

CPU baseline: the FP64 oracle (direct O(p^4) translation matrices, OpenMP), timed
on the host: per-operation rates measured on a bounded sample of the same
workload and projected to the whole job with the plan's own counts.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "vortex elements/s (v + stretching) at rel err 1e-6; FP32-MFMA vs FP64 speedup"
P_STAR = 23  # smallest p with eps2(v), eps2(s) <= 1e-6 on the ring (error-vs-order sweep)
PEAK_FP64_TFLOPS = 78.6          # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (vector and matrix)
PEAK_FP32_VALU_TFLOPS = 78.6     # non-packed FP32 FMA: the same unit count (the build forbids packed FP32)
PEAK_FP32_MFMA_TFLOPS = 157.3    # FP32 matrix cores
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def f_m2l(p: int) -> int:
    """algorithmic flop of one M2L translation (RCR, both potentials, real-packed; FMA = 2)"""
    f_roty = 2 * p * (4 * p * p - 1) // 3
    f_rotz = 3 * p * (p - 1)
    f_coax = 2 * p * (2 * p * p + 1) // 3
    return 2 * (2 * f_roty + 2 * f_rotz + f_coax) + 6 * p * p


def f_mm(p: int) -> int:
    """M2M / L2L translation: the same rotations and a triangular coaxial block (half the
    Hankel block's flop), conversion 4 p^2"""
    f_roty = 2 * p * (4 * p * p - 1) // 3
    f_rotz = 3 * p * (p - 1)
    f_coax = p * (2 * p * p + 1) // 3
    return 2 * (2 * f_roty + 2 * f_rotz + f_coax) + 4 * p * p


def roofline_work(st, p, prec, n):
    """algorithmic flop and compulsory HBM bytes per phase of one execute"""
    T = 8 if prec == 0 else 4
    nbox = sum(st["boxes"])
    nleaf = st["n_leaves"] or st["boxes"][-1]
    exp_b = 2 * p * p * T  # one expansion (phi, chi)
    pairs_u, pairs_wx = st["n_p2p_pairs"], st["n_wx_pairs"]
    return {
        "gather": (0.0, n * (3 * T + 4 + 3 * T) + n * (3 * T + 8 * T)),
        "p2m": (40.0 * p * p * n, 6 * T * n + nleaf * exp_b),
        "m2m": (st["n_m2m"] * f_mm(p), 2.0 * nbox * exp_b),
        "down": (st["n_m2l"] * f_m2l(p) + st["n_l2l"] * f_mm(p), 3.0 * nbox * exp_b),
        "l2p": (34.0 * p * p * n, nleaf * exp_b + 12 * T * n),
        "p2p": (70.0 * pairs_u + 56.0 * pairs_wx, 20 * T * n),
    }


def phase_roofline(st, ph, p, prec, n):
    peak = PEAK_FP64_TFLOPS if prec == 0 else PEAK_FP32_VALU_TFLOPS
    work = roofline_work(st, p, prec, n)
    out, t_roof, t_meas = {}, 0.0, 0.0
    for k, (fl, by) in work.items():
        ms = ph[k]
        tr = max(fl / (peak * 1e12), by / (PEAK_HBM_GBS * 1e9)) * 1e3
        bound = "alu" if fl / (peak * 1e12) >= by / (PEAK_HBM_GBS * 1e9) else "hbm"
        out[k] = {"ms": ms, "flop": fl, "bytes": by, "bound": bound, "t_roof_ms": tr,
                  "frac": tr / ms if ms > 0 else None,
                  "achieved_tflops": fl / (ms * 1e-3) / 1e12 if ms > 0 else None,
                  "achieved_gbs": by / (ms * 1e-3) / 1e9 if ms > 0 else None}
        t_roof += tr
        t_meas += ms
    return out, {"t_roof_ms": t_roof, "t_meas_ms": t_meas, "frac": t_roof / t_meas if t_meas > 0 else None,
                 "peak_alu_tflops": peak, "peak_hbm_gbs": PEAK_HBM_GBS}


# the dominant kernel of the headline per M2L kernel family the plan chose
KERNEL_LABEL = {
    "half": "k_m2l_half<{t},{p}> (batched M2L, half-vector lanes, rotation tables from L2), one launch per level",
    "quarter": "k_m2l_quarter<{p}> (batched M2L, quarter-vector lanes, class rotation tables staged in LDS, "
               "pipelined table reads), one launch per level",
    "qmfma": "k_m2l_qmfma<{p}> (batched M2L on the FP64 matrix cores, vectors in registers), one launch per level",
    "tile": "k_m2l_tile<{t},{p},...> (batched M2L, LDS-tiled target boxes), one launch per level",
}


def measured_traffic(name):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None when the kernel's source changed since"""
    import hashlib
    import re
    try:
        md = open(os.path.join(ROOT, "profiles", f"m2l_{name}_hbm.md")).read()
        js = json.loads(re.search(r"```json\n(.*?)\n```", md, re.S).group(1))[name]
        src = open(os.path.join(ROOT, "paper_1201_5430_amd", "csrc", js["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest()[:16] != js["source_sha256_prefix"]:
            return None
        return js["bytes_per_launch"]
    except Exception:
        return None


def run_leg(lhf, torch, name, x, w, a, p, prec, depth, max_per_leaf, steps, warmup, wx=False, q=None, tune=False):
    """time `steps` plan + execute steps (inputs resident on the device); per-phase times from the
    library's HIP events on the execute stream.  tune: the run-time kernel shapes (M2L tile per
    level, near-field source tile) are measured once on a plan of the workload before the warm-up
    (not timed) and applied to every plan of the timed steps"""
    dt = torch.float64 if prec == lhf.FP64 else torch.float32
    xt = torch.from_numpy(x).to(device="cuda", dtype=dt)
    wt = torch.from_numpy(w).to(device="cuda", dtype=dt)
    v, s = torch.empty_like(wt), torch.empty_like(wt)
    qt = None if q is None else torch.from_numpy(q).to(device="cuda", dtype=dt)
    shapes, tune_s = None, None
    if tune:
        t0 = time.perf_counter()
        pl = lhf.Plan(xt, a, p=p, depth=depth, precision=prec, max_per_leaf=max_per_leaf, wx_expansions=wx)
        shapes = pl.autotune(wt)
        pl.close()
        tune_s = time.perf_counter() - t0
        log(f"bench: {name}: tuned shapes {shapes} in {tune_s:.1f} s")

    def step(profile):
        pl = lhf.Plan(xt, a, p=p, depth=depth, precision=prec, max_per_leaf=max_per_leaf, wx_expansions=wx)
        if shapes is not None:
            pl.set_shapes(shapes)
        if profile:
            pl.profile_begin(1)
        if qt is None:
            pl.execute(wt, v, s)
        else:  # the scalar harmonic FMM of the sources q on the same tree
            pl.execute_scalar(qt)
        ph = pl.profile_end()[0] if profile else None
        st = pl.stats()
        pl.close()
        return ph, st

    for k in range(warmup):
        step(False)
    torch.cuda.synchronize()
    phases = {k: 0.0 for k in lhf.PHASES}
    t0 = time.perf_counter()
    for k in range(steps):
        ph, st = step(True)
        for kk in phases:
            phases[kk] += ph[kk] / steps
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    exec_ms = sum(vv for kk, vv in phases.items() if kk != "m2l")  # m2l is part of "down"
    log(f"bench: {name}: {ms:.2f} ms per step (execute {exec_ms:.2f} ms, M2L {phases['m2l']:.2f} ms)")
    n = x.shape[0]
    # (the flop model counts both potentials: not applied to the scalar FMM)
    m2l_tf = st["n_m2l"] * f_m2l(p) / (phases["m2l"] * 1e-3) / 1e12 if phases["m2l"] > 0 and q is None else None
    res = {"workload": name, "n": n, "p": p, "precision": "fp64" if prec == lhf.FP64 else "fp32",
           "steps": steps, "ms_per_step": ms, "elements_per_s": n / (ms * 1e-3), "execute_ms": exec_ms,
           "plan_ms": ms - exec_ms, "execute_only_elements_per_s": n / (exec_ms * 1e-3), "phases_ms": phases,
           "m2l_kernel": st["m2l_kernel"], "m2l_achieved_tflops": m2l_tf,
           "counts": {"boxes": st["boxes"], "leaves": st["n_leaves"], "m2l": st["n_m2l"], "m2m": st["n_m2m"],
                      "u_pairs": st["n_p2p_pairs"], "wx_pairs": st["n_wx_pairs"], "m2p_pairs": st["n_m2p"],
                      "p2l_pairs": st["n_p2l"]}}
    if wx:
        res["wx_expansions"] = True
    if shapes is not None:
        res["tuned_shapes"] = shapes
        res["tune_s"] = tune_s
    if prec == lhf.FP64:
        res["m2l_frac_of_fp64_peak"] = m2l_tf / PEAK_FP64_TFLOPS if m2l_tf else None
    else:
        res["m2l_frac_of_fp32_valu_peak"] = m2l_tf / PEAK_FP32_VALU_TFLOPS if m2l_tf else None
        res["m2l_frac_of_fp32_mfma_peak"] = m2l_tf / PEAK_FP32_MFMA_TFLOPS if m2l_tf else None
    if q is None:
        res["phase_roofline"], res["aggregate_roofline"] = phase_roofline(st, phases, p, prec, n)
    out = (v.double().cpu().numpy(), s.double().cpu().numpy())
    del xt, wt, v, s
    return res, st, out


def run_filament(lhf, torch, steps, warmup):
    """vortex filaments (Sec. 5.3): 4096 closed rings of 256 straight segments (2^20 segments,
    2^20 vertices) in the unit cube, FP64 p = 12 on a uniform tree of depth 6 over the segment
    centres and the vertices; a step = filament set-up (tree over 2^21 points) + execute"""
    import numpy as np
    import workloads
    X, seg, G = workloads.filament_rings(4096, 256, 81)
    Xt = torch.from_numpy(X).cuda()
    st = torch.from_numpy(seg).cuda()
    Gt = torch.from_numpy(G).cuda()

    def step(profile):
        f = lhf.Filament(Xt, st, p=12, depth=6)
        pl = lhf.load().lhf_filament_plan(f._h)
        if profile:
            lhf._check(lhf.load().lhf_profile_begin(pl, 1))
        v = f.execute(Gt)
        ph = None
        if profile:
            import ctypes as C
            ms = (C.c_double * len(lhf.PHASES))()
            k = C.c_int32()
            lhf._check(lhf.load().lhf_profile_end(pl, ms, C.byref(k)))
            ph = dict(zip(lhf.PHASES, list(ms)))
        s = f.stats()
        f.close()
        return v, ph, s

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    phases = {k: 0.0 for k in lhf.PHASES}
    t0 = time.perf_counter()
    for _ in range(steps):
        v, ph, s = step(True)
        for k in phases:
            phases[k] += ph[k] / steps
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ex = sum(vv for kk, vv in phases.items() if kk != "m2l")
    log(f"bench: filaments: {ms:.2f} ms per step (execute {ex:.2f} ms)")
    return {"workload": "filaments_4096x256_fp64_p12", "segments": int(seg.shape[0]), "vertices": int(X.shape[0]),
            "p": 12, "depth": 6, "quadrature_points": 6, "steps": steps, "ms_per_step": ms, "execute_ms": ex,
            "segments_per_s": seg.shape[0] / (ms * 1e-3), "phases_ms": phases, "n_m2l": s["n_m2l"]}


def rel_err(v, s, tg, vd, sd):
    import numpy as np
    return {"rel_l2_v": float(np.linalg.norm(v[tg] - vd) / np.linalg.norm(vd)),
            "rel_l2_s": float(np.linalg.norm(s[tg] - sd) / np.linalg.norm(sd)),
            "max_v": float(np.abs(v[tg] - vd).max() / np.abs(vd).max()),
            "max_s": float(np.abs(s[tg] - sd).max() / np.abs(sd).max())}


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(x, w, a, p, mx, lmax, st, n_trans=60, n_targets=2048):
    """The FP64 oracle on the headline workload, timed on a bounded sample and projected to the
    whole job with the plan's counts:
      * translations: n_trans M2L translations of the oracle (full O(p^4) matrices, one thread)
        on the workload's own multipoles' shapes; M2M and L2L are costed as M2L (an upper
        bound); the oracle spreads them over its OpenMP threads;
      * near field: the oracle's pair sum (Gaussian core, OpenMP) of n_targets seeded targets
        over 131072 sources, scaled by the job's U and W/X pair count over the pairs sampled;
      * P2M and L2P: oracle calls on the elements of sampled leaves."""
    import numpy as np
    import oracle
    import workloads
    threads = oracle.num_threads()
    rng = np.random.default_rng(7)
    # translations (single thread)
    phi = rng.normal(size=p * p) + 1j * rng.normal(size=p * p)
    chi = rng.normal(size=p * p) + 1j * rng.normal(size=p * p)
    t0 = time.perf_counter()
    for k in range(n_trans):
        t = rng.integers(-3, 4, size=3).astype(float)
        t[0] = 2.0 + k % 2
        oracle.m2l(p, t * 2.0 ** -6, phi, chi)
    t_tr = (time.perf_counter() - t0) / n_trans
    # P2M + L2P per element (single thread), on 64-element boxes of the input
    xs, ws = x[:64], w[:64]
    c = xs.mean(0)
    t0 = time.perf_counter()
    for _ in range(5):
        ph, ch = oracle.p2m(p, c, xs, ws)
        oracle.l2p(p, c, ph, ch, xs, ws)
    t_el = (time.perf_counter() - t0) / (5 * 64)
    # near field: the oracle's pair sum with the Gaussian core (the costlier kernel of the near
    # field) over the first n_src elements for n_targets of them (OpenMP; no tree involved)
    n_src = min(x.shape[0], 131072)
    tg = workloads.sample_targets(n_src, n_targets, seed=4242)
    t0 = time.perf_counter()
    oracle.direct(x[:n_src], w[:n_src], a, mode=oracle.DIRECT_SMOOTH, targets=tg)
    t_near_s = time.perf_counter() - t0
    pairs_sampled = n_targets * (n_src - 1)
    n = x.shape[0]
    n_tr = st["n_m2l"] + st["n_m2m"] + st["n_l2l"]
    pairs_job = st["n_p2p_pairs"] + st["n_wx_pairs"]
    # the direct sum visits every source per target; the job's near field visits its pairs only
    t_near = t_near_s * pairs_job / pairs_sampled
    t_job_all = n_tr * t_tr / threads + n * t_el / threads + t_near
    t_job_1 = n_tr * t_tr + n * t_el + t_near * threads
    return {
        "value": n / t_job_all, "unit": "elements/s", "cores": threads, "kind": "oracle",
        "value_1core": n / t_job_1, "cpu_model": cpu_model(), "projected": True,
        "sample": (f"FP64 oracle (direct O(p^4) translation matrices, OpenMP) on the headline workload "
                   f"(N = {n}, p = {p}): {n_trans} M2L translations timed on one thread "
                   f"({t_tr * 1e3:.2f} ms each), P2M + L2P on 64-element boxes ({t_el * 1e6:.1f} us per element), "
                   f"the smoothed pair sum of {n_targets} targets over {n_src} sources "
                   f"({t_near_s:.2f} s on {threads} threads); projected with the plan's {n_tr} translations and {pairs_job} near-field pairs: "
                   f"{t_job_all:.0f} s on {threads} threads, {t_job_1:.0f} s on one"),
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
    depths, counts = np.unique(info["depths"], return_counts=True)
    res = {
        "workload": "batch256_fp32", "n_systems": ns, "n": n, "p": p,
        "sizes": {"min": int(sizes.min()), "median": int(np.median(sizes)), "max": int(sizes.max())},
        "depth_groups": {int(dd): int(c) for dd, c in zip(depths, counts)},
        "core_split_warning": bool(B.warn_core_split),
        "tune": {"t_box_ns": tune.t_box_ns, "t_pair_ns": tune.t_pair_ns, "seconds": t_tune},
        "plan_ms": t_plan * 1e3, "plan_first_ms": t_plan_cold * 1e3, "execute_ms": ms_exec,
        "elements_per_s": n / ((t_plan * 1e3 + ms_exec) * 1e-3),
        "execute_only_elements_per_s": n / (ms_exec * 1e-3),
        "mean_system_execute_us": ms_exec * 1e3 / ns,
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
            e = rel_err(vh[i0:i1], sh[i0:i1], tg, vd, sd)
            errs.append(dict(e, system=k, n=i1 - i0, depth=int(info["depths"][k])))
        res["accuracy_sampled_systems"] = errs
    B.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--p", type=int, default=P_STAR, help="order of the headline (FP64 ring) leg")
    ap.add_argument("--leg-steps", type=int, default=20, help="timed steps of the ring p = 16 and cube legs")
    ap.add_argument("--legs", default="ring16,wx,scalar,filament,cube,batch",
                    help="comma list of ring16, wx, scalar, filament, cube, batch (or none)")
    ap.add_argument("--targets", type=int, default=4096, help="sample targets of the headline accuracy")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle legs (baseline, accuracy)")
    ap.add_argument("--no-tune", action="store_true",
                    help="built-in kernel shapes (no run-time autotuning of M2L and near-field tiles)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="only copy a buffer of this many MiB on the device (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(see the sharding design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    legs = [s for s in args.legs.split(",") if s and s != "none"]
    with_oracle = not args.no_cpu_baseline

    # ---- headline: the 4M ring in FP64 at the order that reaches 1e-6
    cfg = workloads.CONFIGS["ring4m_fp32"]
    n, mx, lmax = cfg["n"], cfg["max_per_leaf"], 8
    x, w = workloads.vortex_ring(n, cfg["seed"])
    a = workloads.core_radius(n)
    p = args.p
    log(f"bench: headline ring N={n} FP64 p={p} adaptive <= {mx}/leaf, level <= {lmax}")
    head, st, (vh, sh) = run_leg(lhf, torch, f"ring4m_fp64_p{p}", x, w, a, p, lhf.FP64, lmax, mx, args.steps,
                                 args.warmup, tune=not args.no_tune)
    ph = head["phases_ms"]
    launches = sum(1 for l in range(2, len(st["boxes"])) if st["boxes"][l] > 0)
    flops = st["n_m2l"] * f_m2l(p)
    achieved = flops / (ph["m2l"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": head["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ring4m_fp64_p{p}", "n": n, "p": p, "max_per_leaf": mx, "max_level": lmax,
                   "precision": "fp64",
                   "distribution": ("vortex ring R0 = 0.3 (Gaussian cross-section, density ~ exp(-rho^2/0.05^2)) "
                                    "+ 10% uniform background, omega = exp(-rho^2/0.05^2) e_theta, "
                                    "Gaussian core a = 0.5 N^(-1/3)"),
                   "step": "plan (keys, sort, octree, lists, tables) + execute (P2M, M2M, M2L/L2L, L2P, P2P)"},
        "execute_ms": head["execute_ms"],
        "plan_ms": head["plan_ms"],
        "execute_only_elements_per_s": head["execute_only_elements_per_s"],
        "phases_ms": ph,
        "counts": head["counts"],
        "m2l_kernel": head["m2l_kernel"],
        "phase_roofline": head["phase_roofline"],
        "aggregate_roofline": head["aggregate_roofline"],
        "roofline": {
            "kernel": KERNEL_LABEL.get(head["m2l_kernel"], head["m2l_kernel"]).format(t="double", p=p),
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(f"ring4m_fp64_p{p}"),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "launches_per_step": launches,
            "avg_launch_ms": ph["m2l"] / launches,
            "flop_per_launch": flops / launches,
            "flop_per_m2l": f_m2l(p),
        },
    }
    # ---- legs
    outs = {}
    if "ring16" in legs:
        ring = {}
        for prec, nm in ((lhf.FP32, "fp32"), (lhf.FP64, "fp64")):
            r, _, o = run_leg(lhf, torch, f"ring4m_{nm}_p16", x, w, a, 16, prec, lmax, mx, args.leg_steps,
                              args.warmup, tune=not args.no_tune)
            ring[nm] = r
            outs[nm] = o
        ring["speedup_fp32_vs_fp64"] = ring["fp64"]["ms_per_step"] / ring["fp32"]["ms_per_step"]
        ring["speedup_fp32_p16_vs_fp64_headline"] = head["ms_per_step"] / ring["fp32"]["ms_per_step"]
        out["ring_p16"] = ring
    if "wx" in legs:
        # the ring at p = 16 in FP64 with the W/X lists by M2P / P2L instead of direct sums
        r, _, _ = run_leg(lhf, torch, "ring4m_fp64_p16_wx_expansions", x, w, a, 16, lhf.FP64, lmax, mx,
                          max(1, args.leg_steps // 4), args.warmup, wx=True)
        if "ring_p16" in out:
            r["ms_vs_direct_wx"] = r["ms_per_step"] / out["ring_p16"]["fp64"]["ms_per_step"]
        out["ring_p16_wx"] = r
    if "scalar" in legs:
        # the paper's comparison (Sec. 5.2): the scalar harmonic FMM (potential and gradient of
        # sources) on the 2^20 cube against the vortex FMM (v and s) on the same tree and p
        sc = {}
        for wl in ("cube1m_fp64", "cube1m_fp32"):
            c = workloads.make(wl)
            prec = lhf.FP64 if c["precision"] == "fp64" else lhf.FP32
            qv = np.random.default_rng(c["seed"] + 100).normal(size=c["n"])
            r, _, _ = run_leg(lhf, torch, wl + "_scalar", c["x"], c["w"], 0.0, c["p"], prec, c["depth"], 0,
                              args.leg_steps, args.warmup, q=qv)
            rv, _, _ = run_leg(lhf, torch, wl, c["x"], c["w"], c["a"], c["p"], prec, c["depth"], 0,
                               args.leg_steps, args.warmup)
            r["vortex_ms_per_step"] = rv["ms_per_step"]
            r["vortex_execute_ms"] = rv["execute_ms"]
            r["ratio_vortex_to_scalar_execute"] = rv["execute_ms"] / r["execute_ms"]
            r["ratio_vortex_to_scalar_m2l"] = rv["phases_ms"]["m2l"] / r["phases_ms"]["m2l"]
            sc[wl] = r
        out["scalar_vs_vortex"] = sc
    if "filament" in legs:
        out["filament"] = run_filament(lhf, torch, max(1, args.leg_steps // 4), args.warmup)
    if "cube" in legs:
        cube = {}
        for wl in ("cube1m_fp64", "cube1m_fp32"):
            c = workloads.make(wl)
            prec = lhf.FP64 if c["precision"] == "fp64" else lhf.FP32
            r, _, o = run_leg(lhf, torch, wl, c["x"], c["w"], c["a"], c["p"], prec, c["depth"], 0, args.leg_steps,
                              args.warmup)
            cube[wl] = r
            outs[wl] = (o, c)
        cube["speedup_fp32_p10_vs_fp64_p12"] = cube["cube1m_fp64"]["ms_per_step"] / cube["cube1m_fp32"]["ms_per_step"]
        out["cube1m"] = cube
    if "batch" in legs:
        out["batch"] = run_batch(lhf, torch, args.leg_steps, args.warmup, with_oracle)
    # ---- oracle legs: accuracy against the split direct sum, CPU baseline
    if with_oracle:
        import oracle
        log(f"bench: accuracy of the headline on {args.targets} targets (oracle adaptive direct sum) ...")
        tg = workloads.sample_targets(n, args.targets, seed=3000)
        vd, sd = oracle.direct_adaptive(x, w, a, mx, lmax, targets=tg)
        acc = rel_err(vh, sh, tg, vd, sd)
        acc.update(targets=int(len(tg)), meets_1e_6=bool(acc["rel_l2_v"] <= 1e-6 and acc["rel_l2_s"] <= 1e-6),
                   reference="adaptive split-kernel direct sum (Gaussian core between adjacent leaves, singular "
                             "beyond), FP64 oracle")
        out["accuracy"] = acc
        if "ring_p16" in out:
            out["ring_p16"]["fp64"]["accuracy"] = rel_err(*outs["fp64"], tg, vd, sd)
            tg32 = tg[:1024]
            xr, wr = x.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64)
            vd32, sd32 = oracle.direct_adaptive(xr, wr, float(np.float32(a)), mx, lmax, targets=tg32)
            out["ring_p16"]["fp32"]["accuracy"] = dict(
                rel_err(*outs["fp32"], tg32, vd32, sd32), targets=int(len(tg32)),
                reference="same direct sum on the FP32-rounded inputs")
        if "cube1m" in out:
            for wl in ("cube1m_fp64", "cube1m_fp32"):
                (vv, ss), c = outs[wl]
                xc, wc, ac = c["x"], c["w"], c["a"]
                if c["precision"] == "fp32":
                    xc, wc = xc.astype(np.float32).astype(np.float64), wc.astype(np.float32).astype(np.float64)
                    ac = float(np.float32(ac))
                tgc = workloads.sample_targets(xc.shape[0], 1000, seed=1000)
                vdc, sdc = oracle.direct(xc, wc, ac, mode=oracle.DIRECT_SPLIT, depth=c["depth"], targets=tgc)
                out["cube1m"][wl]["accuracy"] = dict(rel_err(vv, ss, tgc, vdc, sdc), targets=1000)
        log("bench: CPU oracle baseline (sampled, projected) ...")
        out["cpu_baseline"] = cpu_baseline(x, w, a, p, mx, lmax, st)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
