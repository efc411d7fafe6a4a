"""GPU parity of the adaptive-octree path against the oracle's adaptive FMM.

Bar: FP64 relative L2 of v and s <= 1e-12 (same tree, same lists, same p);
tree and list counts equal the oracle's exactly; FP32 <= 2e-6 against the FP64
oracle on the FP32-rounded inputs.  W/X interactions are direct sums with the
singular kernel on both sides.
"""
import numpy as np
import pytest

import workloads
from parity_util import check, check32

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _cluster(n, seed, sigma=0.02):
    rng = np.random.default_rng(seed)
    nc = int(0.8 * n)
    xc = np.clip(rng.normal(0.3, sigma, (nc, 3)), 0, 1 - 1e-12)
    xb = rng.uniform(0, 1, (n - nc, 3))
    return np.concatenate([xc, xb]), rng.normal(size=(n, 3))


def _gpu(x, w, a, p, max_per_leaf, depth, precision=0, what=3, **kw):
    torch = _torch()
    import paper_1201_5430_amd as LH
    dt = torch.float64 if precision == 0 else torch.float32
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(device="cuda", dtype=dt)
    plan = LH.Plan(xt, a, p=p, depth=depth, precision=precision, max_per_leaf=max_per_leaf, **kw)
    v, s = plan.execute(wt, what=what)
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    return v.double().cpu().numpy(), s.double().cpu().numpy(), st


def _check_counts(oracle, x, st, ost, mx, depth):
    nb, nl = oracle.adaptive_counts(x, mx, depth)
    assert list(st["boxes"]) == list(nb)
    assert st["n_leaves"] == nl.sum() == ost["n_leaf"]
    assert st["max_level"] == ost["max_level"]
    assert st["n_m2l"] == ost["n_m2l"]
    assert st["n_p2p_pairs"] == ost["n_p2p_pairs"]
    assert st["n_wx_pairs"] == ost["n_wx_pairs"]


@pytest.mark.parametrize("p", [8, 12])
def test_ring_fp64_matches_oracle(oracle, p):
    x, w = workloads.vortex_ring(6000, 41)
    a = workloads.core_radius(6000)
    mx, depth = 16, 7
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, p, mx, depth)
    v, s, st = _gpu(x, w, a, p, mx, depth)
    _check_counts(oracle, x, st, ost, mx, depth)
    ev, es = _rel(v, vr), _rel(s, sr)
    print(f"ring p={p}: rel L2 v {ev:.3e} s {es:.3e}, W/X pairs {st['n_wx_pairs']}", flush=True)
    assert ev <= 1e-12 and es <= 1e-12


@pytest.mark.parametrize("what", [1, 2])
def test_far_and_near_parts(oracle, what):
    x, w = _cluster(4000, 42)
    a = 0.004
    mx, depth = 8, 8
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, 8, mx, depth, far=bool(what & 1), near=bool(what & 2))
    v, s, st = _gpu(x, w, a, 8, mx, depth, what=what)
    ev, es = _rel(v, vr), _rel(s, sr)
    print(f"cluster what={what}: rel L2 v {ev:.3e} s {es:.3e}", flush=True)
    assert ev <= 1e-12 and es <= 1e-12


def test_deep_unbalanced_tree_generic_m2l(oracle):
    # deepest level 10: beyond the dense box maps of the batched M2L, the per-box V-list path runs
    x, w = _cluster(3000, 43, sigma=0.005)
    a = 0.0005
    mx, depth = 8, 10
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, 6, mx, depth)
    v, s, st = _gpu(x, w, a, 6, mx, depth)
    _check_counts(oracle, x, st, ost, mx, depth)
    assert st["max_level"] == 10
    ev, es = _rel(v, vr), _rel(s, sr)
    print(f"deep cluster: rel L2 v {ev:.3e} s {es:.3e}", flush=True)
    assert ev <= 1e-12 and es <= 1e-12


def test_tiled_and_generic_m2l_agree():
    import paper_1201_5430_amd as LH
    x, w = workloads.vortex_ring(8000, 44)
    a = workloads.core_radius(8000)
    v1, s1, _ = _gpu(x, w, a, 10, 32, 7)
    v2, s2, st = _gpu(x, w, a, 10, 32, 7, m2l_kernel=LH.M2L_GENERIC)
    assert st["m2l_kernel"] == "generic"
    check(v1, s1, v2, s2, l2=1e-13, mx=1e-12)


@pytest.mark.parametrize("n,mx", [(50, 64), (300, 64), (700, 100)])
def test_shallow_trees(oracle, n, mx):
    # the root is a leaf (all pairs direct, smoothed) or leaves sit on levels 1 and 2
    rng = np.random.default_rng(45 + n)
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.05
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, 8, mx, 6)
    v, s, st = _gpu(x, w, a, 8, mx, 6)
    _check_counts(oracle, x, st, ost, mx, 6)
    if n <= mx:
        vd, sd = oracle.direct(x, w, a, mode=oracle.DIRECT_SMOOTH)
        assert _rel(v, vd) <= 1e-13 and _rel(s, sd) <= 1e-13
    assert _rel(v, vr) <= 1e-12 and _rel(s, sr) <= 1e-12


def test_fp32_p16_ring(oracle):
    n = 40000
    x, w = workloads.vortex_ring(n, 46)
    x = x.astype(np.float32).astype(np.float64)
    w = w.astype(np.float32).astype(np.float64)
    a = float(np.float32(workloads.core_radius(n)))
    samp = np.random.default_rng(46).choice(n, 30, replace=False)
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, 16, 64, 8, sample=samp)
    m = ~np.isnan(vr[:, 0])
    v, s, st = _gpu(x, w, a, 16, 64, 8, precision=1)
    check32(v[m], s[m], vr[m], sr[m], label="ring FP32 p=16 sampled:")


def test_ring4m_full_size_sampled(oracle):
    # the full clustered workload (4,194,304 elements, <= 64 per leaf, deepest level 8) in FP32,
    # checked on the leaves of 20 seeded elements against the FP64 oracle at p = 8.
    # Bar 5e-6: the far-field stretching of ring targets sums ~190 M2L contributions per box
    # and level whose magnitudes exceed their sum ~30-fold, so FP32 rounding (6e-8) reaches
    # ~2e-6 there (measured: far field alone 1.8e-6, near field 7e-7); still 20x below the
    # p = 8 truncation error (~1e-4).
    cfg = workloads.CONFIGS["ring4m_fp32"]
    x, w = workloads.vortex_ring(cfg["n"], cfg["seed"])
    x = x.astype(np.float32).astype(np.float64)
    w = w.astype(np.float32).astype(np.float64)
    a = float(np.float32(workloads.core_radius(cfg["n"])))
    samp = workloads.sample_targets(cfg["n"], 20, seed=5)
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, 8, cfg["max_per_leaf"], 8, sample=samp)
    m = ~np.isnan(vr[:, 0])
    v, s, st = _gpu(x, w, a, 8, cfg["max_per_leaf"], 8, precision=1)
    assert st["n_leaves"] == ost["n_leaf"] and st["max_level"] == ost["max_level"]
    check32(v[m], s[m], vr[m], sr[m], l2=5e-6, mx=2e-5, label=f"ring4m FP32 p=8 sampled ({m.sum()} elements):")


def test_ring4m_p16_full_size_sampled(oracle):
    # the clustered workload at its own order p = 16: 4,194,304 elements, <= 64 per leaf,
    # deepest level 8, both precisions on the same (FP32-rounded) input, checked on the leaves of
    # 24 seeded elements against the oracle's adaptive FMM at p = 16.  FP64 bar 1e-11 (as for the
    # 2^20 cube); FP32 bar 5e-6 in L2 as at p = 8 (FP32 rounding of the far-field stretching
    # sums, which cancel ~30-fold on ring targets)
    cfg = workloads.CONFIGS["ring4m_fp32"]
    x, w = workloads.vortex_ring(cfg["n"], cfg["seed"])
    x = x.astype(np.float32).astype(np.float64)
    w = w.astype(np.float32).astype(np.float64)
    a = float(np.float32(workloads.core_radius(cfg["n"])))
    mx, p = cfg["max_per_leaf"], cfg["p"]
    v64, s64, st = _gpu(x, w, a, p, mx, 8, precision=0)
    v32, s32, _ = _gpu(x, w, a, p, mx, 8, precision=1)
    samp = workloads.sample_targets(cfg["n"], 24, seed=5)
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, p, mx, 8, sample=samp)
    m = ~np.isnan(vr[:, 0])
    assert m.sum() >= 24
    assert st["n_leaves"] == ost["n_leaf"] and st["max_level"] == ost["max_level"]
    check(v64[m], s64[m], vr[m], sr[m], l2=1e-11, mx=1e-10, label=f"ring4m FP64 p=16 ({m.sum()} elements):")
    check32(v32[m], s32[m], vr[m], sr[m], l2=5e-6, mx=2e-5, label=f"ring4m FP32 p=16 ({m.sum()} elements):")


def test_ring4m_p23_full_size_sampled(oracle):
    # the headline configuration as the benchmark times it: the full clustered workload (4,194,304
    # elements, <= 64 per leaf, deepest level 8) in FP64 at p = 23 (the quarter-vector M2L and
    # M2M/L2L), with the run-time shapes the autotuner picks for it, checked on the leaves of 24
    # seeded elements against the oracle's adaptive FMM at p = 23.  Bar 1e-11 / 1e-10 as for the
    # other full-size FP64 comparisons (the sampled targets sum over every level of the tree)
    torch = _torch()
    import paper_1201_5430_amd as LH
    cfg = workloads.CONFIGS["ring4m_fp32"]
    x, w = workloads.vortex_ring(cfg["n"], cfg["seed"])
    a = workloads.core_radius(cfg["n"])
    mx, p = cfg["max_per_leaf"], 23
    xt = torch.from_numpy(x).to(device="cuda", dtype=torch.float64)
    wt = torch.from_numpy(w).to(device="cuda", dtype=torch.float64)
    plan = LH.Plan(xt, a, p=p, depth=8, precision=LH.FP64, max_per_leaf=mx)
    shapes = plan.autotune(wt)
    plan.close()
    plan = LH.Plan(xt, a, p=p, depth=8, precision=LH.FP64, max_per_leaf=mx)
    plan.set_shapes(shapes)
    v, s = plan.execute(wt)
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    assert st["m2l_kernel"] == "quarter"
    v, s = v.cpu().numpy(), s.cpu().numpy()
    samp = workloads.sample_targets(cfg["n"], 24, seed=7)
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, p, mx, 8, sample=samp)
    m = ~np.isnan(vr[:, 0])
    assert m.sum() >= 24
    assert st["n_leaves"] == ost["n_leaf"] and st["max_level"] == ost["max_level"]
    check(v[m], s[m], vr[m], sr[m], l2=1e-11, mx=1e-10,
          label=f"ring4m FP64 p=23, tuned shapes {shapes} ({m.sum()} elements):")
