"""GPU parity of the W/X treatment by expansions (LHF_WX_EXPANSIONS) against the oracle.

With the flag, an adaptive plan moves the W-list boxes of a leaf (levels >= 2) from the
singular direct sum to M2P of their multipoles at the leaf's elements, and the X sources of
the leaf and of its ancestors to P2L into the leaf's local expansion (App. A, eqs. dt3 and
drt4-drt7 restated in the scaled real basis).  The oracle's adaptive FMM with
``wx_expansions=True`` does the same by composing its pinned operators (P2M about the element,
M2L with the R conversion, L2P), so the two agree to rounding: FP64 bar 1e-12 relative L2 and
1e-11 element-wise; FP32 against the FP64 oracle on FP32-rounded inputs 2e-6 / 1e-5.
Counts: the near-field U pairs are unchanged, the direct W/X pairs are those the oracle still
sums directly.
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


def _cluster(n, seed, sigma=0.02):
    rng = np.random.default_rng(seed)
    nc = int(0.8 * n)
    xc = np.clip(rng.normal(0.3, sigma, (nc, 3)), 0, 1 - 1e-12)
    xb = rng.uniform(0, 1, (n - nc, 3))
    return np.concatenate([xc, xb]), rng.normal(size=(n, 3))


def _gpu(x, w, a, p, max_per_leaf, depth, precision=0, what=3, q=None, grad=False, wx=True, **kw):
    torch = _torch()
    import paper_1201_5430_amd as LH
    dt = torch.float64 if precision == 0 else torch.float32
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(device="cuda", dtype=dt)
    qt = None if q is None else torch.from_numpy(np.ascontiguousarray(q)).to(device="cuda", dtype=dt)
    print(f"wx plan: n={x.shape[0]} p={p} max_per_leaf={max_per_leaf} depth={depth} prec={precision} "
          f"what={what} q={q is not None} grad={grad}", flush=True)
    plan = LH.Plan(xt, a, p=p, depth=depth, precision=precision, max_per_leaf=max_per_leaf, grad=grad,
                   wx_expansions=wx, **kw)
    out = plan.execute(wt, what=what, q=qt, grad=grad)
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    return [o.double().cpu().numpy() for o in out] + [st]


def _counts(st, ost, near=True, far=True):
    # the oracle counts translations only when it runs the far field, pairs only with the near field
    assert st["wx_expansions"]
    assert st["n_leaves"] == ost["n_leaf"] and st["max_level"] == ost["max_level"]
    if far:
        assert st["n_m2l"] == ost["n_m2l"]
    if near:
        assert st["n_p2p_pairs"] == ost["n_p2p_pairs"]
        assert st["n_wx_pairs"] == ost["n_wx_pairs"]


@pytest.mark.parametrize("p", [8, 12, 16])
def test_ring_wx_expansions_fp64(oracle, p):
    x, w = workloads.vortex_ring(6000, 41)
    a = workloads.core_radius(6000)
    mx, depth = 16, 7
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, p, mx, depth, wx_expansions=True)
    v, s, st = _gpu(x, w, a, p, mx, depth)
    _counts(st, ost)
    assert st["n_m2p"] > 0 and st["n_p2l"] > 0
    check(v, s, vr, sr, label=f"ring W/X by expansions p={p} (M2P pairs {st['n_m2p']}, P2L pairs {st['n_p2l']}):")


@pytest.mark.parametrize("what", [1, 2, 3])
def test_cluster_wx_monopoles_and_gradient(oracle, what):
    # far part (M2P and P2L included), near part (U only), whole field; sources and grad v
    x, w = _cluster(4000, 42)
    q = np.random.default_rng(42).normal(size=4000)
    a = 0.004
    mx, depth = 8, 8
    vr, sr, gr, ost = oracle.fmm_adaptive(x, w, a, 10, mx, depth, far=bool(what & 1), near=bool(what & 2),
                                          grad=True, q=q, wx_expansions=True)
    v, s, g, st = _gpu(x, w, a, 10, mx, depth, what=what, q=q, grad=True)
    _counts(st, ost, near=bool(what & 2), far=bool(what & 1))
    check(v, s, vr, sr, label=f"cluster W/X what={what} v, s:")
    check(g.reshape(-1, 9), g.reshape(-1, 9), gr.reshape(-1, 9), gr.reshape(-1, 9), label="  grad v:")


def test_deep_tree_wx(oracle):
    # deepest level 10 (the per-box M2L path) with W boxes many levels below their leaves
    x, w = _cluster(3000, 43, sigma=0.005)
    a = 0.0005
    mx, depth = 8, 10
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, 8, mx, depth, wx_expansions=True)
    v, s, st = _gpu(x, w, a, 8, mx, depth)
    _counts(st, ost)
    check(v, s, vr, sr, label="deep cluster W/X:")


@pytest.mark.parametrize("p", [8, 12])
def test_ring_wx_expansions_fp32(oracle, p):
    n = 10000
    x, w = workloads.vortex_ring(n, 47)
    x = x.astype(np.float32).astype(np.float64)
    w = w.astype(np.float32).astype(np.float64)
    a = float(np.float32(workloads.core_radius(n)))
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, p, 32, 8, wx_expansions=True)
    v, s, st = _gpu(x, w, a, p, 32, 8, precision=1)
    _counts(st, ost)
    check32(v, s, vr, sr, label=f"ring FP32 W/X p={p}:")


def test_wx_modes_differ_by_truncation_only():
    # the two W/X treatments on the GPU: identical U pairs, results within the truncation error
    x, w = workloads.vortex_ring(20000, 48)
    a = workloads.core_radius(20000)
    v0, s0, st0 = _gpu(x, w, a, 16, 32, 8, wx=False)
    v1, s1, st1 = _gpu(x, w, a, 16, 32, 8, wx=True)
    assert not st0["wx_expansions"] and st0["n_m2p"] == 0 and st0["n_p2l"] == 0
    assert st1["n_p2p_pairs"] == st0["n_p2p_pairs"] and st1["n_wx_pairs"] < st0["n_wx_pairs"]
    ev = np.linalg.norm(v1 - v0) / np.linalg.norm(v0)
    es = np.linalg.norm(s1 - s0) / np.linalg.norm(s0)
    print(f"W/X by expansions vs direct, p = 16: rel L2 v {ev:.3e} s {es:.3e}", flush=True)
    # the ring's whole-method error at p = 16 is 3.9e-8 (v) and 1.9e-5 (s) (error-vs-p sweep)
    assert 0 < ev < 1e-6 and 0 < es < 1e-4


def test_uniform_tree_ignores_the_flag(oracle):
    x, w = workloads.uniform_cube(3000, 49)
    a = workloads.core_radius(3000)
    vr, sr = oracle.fmm(x, w, a, 8, 3)[:2]
    v, s, st = _gpu(x, w, a, 8, 0, 3)
    assert not st["wx_expansions"] and st["n_m2p"] == 0
    check(v, s, vr, sr, label="uniform tree with the W/X flag:")


def test_ring4m_wx_full_size_sampled(oracle):
    # the full clustered workload (4,194,304 elements, <= 64 per leaf, level 8) with W/X by
    # expansions at p = 16 in FP64, on the leaves of 16 seeded elements
    cfg = workloads.CONFIGS["ring4m_fp32"]
    x, w = workloads.vortex_ring(cfg["n"], cfg["seed"])
    a = workloads.core_radius(cfg["n"])
    mx = cfg["max_per_leaf"]
    v, s, st = _gpu(x, w, a, 16, mx, 8)
    samp = workloads.sample_targets(cfg["n"], 16, seed=6)
    vr, sr, ost = oracle.fmm_adaptive(x, w, a, 16, mx, 8, sample=samp, wx_expansions=True)
    m = ~np.isnan(vr[:, 0])
    assert m.sum() >= 16
    assert st["n_leaves"] == ost["n_leaf"] and st["max_level"] == ost["max_level"]
    print(f"ring4m W/X: M2P pairs {st['n_m2p']}, P2L pairs {st['n_p2l']}, direct W/X pairs {st['n_wx_pairs']}",
          flush=True)
    check(v[m], s[m], vr[m], sr[m], l2=1e-11, mx=1e-10, label=f"ring4m FP64 p=16 W/X ({m.sum()} elements):")
