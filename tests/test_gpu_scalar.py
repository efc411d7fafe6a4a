"""GPU parity of the scalar harmonic FMM (lhf_execute_scalar) against the oracle's.

Sources q at the plan's elements, Phi_j = sum_{i != j} q_i / r_ij and grad Phi with the singular
kernel, on the plan's uniform tree at its p.  FP64 bar 1e-12 relative L2 and 1e-11 element-wise
(as for the vortex path); FP32 against the FP64 oracle on FP32-rounded inputs 2e-6 / 1e-5.  The
half-vector M2L translates phi alone at p = 8, 10, 12, 16; the other kernels run on (phi, chi = 0)
and must agree with it.
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


def _scalar(x, q, p, depth, precision=0, **kw):
    torch = _torch()
    import paper_1201_5430_amd as LH
    dt = torch.float64 if precision == 0 else torch.float32
    print(f"scalar plan: n={x.shape[0]} p={p} depth={depth} prec={precision} {kw}", flush=True)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)
    qt = torch.from_numpy(np.ascontiguousarray(q)).to(device="cuda", dtype=dt)
    plan = LH.Plan(xt, 0.0, p=p, depth=depth, precision=precision, **kw)
    phi, g = plan.execute_scalar(qt)
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    return phi.double().cpu().numpy(), g.double().cpu().numpy(), st


@pytest.mark.parametrize("p,depth", [(8, 4), (12, 4), (16, 3), (6, 4)])
def test_scalar_fmm_fp64(oracle, p, depth):
    x, _ = workloads.uniform_cube(20000, 61)
    q = np.random.default_rng(61).normal(size=20000)
    pr, gr, ost = oracle.fmm_scalar(x, q, p, depth)
    phi, g, st = _scalar(x, q, p, depth)
    assert st["n_m2l"] == ost["n_m2l"]
    check(phi[:, None], g, pr[:, None], gr, label=f"scalar FMM FP64 p={p} ({st['m2l_kernel']}):")


@pytest.mark.parametrize("p", [8, 10])
def test_scalar_fmm_fp32(oracle, p):
    x, _ = workloads.uniform_cube(20000, 62)
    q = np.random.default_rng(62).normal(size=20000)
    x = x.astype(np.float32).astype(np.float64)
    q = q.astype(np.float32).astype(np.float64)
    pr, gr, _ = oracle.fmm_scalar(x, q, p, 4)
    phi, g, st = _scalar(x, q, p, 4, precision=1)
    check32(phi[:, None], g, pr[:, None], gr, label=f"scalar FMM FP32 p={p} ({st['m2l_kernel']}):")


def test_scalar_kernels_agree_and_vortex_state_is_kept():
    # the scalar half-vector M2L against the generic per-box kernel on (phi, 0); a vortex execute
    # after a scalar one on the same plan gives the vortex result of a fresh plan
    torch = _torch()
    import paper_1201_5430_amd as LH
    x, w = workloads.uniform_cube(8000, 63)
    q = np.random.default_rng(63).normal(size=8000)
    a = workloads.core_radius(8000)
    p1, g1, s1 = _scalar(x, q, 12, 3)
    p2, g2, s2 = _scalar(x, q, 12, 3, m2l_kernel=LH.M2L_GENERIC)
    assert s1["m2l_kernel"] == "half" and s2["m2l_kernel"] == "generic"
    check(p1[:, None], g1, p2[:, None], g2, l2=1e-13, mx=1e-12, label="scalar half vs generic:")
    xt = torch.from_numpy(x).cuda()
    wt = torch.from_numpy(w).cuda()
    qt = torch.from_numpy(q).cuda()
    plan = LH.Plan(xt, a, p=12, depth=3)
    v0, s0 = plan.execute(wt)
    plan.execute_scalar(qt)
    v1, s1_ = plan.execute(wt)
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(v0, v1) or float((v0 - v1).abs().max()) <= 1e-14 * float(v0.abs().max())


def test_scalar_rejects_adaptive_plans():
    torch = _torch()
    import paper_1201_5430_amd as LH
    x, _ = workloads.vortex_ring(3000, 64)
    xt = torch.from_numpy(x).cuda()
    plan = LH.Plan(xt, 0.0, p=8, depth=6, max_per_leaf=32)
    with pytest.raises(LH.LhfError, match="uniform"):
        plan.execute_scalar(torch.ones(3000, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        plan.execute_scalar(torch.ones(3000, dtype=torch.float32, device="cuda"))
    plan.close()


def test_scalar_cube1m_sampled(oracle):
    # the 2^20-element uniform cube at depth 6 and p = 12 (the comparison workload of the vortex
    # cube benchmark) on the leaves of 24 seeded elements
    cfg = workloads.CONFIGS["cube1m_fp64"]
    x, _ = workloads.uniform_cube(cfg["n"], cfg["seed"])
    q = np.random.default_rng(65).normal(size=cfg["n"])
    phi, g, st = _scalar(x, q, 12, 6)
    samp = workloads.sample_targets(cfg["n"], 24, seed=7)
    pr, gr, _ = oracle.fmm_scalar(x, q, 12, 6, sample=samp)
    m = ~np.isnan(pr)
    assert m.sum() >= 24
    check(phi[m][:, None], g[m], pr[m][:, None], gr[m], l2=1e-11, mx=1e-10, label=f"scalar cube1m p=12 ({m.sum()}):")
