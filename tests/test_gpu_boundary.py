"""GPU tests of the boundary's options: the velocity-gradient output, the order
chosen from a tolerance, the deterministic mode and the checks on caller outputs.

grad v is compared element by element with the oracle's FMM gradient (the same
bars as v and s: FP64 1e-12 relative L2 and 1e-11 element-wise; FP32 against
the FP64 oracle on the FP32-rounded inputs 2e-6 / 1e-5).  The order chosen from
tol is the smallest order whose calibrated error reaches tol, and the field it
gives meets tol against the oracle's split-kernel direct sum.
"""
import numpy as np
import pytest

import workloads
from parity_util import check, check32, rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _dev(x, precision):
    torch = _torch()
    dt = torch.float64 if precision == 0 else torch.float32
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


def _host(*ts):
    return [t.double().cpu().numpy() for t in ts]


@pytest.mark.parametrize("prec,p,depth,n", [(0, 8, 3, 6000), (0, 12, 4, 20000), (1, 10, 4, 20000)])
def test_grad_uniform_matches_oracle(oracle, prec, p, depth, n):
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(500 + p)
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    if prec:
        x, w, a = x.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64), float(np.float32(a))
    plan = L.Plan(_dev(x, prec), a, p=p, depth=depth, precision=prec, grad=True)
    v, s, g = plan.execute(_dev(w, prec), grad=True)
    v2, s2 = plan.execute(_dev(w, prec))  # the same plan without the gradient
    _torch().cuda.synchronize()
    plan.close()
    v, s, g, v2, s2 = _host(v, s, g, v2, s2)
    vr, sr, gr, _ = oracle.fmm(x, w, a, p, depth, grad=True)
    chk = check if prec == 0 else check32
    chk(v, s, vr, sr, label=f"grad plan prec={prec} p={p} v, s:")
    chk(g, g, gr, gr, label=f"grad prec={prec} p={p} grad v:")
    if prec == 0:
        check(v, s, v2, s2, l2=1e-13, mx=1e-12, label="with vs without grad:")
    else:
        check32(v, s, v2, s2, label="with vs without grad:")
    # s_k = sum_l omega_l d_l v_k holds in the library's own outputs
    bar = 1e-12 if prec == 0 else 2e-6
    assert rel(np.einsum("ikl,il->ik", g, w), s) < bar


@pytest.mark.parametrize("prec", [0, 1])
def test_grad_adaptive_matches_oracle(oracle, prec):
    import paper_1201_5430_amd as L
    n = 12000
    x, w = workloads.vortex_ring(n, 501)
    a = workloads.core_radius(n)
    if prec:
        x, w, a = x.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64), float(np.float32(a))
    plan = L.Plan(_dev(x, prec), a, p=10, depth=7, precision=prec, max_per_leaf=24, grad=True)
    v, s, g = plan.execute(_dev(w, prec), grad=True)
    _torch().cuda.synchronize()
    st = plan.stats()
    plan.close()
    v, s, g = _host(v, s, g)
    vr, sr, gr, ost = oracle.fmm_adaptive(x, w, a, 10, 24, 7, grad=True)
    assert st["n_wx_pairs"] == ost["n_wx_pairs"] > 0
    chk = check if prec == 0 else check32
    chk(v, s, vr, sr, label=f"adaptive grad plan prec={prec} v, s:")
    chk(g, g, gr, gr, label=f"adaptive prec={prec} grad v:")


def test_grad_needs_the_flag():
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(502)
    x, w = rng.uniform(0, 1, (500, 3)), rng.normal(size=(500, 3))
    plan = L.Plan(_dev(x, 0), 0.05, p=6, depth=3)
    with pytest.raises(L.LhfError) as e:
        plan.execute(_dev(w, 0), grad=True)
    assert e.value.status == -7
    plan.close()


def test_output_tensors_are_checked():
    torch = _torch()
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(503)
    x, w = rng.uniform(0, 1, (400, 3)), rng.normal(size=(400, 3))
    plan = L.Plan(_dev(x, 0), 0.05, p=6, depth=3)
    wt = _dev(w, 0)
    with pytest.raises(TypeError):
        plan.execute(wt, v=torch.empty(400, 3, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        plan.execute(wt, s=torch.empty(399, 3, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        plan.execute(wt, v=torch.empty(400, 3, dtype=torch.float64))
    with pytest.raises(TypeError):
        plan.execute(wt, v=torch.empty(3, 400, dtype=torch.float64, device="cuda").t())
    plan.close()


def test_order_from_tolerance(oracle):
    # p = 0: the smallest order whose calibrated error (uniform class) reaches tol; the field
    # then meets tol against the split direct sum on the same class of input
    import paper_1201_5430_amd as L
    n, depth = 16384, 4
    x, w = workloads.uniform_cube(n, 504)
    a = workloads.core_radius(n)
    tg = workloads.sample_targets(n, 512, seed=505)
    vd, sd = oracle.direct(x, w, a, mode=oracle.DIRECT_SPLIT, depth=depth, targets=tg)
    for tol in (1e-3, 1e-4, 1e-6):
        plan = L.Plan(_dev(x, 0), a, p=0, depth=depth, tol=tol)
        v, s = plan.execute(_dev(w, 0))
        _torch().cuda.synchronize()
        st = plan.stats()
        plan.close()
        assert st["p_from_tol"] and not plan.warn_tol_unmet
        assert max(st["calib_err_v"], st["calib_err_s"]) <= tol
        # one order less would not have met tol by the table
        lower = L.Plan(_dev(x[:64], 0), a, p=st["p"] - 1, depth=2, tol=tol).stats()
        assert max(lower["calib_err_v"], lower["calib_err_s"]) > tol
        v, s = _host(v, s)
        ev, es = rel(v[tg], vd), rel(s[tg], sd)
        print(f"tol {tol:.0e}: p = {st['p']}, eps2 v {ev:.2e} s {es:.2e}", flush=True)
        assert ev <= 2 * tol and es <= 2 * tol
    # unreachable tolerances: the largest order and a warning
    plan = L.Plan(_dev(x, 0), a, p=0, depth=depth, tol=1e-13)
    assert plan.warn_tol_unmet and plan.stats()["p"] == 24
    plan.close()
    plan = L.Plan(_dev(x, 1), a, p=0, depth=depth, tol=1e-7, precision=L.FP32)
    assert plan.warn_tol_unmet and plan.stats()["p"] == 16
    plan.close()


@pytest.mark.parametrize("prec,p,kernel", [(0, 12, "mfma"), (1, 16, "mfma"), (0, 16, "generic"), (1, 10, "half")])
def test_deterministic_mode(oracle, prec, p, kernel):
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(510 + p + prec)
    n = 20000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    if prec:
        x, w, a = x.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64), float(np.float32(a))
    xt, wt = _dev(x, prec), _dev(w, prec)
    plan = L.Plan(xt, a, p=p, depth=4, precision=prec, deterministic=True)
    st = plan.stats()
    assert st["deterministic"] and st["m2l_kernel"] == kernel
    v1, s1 = plan.execute(wt)
    v2, s2 = plan.execute(wt)
    _torch().cuda.synchronize()
    plan.close()
    plan = L.Plan(xt, a, p=p, depth=4, precision=prec, deterministic=True)
    v3, s3 = plan.execute(wt)
    _torch().cuda.synchronize()
    plan.close()
    v1, s1, v2, s2, v3, s3 = _host(v1, s1, v2, s2, v3, s3)
    assert np.array_equal(v1, v2) and np.array_equal(s1, s2)
    assert np.array_equal(v1, v3) and np.array_equal(s1, s3)
    samp = rng.choice(n, 30, replace=False)
    vr, sr, _ = oracle.fmm(x, w, a, p, 4, sample=samp)
    m = ~np.isnan(vr[:, 0])
    (check if prec == 0 else check32)(v1[m], s1[m], vr[m], sr[m], label=f"deterministic {kernel} p={p}:")


def test_kernel_requests():
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(520)
    xt = _dev(rng.uniform(0, 1, (2000, 3)), 0)
    st = L.Plan(xt, 0.02, p=12, depth=3).stats()
    assert st["m2l_kernel"] == "half" and st["mm_kernel"] == "half" and not st["deterministic"]
    st = L.Plan(xt, 0.02, p=16, depth=3).stats()
    assert st["m2l_kernel"] == "quarter" and st["mm_kernel"] == "half"
    st = L.Plan(xt, 0.02, p=23, depth=3).stats()
    assert st["m2l_kernel"] == "quarter" and st["mm_kernel"] == "quarter"
    st = L.Plan(xt, 0.02, p=6, depth=3).stats()
    assert st["m2l_kernel"] == "tile" and st["mm_kernel"] == "generic" and st["deterministic"]
    st = L.Plan(xt, 0.02, p=7, depth=3).stats()
    assert st["m2l_kernel"] == "generic"
    for kw in (dict(p=6, m2l_kernel=L.M2L_HALF), dict(p=16, m2l_kernel=L.M2L_TILE),
               dict(p=12, m2l_kernel=L.M2L_HALF, deterministic=True), dict(p=6, mm_kernel=L.MM_HALF)):
        with pytest.raises(L.LhfError) as e:
            L.Plan(xt, 0.02, depth=3, **kw)
        assert e.value.status == -6, kw


@pytest.mark.parametrize("prec,adaptive", [(0, False), (0, True), (1, False)])
def test_monopoles_and_beta_match_oracle(oracle, prec, adaptive):
    # divergence sources q (eqs. 5-7): v, s, grad v with the monopole terms, and
    # beta = grad v : grad v, against the oracle's FMM with the same sources
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(530 + prec + 2 * adaptive)
    if adaptive:
        n = 12000
        x, w = workloads.vortex_ring(n, 531)
    else:
        n = 20000
        x, w = rng.uniform(0, 1, (n, 3)), rng.normal(size=(n, 3))
    q = rng.normal(size=n)
    a = workloads.core_radius(n)
    if prec:
        x, w, q = (t.astype(np.float32).astype(np.float64) for t in (x, w, q))
        a = float(np.float32(a))
    kw = dict(max_per_leaf=24, depth=7) if adaptive else dict(depth=4)
    plan = L.Plan(_dev(x, prec), a, p=12, precision=prec, grad=True, **kw)
    qt = _dev(q[:, None], prec)[:, 0].contiguous()
    v, s, g, b = plan.execute(_dev(w, prec), q=qt, grad=True, beta=True)
    v0, s0 = plan.execute(_dev(w, prec))  # the same plan without sources
    _torch().cuda.synchronize()
    plan.close()
    v, s, g, b, v0 = _host(v, s, g, b, v0)
    if adaptive:
        vr, sr, gr, _ = oracle.fmm_adaptive(x, w, a, 12, 24, 7, grad=True, q=q)
    else:
        vr, sr, gr, _ = oracle.fmm(x, w, a, 12, 4, grad=True, q=q)
    chk = check if prec == 0 else check32
    chk(v, s, vr, sr, label=f"monopoles prec={prec} adaptive={adaptive} v, s:")
    chk(g, g, gr, gr, label="  grad v:")
    br = (gr ** 2).sum(axis=(1, 2))
    chk(b, b, br, br, label="  beta:")
    assert rel(v0, v) > 1e-2  # the sources do change the field


def test_io_state_errors():
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(540)
    x, w = rng.uniform(0, 1, (500, 3)), rng.normal(size=(500, 3))
    plan = L.Plan(_dev(x, 0), 0.05, p=6, depth=3)
    with pytest.raises(L.LhfError) as e:
        plan.execute(_dev(w, 0), beta=True)
    assert e.value.status == -7
    with pytest.raises(TypeError):
        plan.execute(_dev(w, 0), q=_dev(np.zeros((500, 1)), 0))
    plan.close()
