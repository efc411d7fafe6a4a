"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bar (FP64 path): relative L2 difference of v and of s <= 1e-12 against the
oracle's own FMM on the same tree, p and inputs; element-wise max difference
<= 1e-11 of the max magnitude.  At the full 2^20-element workload the oracle
evaluates a seeded sample of leaves (whole FMM for those leaves) and the bar
is 1e-11.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _gpu_fmm(x, w, a, p, depth, what=3, precision=0, flags=0, **kw):
    torch = _torch()
    import paper_1201_5430_amd as L
    dt = torch.float64 if precision == 0 else torch.float32
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(device="cuda", dtype=dt)
    plan = L.Plan(xt, a, p=p, depth=depth, precision=precision, flags=flags, **kw)
    v, s = plan.execute(wt, what=what)
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    return v.double().cpu().numpy(), s.double().cpu().numpy(), st


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _check(v, s, vr, sr, l2=1e-12, mx=1e-11):
    ev, es = _rel(v, vr), _rel(s, sr)
    mv = np.abs(v - vr).max() / np.abs(vr).max()
    ms = np.abs(s - sr).max() / np.abs(sr).max()
    print(f"rel L2 v {ev:.3e} s {es:.3e}  max v {mv:.3e} s {ms:.3e}", flush=True)
    assert ev <= l2 and es <= l2
    assert mv <= mx and ms <= mx


def _check32(v, s, vr, sr, l2=2e-6, mx=1e-5):
    """FP32 path against the FP64 oracle on the FP32-rounded inputs: relative L2 of v and s
    <= l2 and every element within mx of the largest reference magnitude"""
    _check(v, s, vr, sr, l2=l2, mx=mx)


def test_cube4k_fp64_matches_oracle(oracle):
    cfg = workloads.make("cube4k_fp64")
    x, w, a, p, d = cfg["x"], cfg["w"], cfg["a"], cfg["p"], cfg["depth"]
    vr, sr, ost = oracle.fmm(x, w, a, p, d)
    v, s, st = _gpu_fmm(x, w, a, p, d)
    assert st["n_m2l"] == ost["n_m2l"] and st["n_p2p_pairs"] == ost["n_p2p_pairs"]
    _check(v, s, vr, sr)


@pytest.mark.parametrize("what", [1, 2])
def test_far_and_near_parts(oracle, what):
    rng = np.random.default_rng(21)
    n = 3000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    vr, sr, _ = oracle.fmm(x, w, a, 10, 3, far=(what & 1) != 0, near=(what & 2) != 0)
    v, s, _ = _gpu_fmm(x, w, a, 10, 3, what=what)
    _check(v, s, vr, sr)


@pytest.mark.parametrize("p,depth,n", [(1, 2, 200), (4, 2, 37), (13, 4, 5000), (24, 2, 300), (16, 5, 20000)])
def test_orders_depths_ragged(oracle, p, depth, n):
    # several tiles and ragged leaves: empty boxes, uneven counts, odd p, p at the FP64 limit
    rng = np.random.default_rng(100 + p)
    x = rng.uniform(0, 1, (n, 3)) ** 1.5  # non-uniform: many empty and crowded boxes
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    vr, sr, _ = oracle.fmm(x, w, a, p, depth)
    v, s, _ = _gpu_fmm(x, w, a, p, depth)
    _check(v, s, vr, sr)


def test_edge_cases(oracle):
    # one element: nothing acts on it
    v, s, _ = _gpu_fmm(np.array([[0.3, 0.4, 0.5]]), np.array([[1.0, 2.0, 3.0]]), 0.1, 6, 2)
    assert np.all(v == 0) and np.all(s == 0)
    # coincident elements (Gaussian core: s = f(0) w_i x w_j) and the singular kernel
    x = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.1, 0.9, 0.2], [0.8, 0.1, 0.7]])
    w = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.3, -0.2, 0.5], [-1.0, 0.4, 0.2]])
    for a in (0.2, 0.0):
        vr, sr, _ = oracle.fmm(x, w, a, 8, 2)
        v, s, _ = _gpu_fmm(x, w, a, 8, 2)
        _check(v, s, vr, sr)
    # elements on the domain faces (x = 0 and x = 1 exactly)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (500, 3))
    x[:20, 0] = 0.0
    x[20:40, 1] = 1.0
    w = rng.normal(size=(500, 3))
    vr, sr, _ = oracle.fmm(x, w, 0.05, 8, 3)
    v, s, _ = _gpu_fmm(x, w, 0.05, 8, 3)
    _check(v, s, vr, sr)


def test_domain_errors():
    torch = _torch()
    import paper_1201_5430_amd as L
    x = torch.rand(100, 3, dtype=torch.float64, device="cuda")
    x[7, 2] = 1.5
    with pytest.raises(L.LhfError) as e:
        L.Plan(x, 0.01, p=6, depth=3)
    assert e.value.status == -2
    x[7, 2] = float("nan")
    with pytest.raises(L.LhfError) as e:
        L.Plan(x, 0.01, p=6, depth=3)
    assert e.value.status == -3


def test_cube1m_fp64_sampled_leaves(oracle):
    # the full 2^20-element workload in the configuration the benchmark times;
    # the oracle evaluates the whole FMM for a seeded sample of leaves
    cfg = workloads.make("cube1m_fp64")
    x, w, a, p, d = cfg["x"], cfg["w"], cfg["a"], cfg["p"], cfg["depth"]
    v, s, st = _gpu_fmm(x, w, a, p, d)
    samp = workloads.sample_targets(x.shape[0], 48, seed=7)
    vr, sr, _ = oracle.fmm(x, w, a, p, d, sample=samp)
    m = ~np.isnan(vr[:, 0])
    assert m.sum() >= 48
    _check(v[m], s[m], vr[m], sr[m], l2=1e-11, mx=1e-10)
    assert st["boxes"][d] > 250000


def test_cube1m_fp32_sampled_leaves(oracle):
    # the mixed-precision workload at full size: FP32 elements and expansions, 2^20 elements,
    # depth 6, p = 10; the oracle runs the whole FMM in FP64 on the FP32-rounded inputs for
    # the leaves of 48 seeded elements
    cfg = workloads.make("cube1m_fp32")
    x = cfg["x"].astype(np.float32).astype(np.float64)
    w = cfg["w"].astype(np.float32).astype(np.float64)
    a = float(np.float32(cfg["a"]))
    p, d = cfg["p"], cfg["depth"]
    v, s, st = _gpu_fmm(x, w, a, p, d, precision=1)
    samp = workloads.sample_targets(x.shape[0], 48, seed=8)
    vr, sr, _ = oracle.fmm(x, w, a, p, d, sample=samp)
    m = ~np.isnan(vr[:, 0])
    assert m.sum() >= 48
    print(f"cube1m FP32 p={p} ({m.sum()} elements): ", end="")
    _check32(v[m], s[m], vr[m], sr[m])
    assert st["boxes"][d] > 250000


def test_generic_and_tiled_m2l_agree(oracle):
    # the class-batched M2L kernel and the generic one-wave-per-box kernel give the same field
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(31)
    n = 6000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    v1, s1, st1 = _gpu_fmm(x, w, a, 12, 4)
    v2, s2, st2 = _gpu_fmm(x, w, a, 12, 4, m2l_kernel=L.M2L_GENERIC)
    assert st1["m2l_kernel"] == "half" and st2["m2l_kernel"] == "generic"
    _check(v1, s1, v2, s2, l2=1e-13, mx=1e-12)


@pytest.mark.parametrize("p,depth", [(8, 3), (10, 4), (12, 4), (16, 3)])
def test_fp32_path_matches_fp64_oracle(oracle, p, depth):
    # FP32 elements and expansions; the oracle sees the FP32-rounded inputs in FP64.
    # The FP32 path's own rounding must stay far below the FMM truncation error.
    rng = np.random.default_rng(40 + p)
    n = 8000
    x = rng.uniform(0, 1, (n, 3)).astype(np.float32).astype(np.float64)
    w = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64)
    a = float(np.float32(0.5 * n ** (-1 / 3)))
    vr, sr, _ = oracle.fmm(x, w, a, p, depth)
    v, s, _ = _gpu_fmm(x, w, a, p, depth, precision=1)
    print(f"FP32 p={p} depth={depth}: ", end="")
    _check32(v, s, vr, sr)


@pytest.mark.parametrize("p", [4, 6, 8, 10])
def test_fp32_batched_m2l_orders(oracle, p):
    # every order with a batched-M2L instantiation (both accumulation modes), depth 5 so that
    # tiles hold full sibling groups and the domain boundary cuts others
    rng = np.random.default_rng(60 + p)
    n = 30000
    x = rng.uniform(0, 1, (n, 3)).astype(np.float32).astype(np.float64)
    w = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64)
    a = float(np.float32(0.5 * n ** (-1 / 3)))
    samp = rng.choice(n, 40, replace=False)
    vr, sr, _ = oracle.fmm(x, w, a, p, 5, sample=samp)
    m = ~np.isnan(vr[:, 0])
    v, s, _ = _gpu_fmm(x, w, a, p, 5, precision=1)
    print(f"FP32 p={p} depth=5 sampled: ", end="")
    _check32(v[m], s[m], vr[m], sr[m])


@pytest.mark.parametrize("p", [8, 10])
def test_fp32_two_row_tile(oracle, p):
    # the one-lane ownership tile with two schedule rows per batch: against the oracle and the
    # one-row tile
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(100 + p)
    n = 30000
    x = rng.uniform(0, 1, (n, 3)).astype(np.float32).astype(np.float64)
    w = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64)
    a = float(np.float32(0.5 * n ** (-1 / 3)))
    samp = rng.choice(n, 40, replace=False)
    vr, sr, _ = oracle.fmm(x, w, a, p, 5, sample=samp)
    m = ~np.isnan(vr[:, 0])
    v2, s2, st2 = _gpu_fmm(x, w, a, p, 5, precision=1, m2l_kernel=L.M2L_TILE)
    v1, s1, st1 = _gpu_fmm(x, w, a, p, 5, precision=1, m2l_kernel=L.M2L_TILE1)
    assert st2["m2l_kernel"] == "tile" and st1["m2l_kernel"] == "tile1"
    print(f"two-row tile FP32 p={p}: ", end="")
    _check32(v2[m], s2[m], vr[m], sr[m])
    print("  vs one-row: ", end="")
    _check32(v2, s2, v1, s1)


@pytest.mark.parametrize("prec,p", [(0, 8), (0, 10), (0, 12), (0, 16), (0, 20), (0, 22), (0, 23), (0, 24),
                                    (1, 8), (1, 10), (1, 12), (1, 16)])
def test_half_vector_m2l(oracle, prec, p):
    # the M2L kernel with each part vector split over two lanes by the parity of m (the default
    # at p = 8, 10, 12, 16, and at FP64 p = 20, 22, 23, 24 with its rotation tables read from
    # global memory): against the oracle on sampled leaves and against the one-lane tile (FP64
    # p >= 16: the generic per-box kernel) on every element
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(110 + p + prec)
    n = 30000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    if prec:
        x = x.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
        a = float(np.float32(a))
    samp = rng.choice(n, 40, replace=False)
    vr, sr, _ = oracle.fmm(x, w, a, p, 5, sample=samp)
    m = ~np.isnan(vr[:, 0])
    vh, sh, sth = _gpu_fmm(x, w, a, p, 5, precision=prec, m2l_kernel=L.M2L_HALF)
    other = L.M2L_GENERIC if (prec == 0 and p >= 16) else L.M2L_TILE
    v1, s1, st1 = _gpu_fmm(x, w, a, p, 5, precision=prec, m2l_kernel=other)
    assert sth["m2l_kernel"] == "half" and st1["m2l_kernel"] == L.M2L_NAMES[other]
    print(f"half-vector M2L prec={prec} p={p}: ", end="")
    if prec == 0:
        _check(vh[m], sh[m], vr[m], sr[m])
        _check(vh, sh, v1, s1, l2=1e-13, mx=1e-12)
    else:
        _check32(vh[m], sh[m], vr[m], sr[m])
        _check32(vh, sh, v1, s1)


@pytest.mark.parametrize("p", [8, 12, 16, 20, 22, 23, 24])
def test_quarter_vector_m2l(oracle, p):
    # the FP64 M2L kernel with each part vector split over four lanes by m mod 4: against the
    # oracle on sampled leaves and against the half-vector kernel on every element, on a uniform
    # tree and on an adaptive one (leaves on several levels, tiles whose parent lacks children)
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(210 + p)
    n = 30000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    samp = rng.choice(n, 40, replace=False)
    vr, sr, _ = oracle.fmm(x, w, a, p, 5, sample=samp)
    m = ~np.isnan(vr[:, 0])
    vq, sq, stq = _gpu_fmm(x, w, a, p, 5, m2l_kernel=L.M2L_QUARTER)
    vh, sh, sth = _gpu_fmm(x, w, a, p, 5, m2l_kernel=L.M2L_HALF)
    assert stq["m2l_kernel"] == "quarter" and sth["m2l_kernel"] == "half"
    print(f"quarter-vector M2L p={p}: ", end="")
    _check(vq[m], sq[m], vr[m], sr[m])
    _check(vq, sq, vh, sh, l2=1e-13, mx=1e-12)
    # adaptive tree: the vortex ring with its background, <= 16 per leaf down to level 7
    import workloads
    xr, wr = workloads.vortex_ring(8000, 211)
    ar = workloads.core_radius(8000)
    vq, sq, _ = _gpu_fmm(xr, wr, ar, p, 7, max_per_leaf=16, m2l_kernel=L.M2L_QUARTER)
    vh, sh, _ = _gpu_fmm(xr, wr, ar, p, 7, max_per_leaf=16, m2l_kernel=L.M2L_HALF)
    print(f"  adaptive ring: ", end="")
    _check(vq, sq, vh, sh, l2=1e-13, mx=1e-12)


def test_reused_device_blocks(oracle):
    # a plan built on the blocks of a destroyed one (same sizes) gives the same field as a plan
    # on fresh blocks; p = 6 runs the deterministic ownership tile, so the comparison is exact
    import paper_1201_5430_amd as LH
    rng = np.random.default_rng(77)
    n = 5000
    xa, wa = rng.uniform(0, 1, (n, 3)), rng.normal(size=(n, 3))
    xb, wb = rng.uniform(0, 1, (n, 3)), rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    _gpu_fmm(xa, wa, a, 6, 3)
    v1, s1, _ = _gpu_fmm(xb, wb, a, 6, 3)  # takes the blocks the first plan left
    LH.release_cached_memory()
    v2, s2, _ = _gpu_fmm(xb, wb, a, 6, 3)  # fresh blocks
    assert np.array_equal(v1, v2) and np.array_equal(s1, s2)
    vr, sr, _ = oracle.fmm(xb, wb, a, 6, 3)
    _check(v1, s1, vr, sr)


@pytest.mark.parametrize("prec,p,depth", [(0, 12, 5), (0, 16, 4), (1, 10, 5)])
def test_batched_m2m_l2l_match_generic(prec, p, depth):
    # the half-vector M2M/L2L kernels (the default at p = 8, 10, 12, 16) against the generic
    # per-box shifts
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(120 + p)
    n = 30000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    v1, s1, st1 = _gpu_fmm(x, w, a, p, depth, precision=prec)
    v2, s2, st2 = _gpu_fmm(x, w, a, p, depth, precision=prec, mm_kernel=L.MM_GENERIC)
    assert st1["mm_kernel"] == "half" and st2["mm_kernel"] == "generic"
    print(f"batched vs generic M2M/L2L prec={prec} p={p}: {_rel(v1, v2):.3e} {_rel(s1, s2):.3e}", flush=True)
    if prec == 0:
        _check(v1, s1, v2, s2, l2=1e-13, mx=1e-12)
    else:
        _check32(v1, s1, v2, s2)


@pytest.mark.parametrize("p", [20, 23, 24])
def test_quarter_m2m_l2l_match_generic(oracle, p):
    # the quarter-vector M2M/L2L kernels (the default at FP64 p = 20, 22, 23, 24) against the
    # generic per-box shifts, on a uniform tree and on the adaptive ring (parents with one to eight
    # children), and against the oracle on sampled elements
    import paper_1201_5430_amd as L
    import workloads
    rng = np.random.default_rng(130 + p)
    n = 20000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    v1, s1, st1 = _gpu_fmm(x, w, a, p, 4)
    v2, s2, st2 = _gpu_fmm(x, w, a, p, 4, mm_kernel=L.MM_GENERIC)
    assert st1["mm_kernel"] == "quarter" and st2["mm_kernel"] == "generic"
    print(f"quarter vs generic M2M/L2L p={p}: ", end="")
    _check(v1, s1, v2, s2, l2=1e-13, mx=1e-12)
    samp = rng.choice(n, 30, replace=False)
    vr, sr, _ = oracle.fmm(x, w, a, p, 4, sample=samp)
    m = ~np.isnan(vr[:, 0])
    print("  vs oracle: ", end="")
    _check(v1[m], s1[m], vr[m], sr[m])
    xr, wr = workloads.vortex_ring(8000, 131)
    ar = workloads.core_radius(8000)
    v1, s1, st1 = _gpu_fmm(xr, wr, ar, p, 7, max_per_leaf=16)
    v2, s2, _ = _gpu_fmm(xr, wr, ar, p, 7, max_per_leaf=16, mm_kernel=L.MM_GENERIC)
    assert st1["mm_kernel"] == "quarter"
    print("  adaptive ring: ", end="")
    _check(v1, s1, v2, s2, l2=1e-13, mx=1e-12)


def test_autotuned_shapes(tmp_path):
    # the run-time shape autotuner on an adaptive ring at FP64 p = 23 (quarter-vector M2L tiles per
    # level, near-field source tile): valid shapes, the field unchanged to rounding after tuning,
    # the cache file read back, and out-of-range shapes refused
    torch = _torch()
    import paper_1201_5430_amd as L
    import workloads
    n = 20000
    x, w = workloads.vortex_ring(n, 141)
    a = workloads.core_radius(n)
    xt = torch.from_numpy(x).to("cuda")
    wt = torch.from_numpy(w).to("cuda")
    plan = L.Plan(xt, a, p=23, depth=7, max_per_leaf=32)
    v0, s0 = plan.execute(wt)
    v0, s0 = v0.cpu().numpy(), s0.cpu().numpy()
    cache = str(tmp_path / "shapes.json")
    sh = plan.autotune(wt, cache_path=cache)
    print("tuned shapes", sh, flush=True)
    assert sh["p2p_tile"] in (64, 128, 256)
    st = plan.stats()
    for l in range(9):
        if 2 <= l <= st["depth"] and st["boxes"][l] > 0:
            assert 1 <= sh["m2l_tile"][l] <= 6
        else:
            assert sh["m2l_tile"][l] == 0
    assert plan.get_shapes() == sh
    v1, s1 = plan.execute(wt)
    torch.cuda.synchronize()
    print("after tuning: ", end="")
    _check(v1.cpu().numpy(), s1.cpu().numpy(), v0, s0, l2=1e-13, mx=1e-12)
    # every tile size gives the same field
    for ts in (64, 256):
        plan.set_shapes(dict(m2l_tile=[0, 0, 1, 1, 2, 3, 4, 5, 6], p2p_tile=ts))
        v2, s2 = plan.execute(wt)
        _check(v2.cpu().numpy(), s2.cpu().numpy(), v0, s0, l2=1e-13, mx=1e-12)
    # second plan of the same workload: the shapes come from the cache
    plan2 = L.Plan(xt, a, p=23, depth=7, max_per_leaf=32)
    assert plan2.autotune(wt, cache_path=cache) == sh
    with pytest.raises(L.LhfError):
        plan2.set_shapes(dict(m2l_tile=[0, 0, 7, 0, 0, 0, 0, 0, 0]))
    with pytest.raises(L.LhfError):
        plan2.set_shapes(dict(p2p_tile=100))
    plan.close()
    plan2.close()


@pytest.mark.parametrize("p", [20, 23, 24])
def test_qmfma_m2l(oracle, p):
    # the matrix-core M2L with the vectors in registers (residue layout, both parts per lane): against
    # the oracle on sampled leaves and against the quarter-vector VALU kernel on every element, on a
    # uniform tree and on the adaptive ring
    import paper_1201_5430_amd as L
    rng = np.random.default_rng(220 + p)
    n = 30000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    samp = rng.choice(n, 40, replace=False)
    vr, sr, _ = oracle.fmm(x, w, a, p, 5, sample=samp)
    m = ~np.isnan(vr[:, 0])
    vq, sq, stq = _gpu_fmm(x, w, a, p, 5, m2l_kernel=L.M2L_QMFMA)
    vh, sh, sth = _gpu_fmm(x, w, a, p, 5, m2l_kernel=L.M2L_QUARTER)
    assert stq["m2l_kernel"] == "qmfma" and sth["m2l_kernel"] == "quarter"
    print(f"matrix-core residue-layout M2L p={p}: ", end="")
    _check(vq[m], sq[m], vr[m], sr[m])
    _check(vq, sq, vh, sh, l2=1e-13, mx=1e-12)
    import workloads
    xr, wr = workloads.vortex_ring(8000, 221)
    ar = workloads.core_radius(8000)
    vq, sq, _ = _gpu_fmm(xr, wr, ar, p, 7, max_per_leaf=16, m2l_kernel=L.M2L_QMFMA)
    vh, sh, _ = _gpu_fmm(xr, wr, ar, p, 7, max_per_leaf=16, m2l_kernel=L.M2L_QUARTER)
    print(f"  adaptive ring: ", end="")
    _check(vq, sq, vh, sh, l2=1e-13, mx=1e-12)
