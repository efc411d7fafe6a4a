"""GPU parity of the matrix-core (MFMA) M2L kernel.

Every order with an MFMA instantiation, FP64 against the oracle's FMM (relative L2
<= 1e-12: the MFMA path changes only the summation order of the rotation and
coaxial products) and FP32 against the FP64 oracle on FP32-rounded inputs (<= 2e-6);
plus the adaptive tree, and the MFMA and VALU kernels against each other (the MFMA
kernel is the default for FP32 at p = 16, the VALU kernel elsewhere).
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


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _gpu(x, w, a, p, depth, precision=0, max_per_leaf=0):
    torch = _torch()
    import paper_1201_5430_amd as LH
    dt = torch.float64 if precision == 0 else torch.float32
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(device="cuda", dtype=dt)
    plan = LH.Plan(xt, a, p=p, depth=depth, precision=precision, max_per_leaf=max_per_leaf)
    v, s = plan.execute(wt)
    torch.cuda.synchronize()
    plan.close()
    return v.double().cpu().numpy(), s.double().cpu().numpy()


@pytest.mark.parametrize("p", [4, 6, 8, 10, 12])
def test_fp64_mfma_matches_oracle(oracle, monkeypatch, p):
    monkeypatch.setenv("LHF_MFMA", "1")
    rng = np.random.default_rng(70 + p)
    n = 6000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    vr, sr, _ = oracle.fmm(x, w, a, p, 4)
    v, s = _gpu(x, w, a, p, 4)
    ev, es = _rel(v, vr), _rel(s, sr)
    print(f"MFMA FP64 p={p}: rel L2 v {ev:.3e} s {es:.3e}", flush=True)
    assert ev <= 1e-12 and es <= 1e-12


@pytest.mark.parametrize("p", [4, 6, 8, 10, 12, 16])
def test_fp32_mfma_matches_oracle(oracle, monkeypatch, p):
    monkeypatch.setenv("LHF_MFMA", "1")
    rng = np.random.default_rng(80 + p)
    n = 8000
    x = rng.uniform(0, 1, (n, 3)).astype(np.float32).astype(np.float64)
    w = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64)
    a = float(np.float32(0.5 * n ** (-1 / 3)))
    vr, sr, _ = oracle.fmm(x, w, a, p, 4)
    v, s = _gpu(x, w, a, p, 4, precision=1)
    ev, es = _rel(v, vr), _rel(s, sr)
    print(f"MFMA FP32 p={p}: rel L2 v {ev:.3e} s {es:.3e}", flush=True)
    assert ev < 2e-6 and es < 2e-6


def test_adaptive_ring_mfma(oracle, monkeypatch):
    monkeypatch.setenv("LHF_MFMA", "1")
    x, w = workloads.vortex_ring(6000, 41)
    a = workloads.core_radius(6000)
    vr, sr, _ = oracle.fmm_adaptive(x, w, a, 8, 16, 7)
    v, s = _gpu(x, w, a, 8, 7, max_per_leaf=16)
    ev, es = _rel(v, vr), _rel(s, sr)
    print(f"MFMA adaptive ring: rel L2 v {ev:.3e} s {es:.3e}", flush=True)
    assert ev <= 1e-12 and es <= 1e-12


@pytest.mark.parametrize("p,prec", [(12, 0), (10, 1), (16, 1)])
def test_mfma_and_valu_kernels_agree(monkeypatch, p, prec):
    rng = np.random.default_rng(90 + p)
    n = 40000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    monkeypatch.setenv("LHF_MFMA", "1")
    v1, s1 = _gpu(x, w, a, p, 5, precision=prec)
    monkeypatch.delenv("LHF_MFMA")
    monkeypatch.setenv("LHF_NO_MFMA", "1")
    v2, s2 = _gpu(x, w, a, p, 5, precision=prec)
    bar = 1e-13 if prec == 0 else 2e-6
    print(f"MFMA vs VALU p={p} prec={prec}: {_rel(v1, v2):.3e} {_rel(s1, s2):.3e}", flush=True)
    assert _rel(v1, v2) <= bar and _rel(s1, s2) <= bar
