"""GPU parity of the matrix-core (MFMA) M2L kernel.

Every order with an MFMA instantiation, FP64 against the oracle's FMM (relative L2
<= 1e-12: the MFMA path changes only the summation order of the rotation and
coaxial products) and FP32 against the FP64 oracle on FP32-rounded inputs (<= 2e-6);
plus the adaptive tree, and the MFMA and VALU kernels against each other.  The MFMA
kernel is slower than the VALU kernels at every order measured, so it runs only when
the descriptor asks for it (m2l_kernel = LHF_M2L_MFMA) or a deterministic plan has no
faster atomic-free kernel.
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


def _gpu(x, w, a, p, depth, precision=0, max_per_leaf=0, mfma=True):
    torch = _torch()
    import paper_1201_5430_amd as LH
    dt = torch.float64 if precision == 0 else torch.float32
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(device="cuda", dtype=dt)
    plan = LH.Plan(xt, a, p=p, depth=depth, precision=precision, max_per_leaf=max_per_leaf,
                   m2l_kernel=LH.M2L_MFMA if mfma else LH.M2L_AUTO)
    v, s = plan.execute(wt)
    torch.cuda.synchronize()
    assert (plan.stats()["m2l_kernel"] == "mfma") == mfma
    plan.close()
    return v.double().cpu().numpy(), s.double().cpu().numpy()


@pytest.mark.parametrize("p", [4, 6, 8, 10, 12])
def test_fp64_mfma_matches_oracle(oracle, p):
    rng = np.random.default_rng(70 + p)
    n = 6000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    vr, sr, _ = oracle.fmm(x, w, a, p, 4)
    v, s = _gpu(x, w, a, p, 4)
    check(v, s, vr, sr, label=f"MFMA FP64 p={p}:")


@pytest.mark.parametrize("p", [4, 6, 8, 10, 12, 16])
def test_fp32_mfma_matches_oracle(oracle, p):
    rng = np.random.default_rng(80 + p)
    n = 8000
    x = rng.uniform(0, 1, (n, 3)).astype(np.float32).astype(np.float64)
    w = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64)
    a = float(np.float32(0.5 * n ** (-1 / 3)))
    vr, sr, _ = oracle.fmm(x, w, a, p, 4)
    v, s = _gpu(x, w, a, p, 4, precision=1)
    check32(v, s, vr, sr, label=f"MFMA FP32 p={p}:")


def test_adaptive_ring_mfma(oracle):
    x, w = workloads.vortex_ring(6000, 41)
    a = workloads.core_radius(6000)
    vr, sr, _ = oracle.fmm_adaptive(x, w, a, 8, 16, 7)
    v, s = _gpu(x, w, a, 8, 7, max_per_leaf=16)
    check(v, s, vr, sr, label="MFMA adaptive ring:")


@pytest.mark.parametrize("p,prec", [(12, 0), (10, 1), (16, 1)])
def test_mfma_and_valu_kernels_agree(p, prec):
    rng = np.random.default_rng(90 + p)
    n = 40000
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.5 * n ** (-1 / 3)
    v1, s1 = _gpu(x, w, a, p, 5, precision=prec)
    v2, s2 = _gpu(x, w, a, p, 5, precision=prec, mfma=False)
    if prec == 0:
        check(v1, s1, v2, s2, l2=1e-13, mx=1e-12, label=f"MFMA vs VALU p={p} prec={prec}:")
    else:
        check32(v1, s1, v2, s2, label=f"MFMA vs VALU p={p} prec={prec}:")
