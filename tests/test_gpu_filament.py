"""GPU parity of the vortex-filament path (lhf_filament_*) against the oracle's filament FMM.

Closed polygonal filaments, velocity at the vertices; same octree (uniform, over segment centres
and vertices), same p and quadrature order (eq. vf7) on both sides.  FP64 bar 1e-12 relative L2
and 1e-11 element-wise.  FP32 against the FP64 oracle on FP32-rounded inputs: 2e-5 / 1e-4.  The
closed form of eq. dis2 takes the cross product of the vectors from the vertex to the ends of a
segment of the same filament two or three segments away, nearly parallel on a smooth filament
(angle ~ 2 pi / 50 here), so each term carries eps / sin(angle) ~ 10 eps of rounding, and these
near terms dominate a vertex's velocity (the log-singular self-induction): FP64 measures 9e-14,
FP32 4.5e-6 against the FP64 oracle.
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


def _gpu(X, seg, G, p, depth, precision=0):
    torch = _torch()
    import paper_1201_5430_amd as LH
    dt = torch.float64 if precision == 0 else torch.float32
    print(f"filament: V={X.shape[0]} S={seg.shape[0]} p={p} depth={depth} prec={precision}", flush=True)
    f = LH.Filament(torch.from_numpy(X).to("cuda", dt), torch.from_numpy(seg).cuda(), p=p, depth=depth,
                    precision=precision)
    v = f.execute(torch.from_numpy(G).to("cuda", dt))
    torch.cuda.synchronize()
    st = f.stats()
    f.close()
    return v.double().cpu().numpy(), st


@pytest.mark.parametrize("p,depth", [(8, 3), (12, 4), (16, 3)])
def test_filament_fp64(oracle, p, depth):
    X, seg, G = workloads.filament_rings(200, 50, 71)
    vr, ost = oracle.filament_fmm(X, seg, G, p, depth)
    v, st = _gpu(X, seg, G, p, depth)
    assert st["n_m2l"] == ost["n_m2l"]
    check(v, v, vr, vr, label=f"filaments FP64 p={p}:")


@pytest.mark.parametrize("p", [8, 10])
def test_filament_fp32(oracle, p):
    X, seg, G = workloads.filament_rings(200, 50, 72)
    X = X.astype(np.float32).astype(np.float64)
    G = G.astype(np.float32).astype(np.float64)
    vr, _ = oracle.filament_fmm(X, seg, G, p, 4)
    v, st = _gpu(X, seg, G, p, 4, precision=1)
    check32(v, v, vr, vr, l2=2e-5, mx=1e-4, label=f"filaments FP32 p={p}:")


def test_filament_against_direct_sum(oracle):
    # at p = 16 the FMM is the direct sum of eq. dis2 to the method's truncation error
    X, seg, G = workloads.filament_rings(100, 40, 73)
    vd = oracle.filament_direct(X, seg, G)
    v, _ = _gpu(X, seg, G, 16, 3)
    e = np.linalg.norm(v - vd) / np.linalg.norm(vd)
    print(f"filaments p=16 vs direct: rel L2 {e:.3e}", flush=True)
    assert e < 1e-6


def test_filament_argument_checks():
    torch = _torch()
    import paper_1201_5430_amd as LH
    X = torch.rand((10, 3), dtype=torch.float64, device="cuda")
    bad = torch.tensor([[0, 1], [3, 10]], dtype=torch.int32, device="cuda")
    with pytest.raises(LH.LhfError, match="out of range"):
        LH.Filament(X, bad, p=8, depth=3)
    same = torch.tensor([[2, 2]], dtype=torch.int32, device="cuda")
    with pytest.raises(LH.LhfError, match="coincident"):
        LH.Filament(X, same, p=8, depth=3)
    f = LH.Filament(X, torch.tensor([[0, 1]], dtype=torch.int32, device="cuda"), p=8, depth=3)
    with pytest.raises(TypeError):
        f.execute(torch.ones(1, dtype=torch.float32, device="cuda"))
    f.close()
