"""The allocation-free one-shot entry point (lhf_evaluate_noalloc) against lhf_evaluate.

Both run the same kernels; the allocation-free one takes every device buffer of its plan
from a fixed per-device array.  Two calls in a row (the second smaller, so it runs on
the array as the first call left it) must each match lhf_evaluate on the same input to
the FP64 bar (relative L2 1e-12, element-wise 1e-11 of the largest magnitude).  Inputs
beyond the array's limits are rejected with LHF_ERR_WORKSPACE.
"""
import numpy as np
import pytest

from parity_util import check

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _case(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (n, 3)), rng.normal(size=(n, 3)), 0.5 * n ** (-1 / 3)


def test_noalloc_matches_evaluate_twice():
    torch = _torch()
    import paper_1201_5430_amd as L
    for n, p, depth, seed in ((30000, 8, 4, 601), (3000, 10, 3, 602)):
        x, w, a = _case(n, seed)
        xt = torch.from_numpy(x).cuda()
        wt = torch.from_numpy(w).cuda()
        v0, s0 = L.evaluate(xt, wt, a, p=p, depth=depth)
        v = torch.full_like(wt, float("nan"))
        s = torch.full_like(wt, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        v1, s1 = L.evaluate_noalloc(xt, wt, a, p=p, depth=depth, v=v, s=s)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        print(f"noalloc n={n} p={p} depth={depth}: device free bytes before {free0} after {free1}", flush=True)
        assert free1 >= free0  # the call took no device memory
        check(v1.cpu().numpy(), s1.cpu().numpy(), v0.cpu().numpy(), s0.cpu().numpy(),
              label=f"noalloc vs evaluate n={n}:")


def test_noalloc_rejects_what_does_not_fit():
    torch = _torch()
    import paper_1201_5430_amd as L
    x, w, a = _case(1000, 603)
    # more elements than the entry point accepts: rejected on the host
    big = torch.zeros((1 << 17) + 1, 3, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LhfError) as e:
        L.evaluate_noalloc(big, big, 0.01, p=8, depth=4)
    assert e.value.status == -4
    # a plan larger than the array (FP64 p = 16 at depth 5: 600 MB of expansions)
    xb, wb, ab = _case(100000, 604)
    with pytest.raises(L.LhfError) as e:
        L.evaluate_noalloc(torch.from_numpy(xb).cuda(), torch.from_numpy(wb).cuda(), ab, p=16, depth=5)
    assert e.value.status == -4 and "MiB" in str(e.value)
    # and the entry point still works afterwards
    xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    v0, s0 = L.evaluate(xt, wt, a, p=6, depth=3)
    v1, s1 = L.evaluate_noalloc(xt, wt, a, p=6, depth=3)
    check(v1.cpu().numpy(), s1.cpu().numpy(), v0.cpu().numpy(), s0.cpu().numpy(), label="after rejection:")
