"""Pins of the oracle's M2P and P2L operators and of the adaptive FMM that uses them for the
W and X lists (CPU only).

M2P evaluates a multipole expansion's field at targets outside its ball, P2L forms the local
expansion about a centre of elements outside its ball; both are defined in the oracle by
composing pinned operators (P2M about the element itself, M2L with the R-basis conversion,
L2P).  Pinned here against the Biot-Savart sums they approximate, which they must reach
geometrically in p, and, for the adaptive FMM, against the split direct sum.
"""
import numpy as np
import pytest

import workloads


def _bs(xs, ws, qs, y, wy):
    """singular v, s, grad v at y of sources (xs, ws, qs): the plain sums of eqs. 1 and 7"""
    d = y[None, :] - xs
    r = np.linalg.norm(d, axis=1)
    f = 1.0 / r ** 3
    g = -3.0 / r ** 5
    wxr = np.cross(ws, d)
    v = (f[:, None] * wxr + (qs * f)[:, None] * d).sum(0)
    G = np.zeros((3, 3))
    for i in range(xs.shape[0]):
        eps = np.zeros((3, 3))
        wi = ws[i]
        # d_l (w x r)_k = eps_{k a l} w_a
        eps[0, 1], eps[0, 2], eps[1, 0], eps[1, 2], eps[2, 0], eps[2, 1] = -wi[2], wi[1], wi[2], -wi[0], -wi[1], wi[0]
        G += g[i] * np.outer(wxr[i], d[i]) + f[i] * eps + qs[i] * (g[i] * np.outer(d[i], d[i]) + f[i] * np.eye(3))
    return v, G @ wy, G


@pytest.mark.parametrize("with_q", [False, True])
def test_m2p_converges_to_biot_savart(oracle, with_q):
    rng = np.random.default_rng(21)
    xs = rng.uniform(-0.5, 0.5, (25, 3))
    ws = rng.normal(size=(25, 3))
    qs = rng.normal(size=25) if with_q else np.zeros(25)
    y = np.array([[2.0, -1.5, 1.2], [-1.8, 0.4, -2.1]])
    wy = rng.normal(size=(2, 3))
    errs = []
    for p in (4, 8, 12, 16):
        ph, ch = oracle.p2m(p, np.zeros(3), xs, ws, q=qs if with_q else None)
        v, s, g = oracle.m2p(p, np.zeros(3), ph, ch, y, wy)
        e = 0.0
        for j in range(2):
            vr, sr, gr = _bs(xs, ws, qs, y[j], wy[j])
            e = max(e, np.abs(v[j] - vr).max() / np.abs(vr).max(), np.abs(s[j] - sr).max() / np.abs(sr).max(),
                    np.abs(g[j] - gr).max() / np.abs(gr).max())
        errs.append(e)
    assert all(errs[i + 1] < errs[i] / 4 for i in range(3)), errs
    assert errs[-1] < 1e-6


@pytest.mark.parametrize("with_q", [False, True])
def test_p2l_converges_to_biot_savart(oracle, with_q):
    rng = np.random.default_rng(22)
    xs = np.array([2.2, -1.4, 1.6]) + rng.uniform(-0.4, 0.4, (20, 3))
    ws = rng.normal(size=(20, 3))
    qs = rng.normal(size=20) if with_q else np.zeros(20)
    y = rng.uniform(-0.3, 0.3, (5, 3))
    wy = rng.normal(size=(5, 3))
    errs = []
    for p in (4, 8, 12, 16):
        ph, ch = oracle.p2l(p, np.zeros(3), xs, ws, q=qs if with_q else None)
        v, s, g, iv, _ = oracle.l2p(p, np.zeros(3), ph, ch, y, wy)
        assert np.abs(iv).max() < 1e-12 * np.abs(v).max()
        e = 0.0
        for j in range(5):
            vr, sr, gr = _bs(xs, ws, qs, y[j], wy[j])
            e = max(e, np.abs(v[j] - vr).max() / np.abs(vr).max(), np.abs(s[j] - sr).max() / np.abs(sr).max(),
                    np.abs(g[j] - gr).max() / np.abs(gr).max())
        errs.append(e)
    assert all(errs[i + 1] < errs[i] / 4 for i in range(3)), errs
    assert errs[-1] < 1e-6


def test_adaptive_fmm_with_wx_expansions(oracle):
    # W boxes by M2P and X sources by P2L: the same split direct sum is approached geometrically
    # in p, and the pair coverage of the lists is unchanged
    x, w = workloads.vortex_ring(6000, 23)
    q = np.random.default_rng(23).normal(size=6000) * 0.1
    a = workloads.core_radius(6000)
    mx, lm = 16, 7
    tg = workloads.sample_targets(6000, 400, seed=2)
    vd, sd = oracle.direct_adaptive(x, w, a, mx, lm, targets=tg, q=q)
    errs = []
    for p in (6, 10, 14):
        v, s, st = oracle.fmm_adaptive(x, w, a, p, mx, lm, q=q, wx_expansions=True)
        errs.append(max(np.linalg.norm(v[tg] - vd) / np.linalg.norm(vd), np.linalg.norm(s[tg] - sd) / np.linalg.norm(sd)))
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10, errs
    # far/near parts add up to the whole, and the direct W/X sums are gone from the near field
    v0, s0, st0 = oracle.fmm_adaptive(x, w, a, 10, mx, lm, q=q)
    vf, sf, _ = oracle.fmm_adaptive(x, w, a, 10, mx, lm, q=q, wx_expansions=True, near=False)
    vn, sn, stn = oracle.fmm_adaptive(x, w, a, 10, mx, lm, q=q, wx_expansions=True, far=False)
    v1, s1, _ = oracle.fmm_adaptive(x, w, a, 10, mx, lm, q=q, wx_expansions=True)
    assert np.abs(vf + vn - v1).max() <= 1e-13 * np.abs(v1).max()
    assert st0["n_wx_pairs"] > 0 and stn["n_wx_pairs"] < st0["n_wx_pairs"] // 10
    assert stn["n_p2p_pairs"] == st0["n_p2p_pairs"]
    # the two W/X treatments differ only by the truncation error
    assert np.linalg.norm(v1 - v0) / np.linalg.norm(v0) < 3 * errs[1]
