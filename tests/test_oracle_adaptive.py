"""Pins of the oracle's adaptive-octree FMM (U/V/W/X lists after Carrier, Greengard
and Rokhlin; W and X summed directly with the singular kernel).

- every ordered pair of leaves is carried by exactly one mechanism (U, a V pair of
  ancestors, W, X) -- on a clustered ring and on an unbalanced cluster;
- with max_per_leaf = 0 the adaptive tree is the uniform tree and the result equals
  the uniform FMM (itself pinned in test_oracle_fmm);
- the adaptive direct sum reduces to the smoothed direct sum for a one-leaf tree and
  to the uniform split rule for a full tree;
- the FMM converges to the adaptive direct sum as p grows, with a core radius large
  enough that a wrong kernel on a W/X pair would show.
"""
import numpy as np
import pytest

import workloads


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _cluster(n, seed):
    # a tight Gaussian cluster inside a sparse background: a deep, unbalanced tree
    rng = np.random.default_rng(seed)
    nc = int(0.8 * n)
    xc = np.clip(rng.normal(0.3, 0.02, (nc, 3)), 0, 1 - 1e-12)
    xb = rng.uniform(0, 1, (n - nc, 3))
    x = np.concatenate([xc, xb])
    w = rng.normal(size=(n, 3))
    return x, w


@pytest.mark.parametrize("kind", ["ring", "cluster"])
def test_every_leaf_pair_carried_once(oracle, kind):
    if kind == "ring":
        x, _ = workloads.vortex_ring(4000, 31)
        mx, ml = 16, 7
    else:
        x, _ = _cluster(3000, 32)
        mx, ml = 8, 9
    lo, hi, nleaf = oracle.adaptive_coverage(x, mx, ml)
    nb, nl = oracle.adaptive_counts(x, mx, ml)
    assert nleaf == nl.sum() and nleaf > 200
    assert (nl > 0).sum() >= 3  # leaves on several levels
    assert lo == 1 and hi == 1


def test_leaves_partition_the_elements(oracle):
    x, _ = _cluster(3000, 33)
    leaf = oracle.adaptive_leaf_of(x, 8, 9)
    _, cnt = np.unique(leaf, return_counts=True)
    nb, nl = oracle.adaptive_counts(x, 8, 9)
    assert len(cnt) == nl.sum()
    lev = np.unique(leaf) >> 40
    # a leaf holds at most max_per_leaf elements unless it sits on the deepest level
    assert (cnt[lev < 9] <= 8).all()


def test_full_split_equals_uniform_fmm(oracle):
    x, w = workloads.uniform_cube(2500, 34)
    a = workloads.core_radius(2500)
    for d in (3, 4):
        v1, s1, st1 = oracle.fmm_adaptive(x, w, a, 8, 0, d)
        v2, s2, st2 = oracle.fmm(x, w, a, 8, d)
        assert st1["n_wx_pairs"] == 0 and st1["n_m2l"] == st2["n_m2l"]
        assert st1["n_p2p_pairs"] == st2["n_p2p_pairs"]
        assert np.abs(v1 - v2).max() <= 1e-14 * np.abs(v2).max()
        assert np.abs(s1 - s2).max() <= 1e-14 * np.abs(s2).max()


def test_adaptive_gradient(oracle):
    # grad v of the adaptive FMM: equals the uniform FMM's with every box split, is trace-free
    # (div v = 0 for both the truncated harmonic far field and the near-field kernel sum) and
    # contracts with omega to the stretching term s_k = sum_l omega_l d_l v_k
    x, w = workloads.uniform_cube(2500, 36)
    a = workloads.core_radius(2500)
    _, _, g1, _ = oracle.fmm_adaptive(x, w, a, 8, 0, 3, grad=True)
    _, _, g2, _ = oracle.fmm(x, w, a, 8, 3, grad=True)
    assert np.abs(g1 - g2).max() <= 1e-14 * np.abs(g2).max()
    x, w = workloads.vortex_ring(6000, 37)
    a = workloads.core_radius(6000)
    v, s, g, st = oracle.fmm_adaptive(x, w, a, 16, 16, 7, grad=True)
    assert st["n_wx_pairs"] > 0
    sc = np.abs(g).max()
    assert np.abs(np.trace(g, axis1=1, axis2=2)).max() <= 1e-12 * sc
    assert np.abs(np.einsum("ikl,il->ik", g, w) - s).max() <= 1e-12 * np.abs(s).max()
    # and converges to the split direct sum's gradient like v does (finite differences of v)
    tg = workloads.sample_targets(6000, 20, seed=9)
    h = 1e-6
    for j in tg[:5]:
        for l in range(3):
            xp, xm = x.copy(), x.copy()
            xp[j, l] += h
            xm[j, l] -= h
            # moving element j alone keeps its leaf for these h (tree fixed by the unshifted set)
            vp, _ = oracle.direct_adaptive(xp, w, a, 16, 7, targets=np.array([j]))
            vm, _ = oracle.direct_adaptive(xm, w, a, 16, 7, targets=np.array([j]))
            fd = (vp[0] - vm[0]) / (2 * h)
            assert np.abs(fd - g[j, :, l]).max() <= 1e-4 * sc


def test_adaptive_direct_special_cases(oracle):
    x, w = workloads.uniform_cube(600, 35)
    a = 0.05
    # one leaf (the root): every pair adjacent, smoothed everywhere
    v, s = oracle.direct_adaptive(x, w, a, 10 ** 9, 5)
    vr, sr = oracle.direct(x, w, a, mode=oracle.DIRECT_SMOOTH)
    assert _rel(v, vr) < 1e-15 and _rel(s, sr) < 1e-15
    # full split to depth 3: the uniform split rule
    v, s = oracle.direct_adaptive(x, w, a, 0, 3)
    vr, sr = oracle.direct(x, w, a, mode=oracle.DIRECT_SPLIT, depth=3)
    assert _rel(v, vr) < 1e-15 and _rel(s, sr) < 1e-15


def test_fmm_converges_to_adaptive_direct(oracle):
    x, w = _cluster(2500, 36)
    # a wide core: 1 - K(r; a) is far from 0 at W/X distances, so a smoothed W/X pair would show
    a = 0.01
    vd, sd = oracle.direct_adaptive(x, w, a, 8, 9)
    errs = []
    for p in (6, 10, 14, 18):
        v, s, st = oracle.fmm_adaptive(x, w, a, p, 8, 9)
        errs.append((_rel(v, vd), _rel(s, sd)))
    assert st["n_wx_pairs"] > 0
    for (ev0, es0), (ev1, es1) in zip(errs, errs[1:]):
        assert ev1 < 0.5 * ev0 and es1 < 0.5 * es0
    assert errs[-1][0] < 3e-6 and errs[-1][1] < 1e-4
    # the same tree with the smoothed kernel on W/X pairs is measurably different
    vs_, ss_ = oracle.direct(x, w, a, mode=oracle.DIRECT_SMOOTH)
    assert _rel(vs_, vd) > 1e3 * errs[-1][0]


def test_sampled_leaves_match_full_run(oracle):
    x, w = workloads.vortex_ring(3000, 37)
    a = workloads.core_radius(3000)
    v, s, _ = oracle.fmm_adaptive(x, w, a, 8, 16, 7)
    samp = np.array([5, 100, 2000, 2999])
    vs_, ss_, _ = oracle.fmm_adaptive(x, w, a, 8, 16, 7, sample=samp)
    m = ~np.isnan(vs_[:, 0])
    assert m[samp].all() and m.sum() < 3000
    assert np.abs(vs_[m] - v[m]).max() <= 1e-14 * np.abs(v).max()
    assert np.abs(ss_[m] - s[m]).max() <= 1e-14 * np.abs(s).max()
