"""Pins of the oracle's scalar harmonic FMM (the single-potential comparison workload of Sec. 5.2),
CPU only.

Phi_j = sum_{i != j} q_i / |x_j - x_i| and grad Phi_j with the singular kernel.  Pinned against a
configuration worked by hand, against the vortex FMM (whose monopole far field is pinned
separately) with the sources' sign turned over, and by geometric convergence in p to the direct
sum; the far and near parts add up to the whole.
"""
import numpy as np

import workloads


def test_scalar_direct_by_hand(oracle):
    # q = 2 at the origin, q = -1 at (3, 0, 0), q = 0.5 at (0, 4, 0)
    x = np.array([[0.0, 0, 0], [3.0, 0, 0], [0.0, 4, 0]])
    q = np.array([2.0, -1.0, 0.5])
    phi, g = oracle.scalar_direct(x, q)
    assert np.allclose(phi, [-1 / 3 + 0.5 / 4, 2 / 3 + 0.5 / 5, 2 / 4 - 1 / 5], rtol=0, atol=1e-15)
    # grad at the origin: -sum q r / r^3, r = 0 - x_i
    g0 = -(-1.0) * np.array([-3.0, 0, 0]) / 27 - 0.5 * np.array([0, -4.0, 0]) / 64
    assert np.allclose(g[0], g0, rtol=0, atol=1e-15)
    # targets subset
    phi1, g1 = oracle.scalar_direct(x, q, targets=[2])
    assert phi1.shape == (1,) and abs(phi1[0] - phi[2]) < 1e-15 and np.abs(g1[0] - g[2]).max() < 1e-15


def test_scalar_fmm_gradient_is_the_source_velocity(oracle):
    # grad Phi of the scalar FMM equals the vortex FMM's velocity with no vortex strength and the
    # sources negated (v = -grad(q'/r) there), singular kernel, same tree and p
    x, _ = workloads.uniform_cube(2000, 31)
    q = np.random.default_rng(31).normal(size=2000)
    for p in (6, 10):
        phi, g, _ = oracle.fmm_scalar(x, q, p, 3)
        v, s, _ = oracle.fmm(x, np.zeros_like(x), 0.0, p, 3, q=-q)
        assert np.abs(g - v).max() <= 1e-12 * np.abs(v).max()


def test_scalar_fmm_converges_to_the_direct_sum(oracle):
    x, _ = workloads.uniform_cube(3000, 32)
    q = np.random.default_rng(32).normal(size=3000)
    pd, gd = oracle.scalar_direct(x, q)
    errs = []
    for p in (4, 8, 12, 16):
        phi, g, st = oracle.fmm_scalar(x, q, p, 3)
        errs.append(max(np.linalg.norm(phi - pd) / np.linalg.norm(pd), np.linalg.norm(g - gd) / np.linalg.norm(gd)))
    assert all(errs[i + 1] < errs[i] / 5 for i in range(3)), errs
    assert errs[-1] < 1e-6
    # far + near = whole; sampling evaluates the leaves of the sampled elements
    pf, gf, _ = oracle.fmm_scalar(x, q, 8, 3, near=False)
    pn, gn, _ = oracle.fmm_scalar(x, q, 8, 3, far=False)
    pw, gw, _ = oracle.fmm_scalar(x, q, 8, 3)
    assert np.abs(pf + pn - pw).max() <= 1e-13 * np.abs(pw).max()
    samp = np.array([5, 700, 2999])
    ps, gs, _ = oracle.fmm_scalar(x, q, 8, 3, sample=samp)
    m = ~np.isnan(ps)
    assert m[samp].all() and m.sum() < 3000
    assert np.abs(ps[m] - pw[m]).max() <= 1e-14 * np.abs(pw).max()
