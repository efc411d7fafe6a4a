"""Pins of the oracle's monopole (source) terms, CPU only.

With divergence q (eqs. 5-7) each element adds -grad(q_i/|y - x_i|) to the velocity:
the potential phi gains a monopole (P2M: phi_n^m -= q g_n^m, the expansion of eq.
rsbf5), and the near field gains q_i f r (f = K/r^3, the same smoothing as the vortex
part).  Pinned against a source worked by hand, the closed-form divergence of the
smoothed source, the curl-free far field, M2M exactness with a net source, and the
convergence of the whole FMM to the direct sum.
"""
import numpy as np
import pytest

import workloads


def test_single_source_by_hand(oracle):
    # q = 2 at the origin, target at e_x with strength e_z, singular kernel:
    # v = q r/r^3 = 2 e_x; s = (w . grad) v = q (f w + g r (w . r)) = 2 e_z;
    # grad v = q (I - 3 e_x e_x)
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    w = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    q = np.array([2.0, 0.0])
    v, s, g = oracle.direct(x, w, 0.0, mode=oracle.DIRECT_SINGULAR, grad=True, q=q)
    assert np.allclose(v[1], [2.0, 0.0, 0.0], rtol=0, atol=1e-15)
    assert np.allclose(s[1], [0.0, 0.0, 2.0], rtol=0, atol=1e-15)
    assert np.allclose(g[1], 2.0 * (np.eye(3) - 3.0 * np.outer([1, 0, 0], [1, 0, 0])), atol=1e-15)
    # element 1 (vortex e_z at e_x, no source) acts on element 0: w x r / r^3 = e_z x (-e_x) = -e_y
    assert np.allclose(v[0], [0.0, -1.0, 0.0], atol=1e-15) and np.allclose(s[0], 0.0)


def test_divergence_of_the_smoothed_source(oracle):
    # div v = sum_i q_i (3 f + g r^2) = sum_i q_i K'(r)/r^2 = sum_i q_i sqrt(2/pi) e^{-r^2/2a^2}/a^3
    # for the Gaussian core (eq. vem1), 0 for the singular kernel; the vortex part is divergence-free
    rng = np.random.default_rng(3)
    n, a = 300, 0.08
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    q = rng.normal(size=n)
    _, _, g = oracle.direct(x, w, a, mode=oracle.DIRECT_SMOOTH, grad=True, q=q)
    tr = np.trace(g, axis1=1, axis2=2)
    d = x[None, :, :] - x[:, None, :]
    r2 = (d ** 2).sum(-1)
    dens = q[None, :] * np.sqrt(2 / np.pi) * np.exp(-r2 / (2 * a * a)) / a ** 3
    np.fill_diagonal(dens, 0.0)
    ref = dens.sum(1)
    assert np.abs(tr - ref).max() <= 1e-11 * np.abs(ref).max()
    _, _, g0 = oracle.direct(x, w, a, mode=oracle.DIRECT_SINGULAR, grad=True, q=q)
    assert np.abs(np.trace(g0, axis1=1, axis2=2)).max() <= 1e-12 * np.abs(g0).max()
    # the source part is curl-free: grad v of the q part alone is symmetric
    _, _, gq = oracle.direct(x, np.zeros_like(w), a, mode=oracle.DIRECT_SMOOTH, grad=True, q=q)
    assert np.abs(gq - gq.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(gq).max()


def test_source_multipole_and_m2m(oracle):
    # the phi monopole terms reproduce -grad(sum q/r) far away (error ~ (rho/|y|)^p), and M2M of the
    # children's expansions equals the parent's own P2M (net source: phi_0^0 != 0)
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.5, 0.5, (20, 3))
    w = np.zeros((20, 3))
    q = rng.normal(size=20) + 0.3
    y = np.array([2.5, -1.7, 2.1])
    d = y[None, :] - x
    ref = (q[:, None] * d / (np.linalg.norm(d, axis=1) ** 3)[:, None]).sum(0)
    errs = []
    for p in (4, 8, 12):
        ph, ch = oracle.p2m(p, np.zeros(3), x, w, q=q)
        assert abs(ph[0]) > 0 and np.abs(ch).max() == 0.0
        # v = grad phi by finite differences of the S expansion
        h = 1e-5
        gphi = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fp = np.sum(ph * oracle.basis_S(p, y + e)).real
            fm = np.sum(ph * oracle.basis_S(p, y - e)).real
            gphi[k] = (fp - fm) / (2 * h)
        errs.append(np.linalg.norm(gphi - ref) / np.linalg.norm(ref))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6
    # M2M exactness with sources (and vortices)
    p = 10
    w = rng.normal(size=(20, 3))
    cpar = np.zeros(3)
    kids = [(x[:, 0] < 0), (x[:, 0] >= 0)]
    cc = [np.array([-0.25, 0, 0]), np.array([0.25, 0, 0])]
    acc_ph = np.zeros(p * p, complex)
    acc_ch = np.zeros(p * p, complex)
    for m, c in zip(kids, cc):
        ph, ch = oracle.p2m(p, c, x[m], w[m], q=q[m])
        oph, och = oracle.m2m(p, cpar - c, ph, ch)
        acc_ph += oph
        acc_ch += och
    ph, ch = oracle.p2m(p, cpar, x, w, q=q)
    sc = np.abs(ph).max() + np.abs(ch).max()
    assert np.abs(acc_ph - ph).max() < 1e-13 * sc and np.abs(acc_ch - ch).max() < 1e-13 * sc


def test_fmm_with_sources_converges(oracle):
    # uniform and adaptive FMMs with monopoles converge in p to the split direct sums
    x, w = workloads.uniform_cube(3000, 8)
    q = np.random.default_rng(8).normal(size=3000)
    a = workloads.core_radius(3000)
    vd, sd, gd = oracle.direct(x, w, a, mode=oracle.DIRECT_SPLIT, depth=3, grad=True, q=q)
    prev = None
    for p in (6, 10, 14):
        v, s, g, _ = oracle.fmm(x, w, a, p, 3, grad=True, q=q)
        e = max(np.linalg.norm(v - vd) / np.linalg.norm(vd), np.linalg.norm(s - sd) / np.linalg.norm(sd),
                np.linalg.norm(g - gd) / np.linalg.norm(gd))
        assert prev is None or e < prev / 4
        prev = e
    assert prev < 1e-4  # the method's truncation level at p = 14 (s: ~3e-5)
    xr, wr = workloads.vortex_ring(6000, 9)
    qr = np.random.default_rng(9).normal(size=6000)
    ar = workloads.core_radius(6000)
    tg = workloads.sample_targets(6000, 300, seed=1)
    vd, sd = oracle.direct_adaptive(xr, wr, ar, 32, 7, targets=tg, q=qr)
    errs = []
    for p in (8, 14):
        v, s, _ = oracle.fmm_adaptive(xr, wr, ar, p, 32, 7, q=qr)
        errs.append(max(np.linalg.norm(v[tg] - vd) / np.linalg.norm(vd),
                        np.linalg.norm(s[tg] - sd) / np.linalg.norm(sd)))
    # sources of unit size dominate the ring's vortices here; their far field decays like 1/r^2
    assert errs[1] < errs[0] / 10 and errs[1] < 1e-3
