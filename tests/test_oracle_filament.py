"""Pins of the oracle's vortex-filament operators (Sec. 5.3, App. B), CPU only.

Straight segments of constant circulation, receivers at the vertices.  The closed form of the
segment velocity (eq. dis2) is pinned against a high-order quadrature of the Biot-Savart line
integral (eq. dis1); the Gauss-Legendre rule against the library routine and polynomial
exactness; the quadrature P2M's exactness claim (eq. vf7) by comparison with a much higher
quadrature order; the filament FMM by geometric convergence to the direct sum and by the split
into far and near parts.
"""
import numpy as np

import workloads


def _line_integral(y, x1, x2, G, nq=200):
    # G int dl x (y - x) / |y - x|^3 over the segment (no 1/(4 pi)), composite Gauss-Legendre
    xi, w = np.polynomial.legendre.leggauss(40)
    l = x2 - x1
    v = np.zeros(3)
    for k in range(nq // 40 + 1):
        a, b = k / (nq // 40 + 1), (k + 1) / (nq // 40 + 1)
        t = 0.5 * (a + b) + 0.5 * (b - a) * xi
        x = x1[None, :] + t[:, None] * l[None, :]
        r = y[None, :] - x
        rn = np.linalg.norm(r, axis=1)
        v += (0.5 * (b - a) * w[:, None] * np.cross(l[None, :], r) / rn[:, None] ** 3).sum(0)
    return G * v


def test_segment_closed_form_against_the_line_integral(oracle):
    rng = np.random.default_rng(51)
    X = rng.uniform(0, 1, (6, 3))
    seg = np.array([[0, 1], [2, 3]], np.int32)
    G = np.array([1.3, -0.7])
    for y_idx in (4, 5):
        v = oracle.filament_direct(X, seg, G, targets=[y_idx])[0]
        ref = _line_integral(X[y_idx], X[0], X[1], G[0]) + _line_integral(X[y_idx], X[2], X[3], G[1])
        assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()
    # a vertex of a segment gets nothing from it; a far short segment is a point vortex G l
    X2 = np.array([[0.0, 0, 0], [1e-3, 0, 0], [0.3, 0.4, 0.0], [1.0, 1.0, 1.0]])
    v = oracle.filament_direct(X2, np.array([[0, 1]], np.int32), np.array([2.0]))
    assert np.all(v[0] == 0.0) and np.all(v[1] == 0.0)
    r = X2[2] - np.array([5e-4, 0, 0])
    pv = 2.0 * np.cross(np.array([1e-3, 0, 0]), r) / np.linalg.norm(r) ** 3
    assert np.abs(v[2] - pv).max() <= 1e-5 * np.abs(pv).max()


def test_gauss_legendre(oracle):
    for nq in (1, 2, 5, 12):
        xi, w = oracle.gauss_legendre(nq)
        xr, wr = np.polynomial.legendre.leggauss(nq)
        o = np.argsort(xi)
        assert np.abs(xi[o] - xr).max() < 1e-14 and np.abs(w[o] - wr).max() < 1e-14
        # exact for degree 2 nq - 1
        for d in range(2 * nq):
            exact = 0.0 if d % 2 else 2.0 / (d + 1)
            assert abs((w * xi ** d).sum() - exact) < 1e-13


def test_quadrature_p2m_is_exact_at_vf7(oracle):
    # the filament FMM's far field with N_q = floor((p-1)/2) + 1 equals that with 24 points
    X, seg, G = workloads.filament_rings(20, 40, 52)
    for p in (6, 11):
        v1, _ = oracle.filament_fmm(X, seg, G, p, 3, near=False)
        v2, _ = oracle.filament_fmm(X, seg, G, p, 3, nq=24, near=False)
        assert np.abs(v1 - v2).max() <= 1e-12 * np.abs(v2).max()
    # at p = 6 one point fewer is no longer exact (the terms of degree 2 N_q in the abscissa are
    # visible for these segments; at higher orders they fall below rounding)
    v2, _ = oracle.filament_fmm(X, seg, G, 6, 3, nq=24, near=False)
    v3, _ = oracle.filament_fmm(X, seg, G, 6, 3, nq=2, near=False)
    assert np.abs(v3 - v2).max() > 1e-9 * np.abs(v2).max()


def test_filament_fmm_converges_to_the_direct_sum(oracle):
    X, seg, G = workloads.filament_rings(60, 50, 53)
    vd = oracle.filament_direct(X, seg, G)
    errs = []
    for p in (4, 8, 12, 16):
        v, st = oracle.filament_fmm(X, seg, G, p, 3)
        errs.append(np.linalg.norm(v - vd) / np.linalg.norm(vd))
    assert all(errs[i + 1] < errs[i] / 4 for i in range(3)), errs
    assert errs[-1] < 1e-6
    vf, _ = oracle.filament_fmm(X, seg, G, 8, 3, near=False)
    vn, _ = oracle.filament_fmm(X, seg, G, 8, 3, far=False)
    v, _ = oracle.filament_fmm(X, seg, G, 8, 3)
    assert np.abs(vf + vn - v).max() <= 1e-13 * np.abs(v).max()
