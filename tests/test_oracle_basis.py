"""Pins of the oracle's basis functions and smoothing kernel (CPU only).

Each check compares against something other than the oracle's own formula:
closed forms on the z axis, the R<->S relation, the Green's-function expansion,
harmonicity and the derivative relations by finite differences, a library
Legendre routine, and numerical quadrature of the core integral.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import idx


def test_axis_closed_forms(oracle):
    # On the +z axis P_n^0(1) = 1 and P_n^m(1) = 0 (m > 0), so eq. rsbf2 gives
    # R_n^0 = (-t)^n / n!, S_n^0 = n! / t^(n+1) and zero for m != 0.
    t = 0.7
    R = oracle.basis_R(12, [0, 0, t])
    S = oracle.basis_S(12, [0, 0, t])
    for n in range(12):
        assert R[idx(n, 0)] == pytest.approx((-t) ** n / math.factorial(n), rel=1e-14)
        assert S[idx(n, 0)] == pytest.approx(math.factorial(n) / t ** (n + 1), rel=1e-14)
        for m in range(1, n + 1):
            assert abs(R[idx(n, m)]) < 1e-300 and abs(S[idx(n, -m)]) < 1e-300


def test_legendre_against_scipy(oracle):
    # Legendre functions with the Condon-Shortley phase (eq. rsbf3) vs scipy.special.lpmv,
    # extracted from R on the unit sphere: P_n^|m| = R_n^m (n+|m|)! (-1)^n / (i^|m| e^{i m phi}).
    rng = np.random.default_rng(3)
    for _ in range(5):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        mu, ph = v[2], math.atan2(v[1], v[0])
        R = oracle.basis_R(15, v)
        for n in range(15):
            for m in range(-n, n + 1):
                am = abs(m)
                P = R[idx(n, m)] * math.factorial(n + am) * (-1) ** n / (1j ** am * np.exp(1j * m * ph))
                assert P.real == pytest.approx(special.lpmv(am, n, mu), rel=1e-11, abs=1e-11)
                assert abs(P.imag) < 1e-9 * max(1.0, abs(P.real))


def test_R_S_relation(oracle):
    # eq. rsbf4: S_n^m = (-1)^(n+m) (n-m)! (n+m)! r^(-2n-1) R_n^m
    r = np.array([0.3, -0.4, 0.5])
    rr = np.linalg.norm(r)
    R = oracle.basis_R(14, r)
    S = oracle.basis_S(14, r)
    for n in range(14):
        for m in range(-n, n + 1):
            ref = (-1) ** (n + m) * math.factorial(n - m) * math.factorial(n + m) * rr ** (-2 * n - 1) * R[idx(n, m)]
            assert abs(S[idx(n, m)] - ref) <= 1e-13 * abs(ref) + 1e-300


def test_green_expansion(oracle):
    # eq. rsbf5: 1/|r - r0| = sum R_n^{-m}(-r0) S_n^m(r), r > r0; converges geometrically
    r0 = np.array([0.12, -0.2, 0.16])
    r = np.array([0.7, 0.45, -0.55])
    exact = 1.0 / np.linalg.norm(r - r0)
    errs = []
    for nmax in (5, 10, 20, 30):
        Rm = oracle.basis_R(nmax, -r0)
        S = oracle.basis_S(nmax, r)
        acc = sum(Rm[idx(n, -m)] * S[idx(n, m)] for n in range(nmax) for m in range(-n, n + 1))
        assert abs(acc.imag) < 1e-14
        errs.append(abs(acc.real - exact) / exact)
    assert errs[-1] < 1e-13
    assert errs[0] > errs[1] > errs[2]


def _fd_grad(fun, y, h=1e-5):
    g = np.zeros(3, complex)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        g[d] = (fun(y + e) - fun(y - e)) / (2 * h)
    return g


@pytest.mark.parametrize("kind", ["R", "S"])
def test_harmonic_and_derivative_relations(oracle, kind):
    # Laplacian = 0 (finite differences) and the relations of eq. mr4:
    # D_z F_n^m = -F_{n-/+1}^m, D_{x+iy} F_n^m = i F_{n-/+1}^{m+1}, D_{x-iy} F_n^m = i F_{n-/+1}^{m-1}
    nmax = 9
    basis = oracle.basis_R if kind == "R" else oracle.basis_S
    y0 = np.array([0.35, -0.25, 0.3]) if kind == "R" else np.array([0.9, -0.7, 0.8])
    F0 = basis(nmax + 1, y0)
    sh = -1 if kind == "R" else +1
    for n in range(1, nmax - 1):
        for m in range(-n, n + 1):
            f = lambda y: basis(nmax + 1, y)[idx(n, m)]
            g = _fd_grad(f, y0)
            h = 1e-3
            lap = sum((f(y0 + h * e) - 2 * f(y0) + f(y0 - h * e)) / h ** 2 for e in np.eye(3))
            scale = max(abs(F0[idx(n, m)]), 1e-30) / np.linalg.norm(y0) ** 2
            assert abs(lap) < 1e-4 * scale * (n + 1) ** 2
            nn = n + sh
            get = lambda mm: F0[idx(nn, mm)] if abs(mm) <= nn else 0.0
            tol = 1e-6 * (abs(g).max() + 1e-30)
            assert abs(g[2] - (-get(m))) < tol
            assert abs((g[0] + 1j * g[1]) - 1j * get(m + 1)) < tol
            assert abs((g[0] - 1j * g[1]) - 1j * get(m - 1)) < tol


def test_conjugate_symmetry(oracle):
    # real harmonic functions: F_n^{-m} = (-1)^m conj(F_n^m) for both bases
    r = np.array([-0.31, 0.52, 0.27])
    for F in (oracle.basis_R(10, r), oracle.basis_S(10, r)):
        for n in range(10):
            for m in range(1, n + 1):
                assert abs(F[idx(n, -m)] - (-1) ** m * np.conj(F[idx(n, m)])) <= 1e-14 * abs(F[idx(n, m)])


def test_gaussian_core_against_quadrature(oracle):
    # eq. vem1: K(r) = sqrt(2/pi)/a^3 int_0^r s^2 exp(-s^2/2a^2) ds  (derivative of vem1);
    # f = K/r^3, and g = f'/r checked by finite differences of f.
    a = 0.05
    c = math.sqrt(2 / math.pi)
    for r in (1e-4, 1e-3, 0.005, 0.0099, 0.0101, 0.02, 0.05, 0.1, 0.3):
        K, _ = integrate.quad(lambda s: c / a ** 3 * s * s * math.exp(-s * s / (2 * a * a)), 0, r,
                              epsabs=0, epsrel=1e-13)
        f, g = oracle.kernel_fg(r, a, True)
        assert f == pytest.approx(K / r ** 3, rel=1e-12)
        h = 1e-6 * max(r, a)
        fp, _ = oracle.kernel_fg(r + h, a, True)
        fm, _ = oracle.kernel_fg(r - h, a, True) if r > h else (None, None)
        if fm is not None:
            assert g == pytest.approx((fp - fm) / (2 * h) / r, rel=1e-5)
    # r = 0 limits: f(0) = sqrt(2/pi)/(3a^3), g(0) = -sqrt(2/pi)/(5a^5)
    f0, g0 = oracle.kernel_fg(0.0, a, True)
    assert f0 == pytest.approx(c / (3 * a ** 3), rel=1e-15)
    assert g0 == pytest.approx(-c / (5 * a ** 5), rel=1e-15)
    # far from the core the kernel is the singular one (eq. 2: K = 1 + O(eps), r >> a)
    f, g = oracle.kernel_fg(10 * a, a, True)
    fs, gs = oracle.kernel_fg(10 * a, a, False)
    assert f == pytest.approx(fs, rel=1e-20 + 1e-15) and g == pytest.approx(gs, rel=1e-14)


def test_series_branch_is_continuous(oracle):
    # the Taylor branch (u < 0.02, i.e. r < 0.2a) meets the closed form
    a = 1.0
    r0 = math.sqrt(0.02 * 2) * a
    f1, g1 = oracle.kernel_fg(r0 * (1 - 1e-12), a, True)
    f2, g2 = oracle.kernel_fg(r0 * (1 + 1e-12), a, True)
    assert f1 == pytest.approx(f2, rel=1e-13)
    assert g1 == pytest.approx(g2, rel=1e-12)
