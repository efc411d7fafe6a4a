"""Host check of the sign relation the quarter-vector M2L uses to run the polar angle pi - theta on
the staged rotation table of theta.

The library builds its rotation about y as U = exp(-theta G), G the real skew generator of
D_{r x e_y} in the orthonormal basis (the same matrix entries as the device table builder), then
rescales U into the S- or R-basis blocks of the scaled bar coefficients and splits them into the
blocks acting on real and on imaginary parts.  The kernel relies on, per order n,
    Re block: W(pi - theta)[m'][m] =  (-1)^(n + m + m') W(theta)[m'][m]
    Im block: W(pi - theta)[m'][m] = -(-1)^(n + m + m') W(theta)[m'][m]
for the forward and the backward tables of both bases.  This test evaluates the construction
independently on the CPU (scipy's matrix exponential) and checks the relation, and that it is not
trivially true (the blocks of theta and pi - theta differ)."""
from math import factorial, sqrt

import numpy as np
import pytest
from scipy.linalg import expm


def generator(n):
    """G[m][m'] (m, m' = -n..n): nonzero for m' = m +- 1"""
    D = 2 * n + 1
    G = np.zeros((D, D))
    for i in range(D):
        m = i - n
        for mp in (m - 1, m + 1):
            if abs(mp) > n:
                continue
            if mp == m - 1:
                if m >= 1:
                    v = 0.5 * sqrt((n + m) * (n - m + 1))
                elif m == 0:
                    v = -0.5 * sqrt(n * (n + 1))
                else:
                    v = -0.5 * sqrt((n - m + 1) * (n + m))
            else:
                if m >= 1:
                    v = -0.5 * sqrt((n - m) * (n + m + 1))
                elif m == 0:
                    v = -0.5 * sqrt(n * (n + 1))
                else:
                    v = 0.5 * sqrt((n + m + 1) * (n - m))
            G[i, mp + n] = v
    return G


def blocks(n, theta, sbasis, back):
    """(Re, Im) blocks of one order: Re[m'][m] for m, m' = 0..n, Im[m'][m] for m, m' = 1..n"""
    U = expm(-theta * generator(n))
    N = lambda m: sqrt(factorial(n - abs(m)) * factorial(n + abs(m)))

    def hb(m, mp):
        u = U[mp + n, m + n] if back else U[m + n, mp + n]
        if sbasis:
            return (-1) ** (m + mp) * u * N(m) / N(mp)
        return u * N(mp) / N(m)

    re = np.array([[hb(0, mp) if m == 0 else hb(m, mp) + hb(-m, mp) for m in range(n + 1)] for mp in range(n + 1)])
    im = np.array([[hb(m, mp) - hb(-m, mp) for m in range(1, n + 1)] for mp in range(1, n + 1)])
    return re, im


@pytest.mark.parametrize("n", [1, 2, 3, 6, 11, 16, 22])
@pytest.mark.parametrize("theta", [np.arccos(1 / np.sqrt(3)), np.arccos(2 / 3), np.arccos(3 / np.sqrt(22)),
                                   np.arccos(3 / np.sqrt(10))])
def test_mirror_signs(n, theta):
    _check(n, theta)


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_mirror_signs_axis(n):
    # theta = 0 against theta = pi (the z axis and its reverse); low orders only: the reference
    # exponential at theta = pi loses digits that the S-basis rescaling amplifies at high n
    _check(n, 0.0)


def _check(n, theta):
    for sbasis in (True, False):
        for back in (False, True):
            re, im = blocks(n, theta, sbasis, back)
            rm, imm = blocks(n, np.pi - theta, sbasis, back)
            mp, m = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
            sre = (-1.0) ** (n + m + mp)
            mpi, mi = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), indexing="ij")
            sim = -((-1.0) ** (n + mi + mpi))
            scale = max(np.abs(re).max(), np.abs(im).max() if n else 0.0)
            assert np.abs(rm - sre * re).max() <= 1e-11 * scale
            if n:
                assert np.abs(imm - sim * im).max() <= 1e-11 * scale
            if n >= 1 and 0.0 < theta < np.pi / 2:
                # the relation is not the identity: the two tables differ (at theta = 0 the blocks
                # are diagonal and, for even n, the signs on the diagonal are all +1)
                assert np.abs(rm - re).max() > 1e-6 * scale
