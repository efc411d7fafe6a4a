"""Pins of the oracle's direct sums (eqs. 1, 2, s1.1, vem1), CPU only."""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")


def test_single_vortex_by_hand(oracle):
    pin = json.load(open(GOLDEN))["single_vortex_by_hand"]
    x = np.array([pin["source"], pin["target"]])
    w = np.array([pin["omega"], pin["omega_target"]])
    v, s = oracle.direct(x, w, 0.0, mode=oracle.DIRECT_SINGULAR, targets=[1])
    np.testing.assert_allclose(v[0], pin["v"], atol=1e-15)
    np.testing.assert_allclose(s[0], pin["s"], atol=1e-15)


@pytest.mark.parametrize("mode", [0, 1])
def test_stretching_is_directional_derivative(oracle, mode):
    # s_j = (omega_j . grad) v at x_j (eq. s1.1), checked by moving the receiver
    rng = np.random.default_rng(7)
    n = 40
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.08
    j = 5
    v, s, g = oracle.direct(x, w, a, mode=mode, targets=[j], grad=True)
    h = 1e-6
    G = np.zeros((3, 3))
    for l in range(3):
        xp, xm = x.copy(), x.copy()
        xp[j, l] += h
        xm[j, l] -= h
        vp, _ = oracle.direct(xp, w, a, mode=mode, targets=[j])
        vm, _ = oracle.direct(xm, w, a, mode=mode, targets=[j])
        G[:, l] = (vp[0] - vm[0]) / (2 * h)
    np.testing.assert_allclose(g[0], G, rtol=1e-6, atol=1e-6 * np.abs(G).max())
    np.testing.assert_allclose(s[0], G @ w[j], rtol=1e-6, atol=1e-6 * np.abs(s).max())
    # divergence free (eq. 3): trace of grad v vanishes identically
    assert abs(np.trace(g[0])) < 1e-12 * np.abs(g[0]).max()


def test_scaling_linearity_rotation(oracle):
    rng = np.random.default_rng(8)
    n = 60
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.1
    v, s = oracle.direct(x, w, a, mode=oracle.DIRECT_SMOOTH)
    lam = 2.5
    v2, s2 = oracle.direct(lam * x, w, lam * a, mode=oracle.DIRECT_SMOOTH)
    np.testing.assert_allclose(v2, v / lam ** 2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(s2, s / lam ** 3, rtol=1e-12, atol=1e-14)
    al = -1.7
    v3, s3 = oracle.direct(x, al * w, a, mode=oracle.DIRECT_SMOOTH)
    np.testing.assert_allclose(v3, al * v, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(s3, al * al * s, rtol=1e-13, atol=1e-12)
    # proper rotation Q: v -> Q v, s -> Q s
    A = rng.normal(size=(3, 3))
    Q, _ = np.linalg.qr(A)
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    v4, s4 = oracle.direct(x @ Q.T, w @ Q.T, a, mode=oracle.DIRECT_SMOOTH)
    np.testing.assert_allclose(v4, v @ Q.T, rtol=1e-11, atol=1e-11 * np.abs(v).max())
    np.testing.assert_allclose(s4, s @ Q.T, rtol=1e-11, atol=1e-11 * np.abs(s).max())


def test_coincident_points(oracle):
    # distinct elements at the same place: Gaussian core gives v-term 0 and
    # s-term f(0) w_i x w_j with f(0) = sqrt(2/pi)/(3a^3); singular kernel: defined as 0
    a = 0.2
    x = np.zeros((2, 3))
    w = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    v, s = oracle.direct(x, w, a, mode=oracle.DIRECT_SMOOTH, targets=[1])
    f0 = math.sqrt(2 / math.pi) / (3 * a ** 3)
    np.testing.assert_allclose(v[0], 0.0, atol=0)
    np.testing.assert_allclose(s[0], f0 * np.cross(w[0], w[1]), rtol=1e-15)
    v, s = oracle.direct(x, w, 0.0, mode=oracle.DIRECT_SINGULAR, targets=[1])
    assert np.all(v == 0) and np.all(s == 0)


def test_split_mode_matches_pairwise_rule(oracle):
    # split kernel: smoothed iff the leaves (depth d) of source and target are adjacent
    rng = np.random.default_rng(9)
    n = 80
    x = rng.uniform(0, 1, (n, 3))
    w = rng.normal(size=(n, 3))
    a = 0.05
    d = 2
    vs, ss = oracle.direct(x, w, a, mode=oracle.DIRECT_SPLIT, depth=d)
    leaf = np.floor(x * 2 ** d).astype(int)
    for j in (0, 17, 41):
        vv = np.zeros(3)
        s_ = np.zeros(3)
        for i in range(n):
            if i == j:
                continue
            adj = np.all(np.abs(leaf[i] - leaf[j]) <= 1)
            xx = np.array([x[i], x[j]])
            ww = np.array([w[i], w[j]])
            v1, s1 = oracle.direct(xx, ww, a, mode=1 if adj else 0, targets=[1])
            vv += v1[0]
            s_ += s1[0]
        np.testing.assert_allclose(vs[j], vv, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(ss[j], s_, rtol=1e-13, atol=1e-12)
