"""Pin of the oracle's M2L conversion and of the chi-hat order it needs (CPU only).

The Lamb-Helmholtz form v = grad phi + curl(r chi) (eq. 4) of a field expanded
in the regular basis about a centre is unique for orders n >= 1:

  * r . v = sum_n n phi_n         (the curl term is tangential), and
  * curl v = grad sum_n (n+1) chi_n   (for a harmonic chi_n of degree n,
    curl(grad chi_n x r) = 2 grad chi_n + (r.grad) grad chi_n = (n+1) grad chi_n).

For one vortex element at x0, v = curl(omega / |y - x0|), so
curl v = grad(omega . grad_y 1/|y - x0|).  The local coefficients of order n
are therefore the regular-basis coefficients of (y - c).v(y) divided by n and
of omega . grad_y 1/|y - x0| divided by n + 1.  These are fitted here by least
squares on points around the local centre, using only the (separately pinned)
regular basis, and compared with the oracle's M2L output (the translation of
eq. mr3 followed by the R-basis conversion of eq. drt10).

An element at the centre of its box has a multipole expansion with no
truncation error, so every local coefficient of order n <= p-1 that the M2L
returns must be exact.  The coefficient chi-tilde of order p-1 is formed from
chi-hat of order p; it is exact only if the M2L computes chi-hat to order p
before converting (the reading the oracle and the library both take where the
paper is silent).  Setting chi-hat of order p to zero instead changes that
coefficient at the 1e-2 level, far above the bar below.
"""
import numpy as np
import pytest


def _fit_regular(oracle, nfit, centre, pts, vals):
    """least-squares coefficients c_n^m with vals ~ sum c_n^m R_n^m(pts - centre)"""
    B = np.stack([oracle.basis_R(nfit, y - centre) for y in pts])
    scale = np.linalg.norm(B, axis=0)
    coef, *_ = np.linalg.lstsq(B / scale[None, :], vals.astype(np.complex128), rcond=None)
    return coef / scale


@pytest.mark.parametrize("p,t", [(4, (1.5, -2.0, 2.5)), (6, (2.0, -1.0, 3.0)), (9, (-3.0, 2.0, 2.0))])
def test_m2l_output_is_the_unique_decomposition(oracle, p, t):
    rng = np.random.default_rng(100 + p)
    cs = np.array([0.25, -0.5, 0.75])
    x0 = cs[None, :].copy()  # the element sits at the source centre
    w0 = np.array([[0.3, -0.5, 0.8]])
    ct = cs + np.asarray(t, float)
    phM, chM = oracle.p2m(p, cs, x0, w0)
    phL, chL = oracle.m2l(p, ct - cs, phM, chM)

    # sample points on a sphere of radius rho about the target centre
    rho, nfit, k = 0.6, p + 16, 1500
    u = rng.normal(size=(k, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    rad = rho * rng.uniform(0.5, 1.0, size=k) ** (1 / 3)
    pts = ct + u * rad[:, None]
    d = pts - x0[0]
    r3 = np.linalg.norm(d, axis=1) ** 3
    v = np.cross(w0[0], d) / r3[:, None]          # Biot-Savart, eq. 1 (singular)
    rv = np.einsum("ij,ij->i", pts - ct, v)       # (y - c) . v
    psi = -(d @ w0[0]) / r3                       # omega . grad_y 1/|y - x0|

    cphi = _fit_regular(oracle, nfit, ct, pts, rv)
    cpsi = _fit_regular(oracle, nfit, ct, pts, psi)
    scale = max(np.abs(phL).max(), np.abs(chL).max())
    for n in range(1, p):
        sl = slice(n * n, (n + 1) * (n + 1))
        ref_phi = cphi[sl] / n
        ref_chi = cpsi[sl] / (n + 1)
        assert np.abs(phL[sl] - ref_phi).max() < 1e-9 * scale, ("phi", n)
        assert np.abs(chL[sl] - ref_chi).max() < 1e-9 * scale, ("chi", n)
    # the top order is the one that needs chi-hat of order p: it must carry real content
    top = slice((p - 1) ** 2, p * p)
    assert np.abs(chL[top]).max() > 1e-6 * scale
