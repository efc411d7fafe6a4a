"""Python access to the FP64 CPU oracle (``oracle/lhf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP path (see the header of ``lhf_oracle.c`` for
what is computed and which passage of the paper each routine follows).

Every array crossing this wrapper is a contiguous float64 (or complex128)
numpy array; points and strengths are ``[N, 3]`` row-major.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lhf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_lhf_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_cp = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
               "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Stats(C.Structure):
    _fields_ = [("n_m2l", C.c_int64), ("n_m2m", C.c_int64), ("n_l2l", C.c_int64),
                ("n_p2p_pairs", C.c_int64), ("t_tree", C.c_double), ("t_up", C.c_double),
                ("t_down", C.c_double), ("t_near", C.c_double), ("n_wx_pairs", C.c_int64),
                ("n_leaf", C.c_int64), ("n_box", C.c_int64), ("max_level", C.c_int32),
                ("reserved", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.lho_basis_R.argtypes = [C.c_int, _dp, _cp]
        L.lho_basis_S.argtypes = [C.c_int, _dp, _cp]
        L.lho_kernel_fg.argtypes = [C.c_double, C.c_double, C.c_int, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
        L.lho_p2m_method1.argtypes = [C.c_int, _dp, C.c_int64, _dp, _dp, _cp, _cp]
        L.lho_p2m_method2.argtypes = [C.c_int, _dp, C.c_int64, _dp, _dp, C.c_void_p, _cp, _cp]
        for nm in ("lho_m2m", "lho_m2l", "lho_l2l"):
            getattr(L, nm).argtypes = [C.c_int, _dp, _cp, _cp, _cp, _cp]
        L.lho_l2p.argtypes = [C.c_int, _dp, _cp, _cp, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.lho_direct.argtypes = [C.c_int64, _dp, _dp, C.c_void_p, C.c_double, C.c_int, C.c_int, _dp, C.c_double,
                                 C.c_int64, C.c_void_p, _dp, _dp, C.c_void_p]
        L.lho_fmm.argtypes = [C.c_int64, _dp, _dp, C.c_void_p, C.c_double, C.c_int, C.c_int, _dp, C.c_double,
                              C.c_int, C.c_int, C.c_int64, C.c_void_p, _dp, _dp, C.c_void_p,
                              C.POINTER(_Stats)]
        L.lho_fmm.restype = C.c_int
        L.lho_tree_counts.argtypes = [C.c_int64, _dp, C.c_int, _dp, C.c_double, _ip,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lho_num_threads.restype = C.c_int
        L.lho_fmm_adaptive.argtypes = [C.c_int64, _dp, _dp, C.c_void_p, C.c_double, C.c_int, C.c_int64, C.c_int,
                                       _dp, C.c_double, C.c_int, C.c_int64, C.c_void_p, _dp, _dp, C.c_void_p,
                                       C.c_int, C.POINTER(_Stats)]
        L.lho_p2l.argtypes = [C.c_int, _dp, C.c_int64, _dp, _dp, C.c_void_p, _cp, _cp]
        L.lho_m2p.argtypes = [C.c_int, _dp, _cp, _cp, C.c_int64, _dp, _dp, _dp, _dp, C.c_void_p]
        L.lho_fmm_adaptive.restype = C.c_int
        L.lho_direct_adaptive.argtypes = [C.c_int64, _dp, _dp, C.c_void_p, C.c_double, C.c_int64, C.c_int, _dp,
                                          C.c_double, C.c_int64, C.c_void_p, _dp, _dp]
        L.lho_adaptive_coverage.argtypes = [C.c_int64, _dp, C.c_int64, C.c_int, _dp, C.c_double,
                                            C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lho_adaptive_counts.argtypes = [C.c_int64, _dp, C.c_int64, C.c_int, _dp, C.c_double, _ip, _ip]
        L.lho_scalar_direct.argtypes = [C.c_int64, _dp, _dp, C.c_int64, C.c_void_p, _dp, _dp]
        L.lho_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        L.lho_filament_direct.argtypes = [C.c_int64, _dp, C.c_int64, _i32p, _dp, C.c_int64, C.c_void_p, _dp]
        L.lho_filament_fmm.argtypes = [C.c_int64, _dp, C.c_int64, _i32p, _dp, C.c_int, C.c_int, _dp, C.c_double,
                                       C.c_int, C.c_int, _dp, C.POINTER(_Stats)]
        L.lho_filament_fmm.restype = C.c_int
        L.lho_fmm_scalar.argtypes = [C.c_int64, _dp, _dp, C.c_int, C.c_int, _dp, C.c_double, C.c_int, C.c_int64,
                                     C.c_void_p, _dp, _dp, C.POINTER(_Stats)]
        L.lho_fmm_scalar.restype = C.c_int
        _lib = L
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return int(lib().lho_num_threads())


def idx(n: int, m: int) -> int:
    """storage index of coefficient (n, m)"""
    return n * n + n + m


def basis_R(nmax: int, r) -> np.ndarray:
    out = np.zeros(nmax * nmax, np.complex128)
    lib().lho_basis_R(nmax, _f64(r, (3,)), out)
    return out


def basis_S(nmax: int, r) -> np.ndarray:
    out = np.zeros(nmax * nmax, np.complex128)
    lib().lho_basis_S(nmax, _f64(r, (3,)), out)
    return out


def kernel_fg(r: float, a: float, smooth: bool = True):
    f, g = C.c_double(), C.c_double()
    lib().lho_kernel_fg(float(r), float(a), int(bool(smooth)), C.byref(f), C.byref(g))
    return f.value, g.value


def _qptr(q, n):
    """monopole strengths as a float64 array of n entries and its address (None: no monopoles)"""
    if q is None:
        return None, None
    q = _f64(q).reshape(-1)
    if q.shape[0] != n:
        raise ValueError("q must have one entry per element")
    return q, q.ctypes.data


def p2m(p: int, centre, x, w, method: int = 2, q=None):
    """(phi, chi) multipole coefficients about centre (eq. eve4 / eqs. eve5-eve10); with q,
    monopole strengths added to phi (method 2 only)."""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    phi = np.zeros(p * p, np.complex128)
    chi = np.zeros(p * p, np.complex128)
    if method == 2:
        qa, qp = _qptr(q, x.shape[0])
        lib().lho_p2m_method2(p, _f64(centre, (3,)), x.shape[0], x, w, qp, phi, chi)
    else:
        if q is not None:
            raise ValueError("monopoles: method 2 only")
        lib().lho_p2m_method1(p, _f64(centre, (3,)), x.shape[0], x, w, phi, chi)
    return phi, chi


def _translate(fn, p, t, phi, chi):
    oph = np.zeros(p * p, np.complex128)
    och = np.zeros(p * p, np.complex128)
    fn(p, _f64(t, (3,)), np.ascontiguousarray(phi, np.complex128),
       np.ascontiguousarray(chi, np.complex128), oph, och)
    return oph, och


def m2m(p, t, phi, chi):
    return _translate(lib().lho_m2m, p, t, phi, chi)


def m2l(p, t, phi, chi):
    return _translate(lib().lho_m2l, p, t, phi, chi)


def l2l(p, t, phi, chi):
    return _translate(lib().lho_l2l, p, t, phi, chi)


def l2p(p, centre, phi, chi, x, w):
    """Evaluate a local expansion: returns v, s, grad v, Im v, Im grad v."""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    n = x.shape[0]
    v = np.zeros((n, 3)); s = np.zeros((n, 3)); g = np.zeros((n, 9))
    iv = np.zeros((n, 3)); ig = np.zeros((n, 9))
    lib().lho_l2p(p, _f64(centre, (3,)), np.ascontiguousarray(phi, np.complex128),
                  np.ascontiguousarray(chi, np.complex128), n, x, w, v, s, g, iv, ig)
    return v, s, g.reshape(n, 3, 3), iv, ig.reshape(n, 3, 3)


DIRECT_SINGULAR, DIRECT_SMOOTH, DIRECT_SPLIT = 0, 1, 2


def direct(x, w, a, mode=DIRECT_SPLIT, depth=2, lo=(0.0, 0.0, 0.0), L=1.0, targets=None,
           grad=False, q=None):
    """Direct O(N |targets|) sums of v, s (and grad v) -- eqs. 1, 2, s1.1, vem1.

    mode: DIRECT_SINGULAR (K=1), DIRECT_SMOOTH (Gaussian everywhere) or
    DIRECT_SPLIT (Gaussian between adjacent leaves of the depth-``depth``
    octree on [lo, lo+L]^3, singular otherwise)."""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, np.int64)
        nt, tp = targets.shape[0], targets.ctypes.data
    v = np.zeros((nt, 3)); s = np.zeros((nt, 3))
    g = np.zeros((nt, 9)) if grad else None
    qa, qp = _qptr(q, n)
    lib().lho_direct(n, x, w, qp, float(a), int(mode), int(depth), _f64(lo, (3,)), float(L), nt, tp, v, s,
                     g.ctypes.data if grad else None)
    return (v, s, g.reshape(nt, 3, 3)) if grad else (v, s)


def fmm(x, w, a, p, depth, lo=(0.0, 0.0, 0.0), L=1.0, far=True, near=True, p2m_method=2,
        sample=None, grad=False, q=None):
    """Plain FP64 two-potential FMM (direct-mode translations).

    With ``sample`` (element indices), only the leaves holding those elements
    are evaluated; the outputs of the other elements are NaN."""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    n = x.shape[0]
    v = np.zeros((n, 3)); s = np.zeros((n, 3))
    g = np.zeros((n, 9)) if grad else None
    if sample is None:
        ns, sp = 0, None
    else:
        sample = np.ascontiguousarray(sample, np.int64)
        ns, sp = sample.shape[0], sample.ctypes.data
    st = _Stats()
    what = (1 if far else 0) | (2 if near else 0)
    qa, qp = _qptr(q, n)
    rc = lib().lho_fmm(n, x, w, qp, float(a), int(p), int(depth), _f64(lo, (3,)), float(L), what,
                       int(p2m_method), ns, sp, v, s, g.ctypes.data if grad else None, C.byref(st))
    if rc != 0:
        raise ValueError("oracle fmm rejected its arguments")
    if sample is not None:
        # mark untouched outputs
        mask = np.zeros(n, bool)
        mask[_leaf_members(x, depth, lo, L, sample)] = True
        v[~mask] = np.nan
        s[~mask] = np.nan
        if grad:
            g[~mask] = np.nan
    stats = dict(n_m2l=st.n_m2l, n_l2l=st.n_l2l, n_p2p_pairs=st.n_p2p_pairs, t_tree=st.t_tree,
                 t_up=st.t_up, t_down=st.t_down, t_near=st.t_near)
    out = (v, s, g.reshape(n, 3, 3)) if grad else (v, s)
    return out + (stats,)


def _leaf_coords(x, depth, lo, L):
    scale = float(2 ** 21) / L
    q = np.floor((x - np.asarray(lo)[None, :]) * scale)
    q = np.clip(q, 0, 2 ** 21 - 1).astype(np.int64)
    return q >> (21 - depth)


def _leaf_members(x, depth, lo, L, sample):
    lc = _leaf_coords(x, depth, lo, L)
    keys = lc[:, 0] * (1 << 42) + lc[:, 1] * (1 << 21) + lc[:, 2]
    return np.isin(keys, np.unique(keys[sample]))


def tree_counts(x, depth, lo=(0.0, 0.0, 0.0), L=1.0):
    x = _f64(x).reshape(-1, 3)
    nb = np.zeros(depth + 1, np.int64)
    a, b = C.c_int64(), C.c_int64()
    lib().lho_tree_counts(x.shape[0], x, int(depth), _f64(lo, (3,)), float(L), nb, C.byref(a), C.byref(b))
    return nb, a.value, b.value


def p2l(p, centre, x, w, q=None):
    """local (phi, chi) expansion about centre of the field of elements outside its ball"""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    phi = np.zeros(p * p, np.complex128)
    chi = np.zeros(p * p, np.complex128)
    qa, qp = _qptr(q, x.shape[0])
    lib().lho_p2l(p, _f64(centre, (3,)), x.shape[0], x, w, qp, phi, chi)
    return phi, chi


def m2p(p, centre, phi, chi, y, w):
    """v, s, grad v at targets y (strengths w) of a multipole expansion about centre"""
    y = _f64(y).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    n = y.shape[0]
    v = np.zeros((n, 3)); s = np.zeros((n, 3)); g = np.zeros((n, 9))
    lib().lho_m2p(p, _f64(centre, (3,)), np.ascontiguousarray(phi, np.complex128),
                  np.ascontiguousarray(chi, np.complex128), n, y, w, v, s, g.ctypes.data)
    return v, s, g.reshape(n, 3, 3)


def fmm_adaptive(x, w, a, p, max_per_leaf=64, max_level=10, lo=(0.0, 0.0, 0.0), L=1.0, far=True, near=True,
                 sample=None, grad=False, q=None, wx_expansions=False):
    """Adaptive-octree FMM (split while a box holds more than max_per_leaf elements, down to
    max_level); W/X interactions summed directly with the singular kernel.  With ``sample``
    only the leaves holding those elements are evaluated (other outputs NaN).  With ``grad``
    also grad v ([N,3,3], [i,k,l] = d v_k / d x_l) is returned after s.  With ``wx_expansions``
    the W boxes act by M2P and the X sources by P2L (both part of the far field) instead of
    direct singular sums (near field); boxes above level 2 keep the direct sums."""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    n = x.shape[0]
    v = np.zeros((n, 3)); s = np.zeros((n, 3))
    g = np.zeros((n, 9)) if grad else None
    if sample is None:
        ns, sp = 0, None
    else:
        sample = np.ascontiguousarray(sample, np.int64)
        ns, sp = sample.shape[0], sample.ctypes.data
    st = _Stats()
    what = (1 if far else 0) | (2 if near else 0)
    qa, qp = _qptr(q, n)
    rc = lib().lho_fmm_adaptive(n, x, w, qp, float(a), int(p), int(max_per_leaf), int(max_level), _f64(lo, (3,)),
                                float(L), what, ns, sp, v, s, g.ctypes.data if grad else None,
                                int(bool(wx_expansions)), C.byref(st))
    if rc != 0:
        raise ValueError("oracle adaptive fmm rejected its arguments")
    if sample is not None:
        leaf = adaptive_leaf_of(x, max_per_leaf, max_level, lo, L)
        mask = np.isin(leaf, np.unique(leaf[sample]))
        v[~mask] = np.nan
        s[~mask] = np.nan
        if grad:
            g[~mask] = np.nan
    stats = dict(n_m2l=st.n_m2l, n_p2p_pairs=st.n_p2p_pairs, n_wx_pairs=st.n_wx_pairs, n_leaf=st.n_leaf,
                 n_box=st.n_box, max_level=st.max_level, t_tree=st.t_tree, t_up=st.t_up, t_down=st.t_down,
                 t_near=st.t_near)
    if grad:
        return v, s, g.reshape(n, 3, 3), stats
    return v, s, stats


def adaptive_leaf_of(x, max_per_leaf, max_level, lo=(0.0, 0.0, 0.0), L=1.0):
    """(level << 40) | cell index of the adaptive leaf holding each element (numpy, for sampling)"""
    q = np.clip(np.floor((np.asarray(x) - np.asarray(lo)[None, :]) * (float(2 ** 21) / L)), 0, 2 ** 21 - 1)
    q = q.astype(np.int64)
    out = np.full(q.shape[0], -1, np.int64)
    undecided = np.ones(q.shape[0], bool)
    for l in range(max_level + 1):
        c = q >> (21 - l)
        cell = (c[:, 0] << (2 * l)) | (c[:, 1] << l) | c[:, 2]
        _, inv, cnt = np.unique(cell, return_inverse=True, return_counts=True)
        stop = undecided & ((cnt[inv] <= max_per_leaf) | (l == max_level))
        out[stop] = (l << 40) | cell[stop]
        undecided &= ~stop
    return out


def direct_adaptive(x, w, a, max_per_leaf=64, max_level=10, lo=(0.0, 0.0, 0.0), L=1.0, targets=None, q=None):
    """Direct sums with the adaptive split rule (smoothed kernel between adjacent leaves)."""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, np.int64)
        nt, tp = targets.shape[0], targets.ctypes.data
    v = np.zeros((nt, 3)); s = np.zeros((nt, 3))
    qa, qp = _qptr(q, n)
    lib().lho_direct_adaptive(n, x, w, qp, float(a), int(max_per_leaf), int(max_level), _f64(lo, (3,)), float(L),
                              nt, tp, v, s)
    return v, s


def adaptive_coverage(x, max_per_leaf, max_level, lo=(0.0, 0.0, 0.0), L=1.0):
    """(min, max) number of mechanisms carrying each ordered leaf pair, and the leaf count"""
    x = _f64(x).reshape(-1, 3)
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    lib().lho_adaptive_coverage(x.shape[0], x, int(max_per_leaf), int(max_level), _f64(lo, (3,)), float(L),
                                C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def adaptive_counts(x, max_per_leaf, max_level, lo=(0.0, 0.0, 0.0), L=1.0):
    """boxes and leaves per level of the adaptive tree"""
    x = _f64(x).reshape(-1, 3)
    nb = np.zeros(max_level + 1, np.int64)
    nl = np.zeros(max_level + 1, np.int64)
    lib().lho_adaptive_counts(x.shape[0], x, int(max_per_leaf), int(max_level), _f64(lo, (3,)), float(L), nb, nl)
    return nb, nl


def scalar_direct(x, q, targets=None):
    """Direct sums of the scalar potential Phi_j = sum_{i != j} q_i / |x_j - x_i| and of grad Phi
    (singular kernel) at the targets (all elements when None): returns (phi [T], grad [T, 3])."""
    x = _f64(x).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    n = x.shape[0]
    if targets is None:
        nt, tp, m = 0, None, n
    else:
        targets = np.ascontiguousarray(targets, np.int64)
        nt, tp, m = targets.shape[0], targets.ctypes.data, targets.shape[0]
    phi = np.zeros(m)
    g = np.zeros((m, 3))
    lib().lho_scalar_direct(n, x, q, nt, tp, phi, g)
    return phi, g


def fmm_scalar(x, q, p, depth, lo=(0.0, 0.0, 0.0), L=1.0, far=True, near=True, sample=None):
    """Scalar harmonic FMM of Phi and grad Phi on the uniform octree (the single-potential
    comparison workload): returns (phi [N], grad [N, 3], stats); with ``sample`` only the leaves
    holding those elements are evaluated (other outputs NaN)."""
    x = _f64(x).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    n = x.shape[0]
    phi = np.zeros(n)
    g = np.zeros((n, 3))
    if sample is None:
        ns, sp = 0, None
    else:
        sample = np.ascontiguousarray(sample, np.int64)
        ns, sp = sample.shape[0], sample.ctypes.data
    st = _Stats()
    what = (1 if far else 0) | (2 if near else 0)
    rc = lib().lho_fmm_scalar(n, x, q, int(p), int(depth), _f64(lo, (3,)), float(L), what, ns, sp, phi, g,
                              C.byref(st))
    if rc != 0:
        raise ValueError("oracle scalar fmm rejected its arguments")
    if sample is not None:
        mask = np.zeros(n, bool)
        mask[_leaf_members(x, depth, lo, L, sample)] = True
        phi[~mask] = np.nan
        g[~mask] = np.nan
    return phi, g, dict(n_m2l=st.n_m2l, n_p2p_pairs=st.n_p2p_pairs)


def gauss_legendre(nq):
    """Gauss-Legendre nodes and weights on [-1, 1]"""
    xi = np.zeros(nq)
    w = np.zeros(nq)
    lib().lho_gauss_legendre(int(nq), xi, w)
    return xi, w


def _segs(seg):
    return np.ascontiguousarray(np.asarray(seg).reshape(-1, 2), np.int32)


def filament_direct(X, seg, G, targets=None):
    """velocity (eq. dis2, no 1/(4 pi)) of the straight segments seg [S, 2] (vertex indices) with
    circulations G at the vertices X (the targets' own segments skipped): [T, 3]"""
    X = _f64(X).reshape(-1, 3)
    seg = _segs(seg)
    G = _f64(G).reshape(-1)
    nv = X.shape[0]
    if targets is None:
        nt, tp, m = 0, None, nv
    else:
        targets = np.ascontiguousarray(targets, np.int64)
        nt, tp, m = targets.shape[0], targets.ctypes.data, targets.shape[0]
    v = np.zeros((m, 3))
    lib().lho_filament_direct(nv, X, seg.shape[0], seg, G, nt, tp, v)
    return v


def filament_fmm(X, seg, G, p, depth, lo=(0.0, 0.0, 0.0), L=1.0, nq=0, far=True, near=True):
    """FMM of the filament velocity at the vertices (tree on segment centres and vertices,
    quadrature P2M with nq points per segment, 0: floor((p-1)/2)+1): returns (v [V, 3], stats)"""
    X = _f64(X).reshape(-1, 3)
    seg = _segs(seg)
    G = _f64(G).reshape(-1)
    v = np.zeros((X.shape[0], 3))
    st = _Stats()
    what = (1 if far else 0) | (2 if near else 0)
    rc = lib().lho_filament_fmm(X.shape[0], X, seg.shape[0], seg, G, int(p), int(depth), _f64(lo, (3,)), float(L),
                                int(nq), what, v, C.byref(st))
    if rc != 0:
        raise ValueError("oracle filament fmm rejected its arguments")
    return v, dict(n_m2l=st.n_m2l, n_p2p_pairs=st.n_p2p_pairs)
