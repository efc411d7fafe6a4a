"""MI355X (gfx950) Lamb-Helmholtz vortex FMM: Python binding of liblhfmm.

The binding only marshals arguments: every step of the evaluation runs in the
HIP kernels of ``liblhfmm.so`` behind the C ABI declared in ``include/lhfmm.h``.
PyTorch supplies device memory (tensors) and the current HIP stream.  There is
no CPU fallback: if the library is missing, loading fails with an error.

    plan = Plan(x, a=0.005, p=12, depth=6)          # x: [N,3] cuda tensor
    v, s = plan.execute(omega)                      # omega: [N,3] cuda tensor
    v, s = evaluate(x, omega, a, p=12, depth=6)     # one shot
    plan = Plan(x, a, p=0, tol=1e-6, grad=True)     # order from tol; velocity gradient output
    v, s, g = plan.execute(omega, grad=True)        # g: [N,3,3], g[i,k,l] = d v_k / d x_l
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblhfmm.so")

FP64, FP32 = 0, 1
LHF_SINGULAR, LHF_DETERMINISTIC, LHF_OUT_GRAD, LHF_WX_EXPANSIONS = 0x1, 0x2, 0x4, 0x8
TRANS_RCR, TRANS_DIRECT = 0, 1
M2L_AUTO, M2L_HALF, M2L_TILE, M2L_TILE1, M2L_MFMA, M2L_GENERIC, M2L_QUARTER, M2L_QMFMA = range(8)
MM_AUTO, MM_HALF, MM_GENERIC, MM_QUARTER = range(4)
M2L_NAMES = ("auto", "half", "tile", "tile1", "mfma", "generic", "quarter", "qmfma")
STATUS = {0: "LHF_OK", 1: "LHF_WARN_CORE_SPLIT", 2: "LHF_WARN_TOL_UNMET", -1: "LHF_ERR_ARG",
          -2: "LHF_ERR_DOMAIN", -3: "LHF_ERR_NONFINITE", -4: "LHF_ERR_WORKSPACE", -5: "LHF_ERR_HIP",
          -6: "LHF_ERR_UNSUPPORTED", -7: "LHF_ERR_STATE"}

#: every entry point declared in include/lhfmm.h
EXPORTS = ("lhf_desc_default", "lhf_plan_create", "lhf_plan_create_multi", "lhf_execute", "lhf_execute_parts",
           "lhf_evaluate", "lhf_plan_stats", "lhf_plan_destroy", "lhf_last_error", "lhf_version",
           "lhf_profile_begin", "lhf_profile_end", "lhf_tune_default", "lhf_autotune", "lhf_choose_depth",
           "lhf_batch_create", "lhf_batch_execute", "lhf_batch_info", "lhf_batch_destroy",
           "lhf_release_cached_memory", "lhf_evaluate_noalloc", "lhf_execute_io", "lhf_execute_scalar",
           "lhf_filament_create", "lhf_filament_execute", "lhf_filament_plan", "lhf_filament_destroy",
           "lhf_plan_autotune", "lhf_plan_set_shapes", "lhf_plan_get_shapes")
PHASES = ("gather", "p2m", "m2m", "down", "l2p", "p2p", "m2l")


class Desc(C.Structure):
    _fields_ = [("p", C.c_int32), ("tol", C.c_double), ("depth", C.c_int32), ("max_per_leaf", C.c_int32),
                ("domain_lo", C.c_double * 3), ("domain_len", C.c_double), ("precision", C.c_int32),
                ("flags", C.c_uint32), ("translation", C.c_int32), ("m2l_kernel", C.c_int32),
                ("mm_kernel", C.c_int32), ("reserved", C.c_int32)]


class IO(C.Structure):
    _fields_ = [("omega", C.c_void_p), ("q", C.c_void_p), ("v", C.c_void_p), ("s", C.c_void_p),
                ("grad_v", C.c_void_p), ("beta", C.c_void_p), ("what", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("depth", C.c_int32), ("p", C.c_int32), ("boxes", C.c_int64 * 11),
                ("n_m2l", C.c_int64), ("n_m2m", C.c_int64), ("n_l2l", C.c_int64), ("n_p2p_pairs", C.c_int64),
                ("n_theta_classes", C.c_int32), ("max_level", C.c_int32), ("n_leaves", C.c_int64),
                ("n_wx_pairs", C.c_int64), ("m2l_kernel", C.c_int32), ("mm_kernel", C.c_int32),
                ("deterministic", C.c_int32), ("p_from_tol", C.c_int32), ("calib_err_v", C.c_double),
                ("calib_err_s", C.c_double), ("warnings", C.c_int32), ("wx_expansions", C.c_int32),
                ("n_m2p", C.c_int64), ("n_p2l", C.c_int64)]


class Tune(C.Structure):
    _fields_ = [("p", C.c_int32), ("precision", C.c_int32), ("t_box_ns", C.c_double), ("t_pair_ns", C.c_double)]


class Shapes(C.Structure):
    _fields_ = [("m2l_tile", C.c_int32 * 9), ("p2p_tile", C.c_int32)]


class LhfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load liblhfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1201_5430_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lhf_desc_default.argtypes = [C.POINTER(Desc)]
        L.lhf_desc_default.restype = None
        L.lhf_plan_create.argtypes = [C.POINTER(vp), C.POINTER(Desc), C.c_int64, vp, C.c_double, vp]
        L.lhf_plan_create.restype = C.c_int
        L.lhf_execute.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lhf_execute.restype = C.c_int
        L.lhf_execute_parts.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp]
        L.lhf_execute_io.argtypes = [vp, C.POINTER(IO), vp]
        L.lhf_execute_io.restype = C.c_int
        L.lhf_execute_scalar.argtypes = [vp, vp, vp, vp, vp]
        L.lhf_execute_scalar.restype = C.c_int
        L.lhf_filament_create.argtypes = [C.POINTER(vp), C.POINTER(Desc), C.c_int64, vp, C.c_int64, vp, vp]
        L.lhf_filament_create.restype = C.c_int
        L.lhf_filament_execute.argtypes = [vp, vp, vp, vp]
        L.lhf_filament_execute.restype = C.c_int
        L.lhf_filament_plan.argtypes = [vp]
        L.lhf_filament_plan.restype = vp
        L.lhf_filament_destroy.argtypes = [vp]
        L.lhf_filament_destroy.restype = C.c_int
        L.lhf_execute_parts.restype = C.c_int
        L.lhf_evaluate.argtypes = [C.POINTER(Desc), C.c_int64, vp, vp, C.c_double, vp, vp, vp]
        L.lhf_evaluate.restype = C.c_int
        L.lhf_evaluate_noalloc.argtypes = [C.POINTER(Desc), C.c_int64, vp, vp, C.c_double, vp, vp, vp]
        L.lhf_evaluate_noalloc.restype = C.c_int
        L.lhf_plan_stats.argtypes = [vp, C.POINTER(Stats)]
        L.lhf_plan_stats.restype = C.c_int
        L.lhf_plan_destroy.argtypes = [vp]
        L.lhf_plan_destroy.restype = C.c_int
        L.lhf_release_cached_memory.argtypes = []
        L.lhf_release_cached_memory.restype = C.c_int
        L.lhf_last_error.restype = C.c_char_p
        L.lhf_version.restype = C.c_char_p
        L.lhf_profile_begin.argtypes = [vp, C.c_int32]
        L.lhf_profile_begin.restype = C.c_int
        L.lhf_profile_end.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.lhf_profile_end.restype = C.c_int
        dp, i64p, i32p = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        L.lhf_plan_create_multi.argtypes = [C.POINTER(vp), C.POINTER(Desc), C.c_int32, i64p, vp, dp, dp, dp, vp]
        L.lhf_plan_create_multi.restype = C.c_int
        L.lhf_tune_default.argtypes = [C.c_int32, C.c_int32, C.POINTER(Tune)]
        L.lhf_tune_default.restype = None
        L.lhf_autotune.argtypes = [C.c_int32, C.c_int32, C.c_char_p, C.POINTER(Tune), vp]
        L.lhf_autotune.restype = C.c_int
        L.lhf_choose_depth.argtypes = [C.POINTER(Tune), C.c_int64, C.c_double, C.c_double, C.c_double, i32p]
        L.lhf_choose_depth.restype = C.c_int
        L.lhf_batch_create.argtypes = [C.POINTER(vp), C.POINTER(Desc), C.c_int32, i64p, vp, dp, dp, dp, i32p,
                                       C.POINTER(Tune), vp]
        L.lhf_batch_create.restype = C.c_int
        L.lhf_batch_execute.argtypes = [vp, vp, vp, vp, C.c_int32, vp]
        L.lhf_batch_execute.restype = C.c_int
        L.lhf_batch_info.argtypes = [vp, i32p, i32p, C.POINTER(Stats)]
        L.lhf_batch_info.restype = C.c_int
        L.lhf_batch_destroy.argtypes = [vp]
        L.lhf_batch_destroy.restype = C.c_int
        L.lhf_plan_autotune.argtypes = [vp, vp, C.c_char_p, C.POINTER(Shapes), vp]
        L.lhf_plan_autotune.restype = C.c_int
        L.lhf_plan_set_shapes.argtypes = [vp, C.POINTER(Shapes)]
        L.lhf_plan_set_shapes.restype = C.c_int
        L.lhf_plan_get_shapes.argtypes = [vp, C.POINTER(Shapes)]
        L.lhf_plan_get_shapes.restype = C.c_int
        _lib = L
    return _lib


def _check(status):
    if status < 0:
        raise LhfError(status, load().lhf_last_error().decode())
    return status


def make_desc(p=12, depth=4, precision=FP64, lo=(0.0, 0.0, 0.0), L=1.0, tol=1e-6, flags=0, max_per_leaf=0,
              m2l_kernel=M2L_AUTO, mm_kernel=MM_AUTO, translation=TRANS_RCR):
    d = Desc()
    load().lhf_desc_default(C.byref(d))
    d.p, d.depth, d.precision, d.tol, d.flags = int(p), int(depth), int(precision), float(tol), int(flags)
    d.max_per_leaf = int(max_per_leaf)
    d.m2l_kernel, d.mm_kernel, d.translation = int(m2l_kernel), int(mm_kernel), int(translation)
    for k in range(3):
        d.domain_lo[k] = float(lo[k])
    d.domain_len = float(L)
    return d


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_array(t, dtype, name, n=None, width=3):
    """check a caller tensor before its pointer crosses the C ABI: on the device, of the plan's
    dtype, contiguous, [N, width] ([N] when width is None; N == n when given)"""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a HIP device tensor")
    if width is None:
        if t.dtype != dtype or t.dim() != 1 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous [N] {dtype} tensor")
    elif t.dtype != dtype or t.dim() != 2 or t.shape[1] != width or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous [N,{width}] {dtype} tensor")
    if n is not None and t.shape[0] != n:
        raise ValueError(f"{name} has {t.shape[0]} rows, the plan has {n} elements")
    return t


def _systems(offsets, lo, L, a):
    """host arrays (int64 offsets[ns+1], float64 lo[ns][3], L[ns], a[ns]) for the multi-system calls"""
    import numpy as np
    off = np.ascontiguousarray(offsets, np.int64).reshape(-1)
    ns = off.shape[0] - 1
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, np.float64), (ns, 3)))
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.float64), (ns,)))
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (ns,)))
    return ns, off, lo, L, a


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class Plan:
    """An octree plan over fixed element positions (the paper's 'FMM set' stage).

    With ``offsets`` (host, n_systems + 1 entries), x holds several independent
    systems; ``lo``, ``L`` and ``a`` are then per system (or broadcast).  With
    ``max_per_leaf`` > 0 the octree is adaptive and ``depth`` its deepest level.
    ``p = 0`` chooses the order from ``tol``; ``grad`` keeps room for the velocity
    gradient; ``deterministic`` makes repeated executes bitwise identical;
    ``m2l_kernel`` / ``mm_kernel`` force a kernel (M2L_* / MM_* constants); ``wx_expansions``
    (adaptive tree) treats the W and X lists by M2P and P2L instead of direct sums."""

    def __init__(self, x, a, p=12, depth=4, precision=FP64, lo=(0.0, 0.0, 0.0), L=1.0, tol=1e-6, flags=0,
                 offsets=None, max_per_leaf=0, grad=False, deterministic=False, m2l_kernel=M2L_AUTO,
                 mm_kernel=MM_AUTO, translation=TRANS_RCR, wx_expansions=False):
        import torch
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        x = _dev_array(x, self.dtype, "x")
        self.n = x.shape[0]
        flags = (int(flags) | (LHF_OUT_GRAD if grad else 0) | (LHF_DETERMINISTIC if deterministic else 0)
                 | (LHF_WX_EXPANSIONS if wx_expansions else 0))
        self.desc = make_desc(p, depth, precision, lo if offsets is None else (0.0, 0.0, 0.0),
                              L if offsets is None else 1.0, tol, flags, max_per_leaf, m2l_kernel, mm_kernel,
                              translation)
        self._h = C.c_void_p()
        if offsets is None:
            self.status = _check(load().lhf_plan_create(C.byref(self._h), C.byref(self.desc), self.n,
                                                        C.c_void_p(x.data_ptr()), float(a), _stream()))
        else:
            ns, off, glo, gL, ga = _systems(offsets, lo, L, a)
            if off[-1] != self.n:
                raise ValueError("offsets[-1] must equal the number of elements")
            self.status = _check(load().lhf_plan_create_multi(
                C.byref(self._h), C.byref(self.desc), ns, _ptr(off, C.c_int64), C.c_void_p(x.data_ptr()),
                _ptr(glo, C.c_double), _ptr(gL, C.c_double), _ptr(ga, C.c_double), _stream()))
        st = self.stats()
        self.warn_core_split = bool(st["warnings"] & 1)
        self.warn_tol_unmet = bool(st["warnings"] & 2)
        self.p = st["p"]

    def execute(self, omega, v=None, s=None, what=3, grad=False, g=None, q=None, beta=False):
        """(v, s); with grad=True also grad v ([N,3,3], [i,k,l] = d v_k/d x_l); with beta=True also
        beta = grad v : grad v ([N]); q: [N] monopole strengths (divergence sources) or None"""
        import torch
        omega = _dev_array(omega, self.dtype, "omega", self.n)
        v = torch.empty_like(omega) if v is None else _dev_array(v, self.dtype, "v", self.n)
        s = torch.empty_like(omega) if s is None else _dev_array(s, self.dtype, "s", self.n)
        io = IO()
        io.omega, io.v, io.s, io.what = omega.data_ptr(), v.data_ptr(), s.data_ptr(), int(what)
        if q is not None:
            if not isinstance(q, torch.Tensor) or not q.is_cuda or q.dtype != self.dtype or \
                    not q.is_contiguous() or q.dim() != 1 or q.shape[0] != self.n:
                raise TypeError(f"q must be a contiguous [N] {self.dtype} device tensor with N = {self.n}")
            io.q = q.data_ptr()
        if grad or g is not None:
            if g is None:
                g = torch.empty((self.n, 9), dtype=self.dtype, device=omega.device)
            else:
                g = _dev_array(g.reshape(self.n, 9) if g.is_contiguous() else g, self.dtype, "g", self.n, 9)
            io.grad_v = g.data_ptr()
        b = None
        if beta:
            b = torch.empty(self.n, dtype=self.dtype, device=omega.device)
            io.beta = b.data_ptr()
        _check(load().lhf_execute_io(self._h, C.byref(io), _stream()))
        out = (v, s)
        if io.grad_v:
            out = out + (g.view(self.n, 3, 3),)
        if b is not None:
            out = out + (b,)
        return out

    def execute_scalar(self, q, phi=None, grad=None):
        """Scalar harmonic FMM (singular kernel): phi_j = sum_{i != j} q_i / r_ij and grad phi
        ([N], [N, 3]); uniform single-system plans only."""
        import torch
        q = _dev_array(q, self.dtype, "q", self.n, width=None)
        phi = torch.empty_like(q) if phi is None else _dev_array(phi, self.dtype, "phi", self.n, width=None)
        grad = (torch.empty((self.n, 3), dtype=self.dtype, device=q.device) if grad is None
                else _dev_array(grad, self.dtype, "grad", self.n))
        _check(load().lhf_execute_scalar(self._h, C.c_void_p(q.data_ptr()), C.c_void_p(phi.data_ptr()),
                                         C.c_void_p(grad.data_ptr()), _stream()))
        return phi, grad

    def stats(self):
        st = Stats()
        _check(load().lhf_plan_stats(self._h, C.byref(st)))
        return dict(n=st.n, depth=st.depth, p=st.p, boxes=list(st.boxes[:st.depth + 1]), n_m2l=st.n_m2l,
                    n_m2m=st.n_m2m, n_l2l=st.n_l2l, n_p2p_pairs=st.n_p2p_pairs,
                    n_theta_classes=st.n_theta_classes, max_level=st.max_level, n_leaves=st.n_leaves,
                    n_wx_pairs=st.n_wx_pairs, m2l_kernel=M2L_NAMES[st.m2l_kernel],
                    mm_kernel=("auto", "half", "generic", "quarter")[st.mm_kernel], deterministic=bool(st.deterministic),
                    p_from_tol=bool(st.p_from_tol), calib_err_v=st.calib_err_v, calib_err_s=st.calib_err_s,
                    warnings=st.warnings, wx_expansions=bool(st.wx_expansions), n_m2p=st.n_m2p, n_p2l=st.n_p2l)

    def autotune(self, omega, cache_path=None):
        """measure the run-time kernel shapes on this plan (one evaluation, then timed candidates);
        returns them as dict(m2l_tile=[levels 0..8], p2p_tile=...)"""
        omega = _dev_array(omega, self.dtype, "omega", self.n)
        sh = Shapes()
        cp = cache_path.encode() if cache_path else None
        _check(load().lhf_plan_autotune(self._h, C.c_void_p(omega.data_ptr()), cp, C.byref(sh), _stream()))
        return dict(m2l_tile=list(sh.m2l_tile), p2p_tile=sh.p2p_tile)

    def set_shapes(self, shapes):
        sh = Shapes()
        for i, t in enumerate(shapes.get("m2l_tile", [0] * 9)):
            sh.m2l_tile[i] = int(t)
        sh.p2p_tile = int(shapes.get("p2p_tile", 0))
        _check(load().lhf_plan_set_shapes(self._h, C.byref(sh)))

    def get_shapes(self):
        sh = Shapes()
        _check(load().lhf_plan_get_shapes(self._h, C.byref(sh)))
        return dict(m2l_tile=list(sh.m2l_tile), p2p_tile=sh.p2p_tile)

    def profile_begin(self, max_exec):
        _check(load().lhf_profile_begin(self._h, int(max_exec)))

    def profile_end(self):
        """summed per-phase milliseconds over the profiled executes, and their number"""
        ms = (C.c_double * len(PHASES))()
        k = C.c_int32()
        _check(load().lhf_profile_end(self._h, ms, C.byref(k)))
        return dict(zip(PHASES, list(ms))), k.value

    def close(self):
        if self._h:
            _check(load().lhf_plan_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def evaluate(x, omega, a, p=12, depth=4, precision=FP64, lo=(0.0, 0.0, 0.0), L=1.0, tol=1e-6):
    """One-shot evaluation: (v, s) for elements x with strengths omega."""
    import torch
    dtype = torch.float64 if precision == FP64 else torch.float32
    x = _dev_array(x, dtype, "x")
    omega = _dev_array(omega, dtype, "omega", x.shape[0])
    v = torch.empty_like(omega)
    s = torch.empty_like(omega)
    d = make_desc(p, depth, precision, lo, L, tol)
    _check(load().lhf_evaluate(C.byref(d), x.shape[0], C.c_void_p(x.data_ptr()), C.c_void_p(omega.data_ptr()),
                               float(a), C.c_void_p(v.data_ptr()), C.c_void_p(s.data_ptr()), _stream()))
    return v, s


def evaluate_noalloc(x, omega, a, p=8, depth=4, precision=FP64, lo=(0.0, 0.0, 0.0), L=1.0, tol=1e-6, v=None,
                     s=None):
    """One-shot evaluation that allocates no device memory inside the library (its plan lives in
    a fixed per-device array); pass v and s to avoid torch allocations as well."""
    import torch
    dtype = torch.float64 if precision == FP64 else torch.float32
    x = _dev_array(x, dtype, "x")
    n = x.shape[0]
    omega = _dev_array(omega, dtype, "omega", n)
    v = torch.empty_like(omega) if v is None else _dev_array(v, dtype, "v", n)
    s = torch.empty_like(omega) if s is None else _dev_array(s, dtype, "s", n)
    d = make_desc(p, depth, precision, lo, L, tol)
    _check(load().lhf_evaluate_noalloc(C.byref(d), n, C.c_void_p(x.data_ptr()), C.c_void_p(omega.data_ptr()),
                                       float(a), C.c_void_p(v.data_ptr()), C.c_void_p(s.data_ptr()), _stream()))
    return v, s


def release_cached_memory():
    """Return the idle device blocks the library keeps for later plans to the HIP runtime."""
    _check(load().lhf_release_cached_memory())


def tune_default(p, precision=FP32):
    t = Tune()
    load().lhf_tune_default(int(p), int(precision), C.byref(t))
    return t


def autotune(p, precision=FP32, cache_path=None):
    """measured unit costs of the depth cost model (device work; cached in a JSON file if given)"""
    t = Tune()
    _check(load().lhf_autotune(int(p), int(precision), cache_path.encode() if cache_path else None, C.byref(t),
                               _stream()))
    return t


def choose_depth(tune, n, L=1.0, a=0.0, tol=1e-6):
    """(depth, core_split_warning) for n uniform elements in a cube of side L"""
    d = C.c_int32()
    st = _check(load().lhf_choose_depth(C.byref(tune), int(n), float(L), float(a), float(tol), C.byref(d)))
    return d.value, st == 1


class Batch:
    """Independent systems with per-system depth, evaluated by one HIP graph."""

    def __init__(self, x, offsets, a, p=10, precision=FP32, lo=(0.0, 0.0, 0.0), L=1.0, tol=1e-6, flags=0,
                 depths=None, tune=None):
        import numpy as np
        import torch
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        x = _dev_array(x, self.dtype, "x")
        self.n = x.shape[0]
        self.ns, off, glo, gL, ga = _systems(offsets, lo, L, a)
        if off[-1] != self.n:
            raise ValueError("offsets[-1] must equal the number of elements")
        self.desc = make_desc(p, 4, precision, (0.0, 0.0, 0.0), 1.0, tol, flags)
        dep = None
        if depths is not None:
            dep = np.ascontiguousarray(np.broadcast_to(np.asarray(depths, np.int32), (self.ns,)))
        self._h = C.c_void_p()
        self.status = _check(load().lhf_batch_create(
            C.byref(self._h), C.byref(self.desc), self.ns, _ptr(off, C.c_int64), C.c_void_p(x.data_ptr()),
            _ptr(glo, C.c_double), _ptr(gL, C.c_double), _ptr(ga, C.c_double),
            _ptr(dep, C.c_int32) if dep is not None else None, C.byref(tune) if tune is not None else None,
            _stream()))
        self.warn_core_split = self.status == 1

    def execute(self, omega, v=None, s=None, graph=True):
        import torch
        omega = _dev_array(omega, self.dtype, "omega", self.n)
        v = torch.empty_like(omega) if v is None else _dev_array(v, self.dtype, "v", self.n)
        s = torch.empty_like(omega) if s is None else _dev_array(s, self.dtype, "s", self.n)
        _check(load().lhf_batch_execute(self._h, C.c_void_p(omega.data_ptr()), C.c_void_p(v.data_ptr()),
                                        C.c_void_p(s.data_ptr()), int(bool(graph)), _stream()))
        return v, s

    def info(self):
        import numpy as np
        ng = C.c_int32()
        dep = np.zeros(self.ns, np.int32)
        st = Stats()
        _check(load().lhf_batch_info(self._h, C.byref(ng), _ptr(dep, C.c_int32), C.byref(st)))
        return dict(n_groups=ng.value, depths=dep, n_m2l=st.n_m2l, n_p2p_pairs=st.n_p2p_pairs,
                    boxes=list(st.boxes[:st.depth + 1]))

    def close(self):
        if self._h:
            _check(load().lhf_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Filament:
    """Vortex filaments: straight segments seg [S, 2] (vertex indices) between the vertices X
    [V, 3], velocity at the vertices (uniform octree over segment centres and vertices).
    ``execute(G)`` takes the circulations [S] and returns v [V, 3]."""

    def __init__(self, X, seg, p=12, depth=4, precision=FP64, lo=(0.0, 0.0, 0.0), L=1.0, tol=1e-6,
                 m2l_kernel=M2L_AUTO):
        import torch
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        X = _dev_array(X, self.dtype, "X")
        if not isinstance(seg, torch.Tensor) or not seg.is_cuda or seg.dtype != torch.int32 or \
                seg.dim() != 2 or seg.shape[1] != 2 or not seg.is_contiguous():
            raise TypeError("seg must be a contiguous [S,2] int32 device tensor")
        self.nv, self.ns = X.shape[0], seg.shape[0]
        self.desc = make_desc(p, depth, precision, lo, L, tol, 0, 0, m2l_kernel)
        self._h = C.c_void_p()
        self.status = _check(load().lhf_filament_create(C.byref(self._h), C.byref(self.desc), self.nv,
                                                        C.c_void_p(X.data_ptr()), self.ns,
                                                        C.c_void_p(seg.data_ptr()), _stream()))

    def execute(self, G, v=None):
        import torch
        G = _dev_array(G, self.dtype, "G", self.ns, width=None)
        v = torch.empty((self.nv, 3), dtype=self.dtype, device=G.device) if v is None else \
            _dev_array(v, self.dtype, "v", self.nv)
        _check(load().lhf_filament_execute(self._h, C.c_void_p(G.data_ptr()), C.c_void_p(v.data_ptr()), _stream()))
        return v

    def stats(self):
        st = Stats()
        _check(load().lhf_plan_stats(load().lhf_filament_plan(self._h), C.byref(st)))
        return dict(n=st.n, p=st.p, n_m2l=st.n_m2l, boxes=list(st.boxes[:st.depth + 1]))

    def close(self):
        if self._h:
            load().lhf_filament_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
