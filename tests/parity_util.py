"""Comparison helpers shared by the GPU parity tests (no method arithmetic)."""
import numpy as np


def rel(a, b):
    """relative L2 difference ||a - b|| / ||b||"""
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def check(v, s, vr, sr, l2=1e-12, mx=1e-11, label=""):
    """relative L2 of v and of s <= l2, and every element within mx of the largest
    reference magnitude (the FP64 bar by default)"""
    ev, es = rel(v, vr), rel(s, sr)
    mv = np.abs(v - vr).max() / max(np.abs(vr).max(), 1e-300)
    ms = np.abs(s - sr).max() / max(np.abs(sr).max(), 1e-300)
    print(f"{label} rel L2 v {ev:.3e} s {es:.3e}  max v {mv:.3e} s {ms:.3e}", flush=True)
    assert ev <= l2 and es <= l2, (ev, es)
    assert mv <= mx and ms <= mx, (mv, ms)
    return ev, es, mv, ms


def check32(v, s, vr, sr, l2=2e-6, mx=1e-5, label=""):
    """FP32 path against the FP64 oracle on the FP32-rounded inputs (or against another FP32
    kernel): relative L2 <= 2e-6 and element-wise <= 1e-5 of the largest magnitude"""
    return check(v, s, vr, sr, l2=l2, mx=mx, label=label)
