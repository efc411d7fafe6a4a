"""Seeded synthetic inputs for the vortex FMM workloads.

This module holds only random-number draws and geometry of the input
distributions -- none of the method's arithmetic -- so that the oracle side
(tests, CPU baseline) and the GPU side (library tests, bench) receive the same
inputs from one place and share nothing else.

The paper tests on synthetic distributions only (elements uniform in a cube or
on a sphere surface, vortex rings); these generators reproduce those shapes:

  uniform_cube   x ~ U[0,1)^3, omega ~ N(0,1)^3                     (Sec. 5.1)
  vortex_ring    90% of the elements on a torus of major radius 0.3 about the
                 centre of the unit cube (axis z) with a Gaussian cross-section
                 (density ~ exp(-rho^2/0.05^2)), 10% uniform background;
                 omega = exp(-rho^2/0.05^2) e_theta (tangent to the ring)
  batched        many independent uniform-cube systems of log-uniform size
All positions are drawn before the strengths; arrays are float64 [N, 3].
"""
from __future__ import annotations

import math

import numpy as np

#: the workloads the library is measured on (name -> description)
CONFIGS = {
    "cube4k_fp64": dict(n=4096, seed=1, depth=3, p=8, precision="fp64",
                        desc="N=4096 uniform cube, depth 3, p=8, FP64"),
    "cube1m_fp64": dict(n=1 << 20, seed=2, depth=6, p=12, precision="fp64",
                        desc="N=1,048,576 uniform cube, depth 6, p=12, FP64"),
    "cube1m_fp32": dict(n=1 << 20, seed=2, depth=6, p=10, precision="fp32",
                        desc="N=1,048,576 uniform cube, depth 6, p=10, FP32 elements and expansions"),
    "ring4m_fp32": dict(n=1 << 22, seed=4, depth=0, max_per_leaf=64, p=16, precision="fp32",
                        desc="N=4,194,304 vortex ring + 10% background, adaptive <=64/leaf, p=16"),
    "batch256_fp32": dict(n_systems=256, seed=5, p=10, precision="fp32",
                          desc="256 systems, N log-uniform in [1024, 65536], p=10"),
}


def core_radius(n: int) -> float:
    """Gaussian core a = 0.5 * N^(-1/3) (half the mean element spacing)."""
    return 0.5 * float(n) ** (-1.0 / 3.0)


def uniform_cube(n: int, seed: int):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 3))
    w = rng.normal(0.0, 1.0, size=(n, 3))
    return x, w


def vortex_ring(n: int, seed: int, major=0.3, sigma=0.05, background=0.1):
    rng = np.random.default_rng(seed)
    nb = int(round(background * n))
    nr = n - nb
    theta = rng.uniform(0.0, 2.0 * math.pi, size=nr)
    # 2-D Gaussian offsets in the cross-section, per-axis std sigma/sqrt(2)
    off = rng.normal(0.0, sigma / math.sqrt(2.0), size=(nr, 2))
    rad = major + off[:, 0]
    xr = np.stack([0.5 + rad * np.cos(theta), 0.5 + rad * np.sin(theta), 0.5 + off[:, 1]], axis=1)
    xb = rng.uniform(0.0, 1.0, size=(nb, 3))
    x = np.concatenate([xr, xb], axis=0)
    perm = rng.permutation(n)
    x = np.clip(x[perm], 0.0, np.nextafter(1.0, 0.0))
    # strengths: tangent to the ring, magnitude exp(-rho^2/sigma^2)
    dx, dy = x[:, 0] - 0.5, x[:, 1] - 0.5
    rxy = np.hypot(dx, dy)
    rxy = np.where(rxy == 0.0, 1e-300, rxy)
    rho2 = (rxy - major) ** 2 + (x[:, 2] - 0.5) ** 2
    mag = np.exp(-rho2 / sigma ** 2)
    w = np.stack([-dy / rxy * mag, dx / rxy * mag, np.zeros(n)], axis=1)
    return x, w


def batched_sizes(n_systems: int, seed: int, lo=1024, hi=65536):
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_systems))).astype(np.int64)
    return sizes, rng


def batched(n_systems: int, seed: int):
    """Return (sizes, list of (x, w)) for independent uniform-cube systems."""
    sizes, rng = batched_sizes(n_systems, seed)
    kids = rng.spawn(n_systems)
    out = []
    for k, nk in enumerate(sizes):
        x = kids[k].uniform(0.0, 1.0, size=(int(nk), 3))
        w = kids[k].normal(0.0, 1.0, size=(int(nk), 3))
        out.append((x, w))
    return sizes, out


def make(name: str):
    """Inputs for a named workload: dict with x, w (float64) and metadata."""
    cfg = dict(CONFIGS[name])
    if name.startswith("cube"):
        x, w = uniform_cube(cfg["n"], cfg["seed"])
    elif name.startswith("ring"):
        x, w = vortex_ring(cfg["n"], cfg["seed"])
    else:
        raise ValueError("use batched() for the batched workload")
    cfg.update(x=x, w=w, a=core_radius(x.shape[0]))
    return cfg


def filament_rings(n_rings: int, n_per_ring: int, seed: int, rmin=0.03, rmax=0.12):
    """Closed polygonal vortex filaments (Sec. 5.3): n_rings circles of n_per_ring straight
    segments each, radius ~ U[rmin, rmax], random orientation, centres uniform in the part of the
    unit cube that keeps every ring inside it, circulation ~ N(0, 1) per ring.  Returns
    (X [V, 3] vertices, seg [S, 2] int32 vertex indices, G [S] circulations), V = S."""
    rng = np.random.default_rng(seed)
    X, seg, G = [], [], []
    for k in range(n_rings):
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r, 1.0 - r, size=3)
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        u = np.cross(ax, [1.0, 0.0, 0.0] if abs(ax[0]) < 0.9 else [0.0, 1.0, 0.0])
        u /= np.linalg.norm(u)
        v = np.cross(ax, u)
        th = 2.0 * math.pi * (np.arange(n_per_ring) + rng.uniform()) / n_per_ring
        pts = c[None, :] + r * (np.cos(th)[:, None] * u[None, :] + np.sin(th)[:, None] * v[None, :])
        base = k * n_per_ring
        X.append(np.clip(pts, 0.0, np.nextafter(1.0, 0.0)))
        i = np.arange(n_per_ring)
        seg.append(np.stack([base + i, base + (i + 1) % n_per_ring], axis=1))
        G.append(np.full(n_per_ring, rng.normal()))
    return np.concatenate(X), np.concatenate(seg).astype(np.int32), np.concatenate(G)


def sample_targets(n: int, k: int, seed: int = 12345):
    """Seeded sample of k distinct element indices (the paper measures errors
    on 1000 random source points)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
