"""Independent references used to pin the oracle: library routines (SciPy's
RegularGridInterpolator and root finder, NumPy, PyTorch float64 autograd),
closed forms and brute force.  Nothing here calls the oracle or the HIP path.
"""
from __future__ import annotations

import numpy as np
import scipy.interpolate as si


def grid_interp(W, aabb):
    """Trilinear (align-corners, clamped) interpolator of a [Dz,Dy,Dx,C] grid
    over the box aabb = (lo xyz, hi xyz), via SciPy."""
    Dz, Dy, Dx = W.shape[:3]
    lo, hi = np.asarray(aabb[:3], float), np.asarray(aabb[3:], float)
    axes = (np.linspace(lo[2], hi[2], Dz), np.linspace(lo[1], hi[1], Dy), np.linspace(lo[0], hi[0], Dx))
    f = si.RegularGridInterpolator(axes, np.asarray(W, np.float64), method="linear")

    def ev(x):
        x = np.clip(np.asarray(x, np.float64).reshape(-1, 3), lo, hi)
        return f(x[:, ::-1])
    return ev


def lbs_scipy(B, W, aabb):
    """x -> sum_b w_b(x) B_b [x; 1] with w from SciPy's interpolator."""
    wf = grid_interp(W, aabb)
    B = np.asarray(B, np.float64)

    def f(x):
        x = np.asarray(x, np.float64).reshape(-1, 3)
        w = wf(x)
        xh = np.concatenate([x, np.ones((x.shape[0], 1))], 1)
        y = np.einsum("bij,nj->nbi", B, xh)
        return np.einsum("nb,nbi->ni", w, y)
    return f


def hash_index_bigint(v, N, T):
    """Instant-NGP vertex index with Python integers (no fixed-width overflow)."""
    side = N + 1
    if side ** 3 <= T:
        return v[0] + side * (v[1] + side * v[2])
    h = (v[0] * 1) ^ (v[1] * 2654435761) ^ (v[2] * 805459861)
    return (h % 2 ** 32) % T
