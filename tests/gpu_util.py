"""Helpers for the GPU parity tests (tolerance checks, device uploads)."""
from __future__ import annotations

import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def up(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device=dev(), dtype=dtype)


def soa(a, ld=None, dtype=torch.float32):
    """[n,3] host array -> [3][ld] device tensor (zero padded)."""
    a = np.asarray(a)
    n = a.shape[0]
    ld = n if ld is None else ld
    out = np.zeros((3, ld), np.float64)
    out[:, :n] = a.T
    return up(out, dtype)


def feat_dev(rows, ld=None, dtype=torch.float32):
    """[S][32] per-sample feature rows -> level-major [16][ld][2] device
    tensor (flat, zero padded past S)."""
    rows = np.asarray(rows)
    S = rows.shape[0]
    ld = S if ld is None else ld
    out = np.zeros((16, ld, 2), np.float64)
    out[:, :S, :] = rows.reshape(S, 16, 2).transpose(1, 0, 2)
    return up(out.reshape(-1), dtype)


def feat_host(t, S, ld=None):
    """Level-major [16][ld][2] device features -> [S][32] host rows."""
    ld = S if ld is None else ld
    return host(t).reshape(16, ld, 2)[:, :S, :].transpose(1, 0, 2).reshape(S, 32)


def host(t):
    return t.detach().double().cpu().numpy()


def assert_mixed(got, ref, tol, what="", scale=1.0):
    """|got - ref| <= tol * max(scale, |ref|) elementwise (mixed relative)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    err = np.abs(got - ref) / np.maximum(scale, np.abs(ref))
    if err.size and not (err <= tol).all():
        i = np.unravel_index(np.argmax(err), err.shape)
        raise AssertionError(f"{what}: max mixed error {err.max():.3e} > {tol:.1e} at {i}: got {got[i]!r} "
                             f"ref {ref[i]!r} ({(err > tol).sum()} of {err.size} elements)")
    return float(err.max()) if err.size else 0.0


def unpack_bricks(bits, G):
    """Host decode of the packed occupancy layout (8 x 8 x 16 bricks, bit
    lx + 8 ly + 64 lz of a 32-word brick) into a [z][y][x] bool grid."""
    words = bits.astype(np.uint32)
    nb, nbz = (G + 7) // 8, (G + 15) // 16
    out = np.zeros((nbz * 16, nb * 8, nb * 8), dtype=bool)
    for bz in range(nbz):
        for by in range(nb):
            for bx in range(nb):
                brick = words[32 * (bx + nb * (by + nb * bz)):][:32]
                cells = ((brick[:, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(-1)  # 1024 bits
                out[16 * bz:16 * bz + 16, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8] = cells.reshape(16, 8, 8)
    return out
