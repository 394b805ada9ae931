"""Oracle of the exact Euclidean distance transform of a site grid
(cuRoboV2 Sec. 5, "Stage 2: Distance Propagation": the dense ESDF's
nearest-site assignment, which PBA+ computes exactly).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
CPU-baseline leg, never by the HIP library or its binding; it shares no code
with the HIP path.

The result has a plain definition, so the oracle is that definition written
out: for every voxel v of an nz x ny x nx grid and the set S of site voxels,
    d2(v) = min over s in S of |v - s|^2     (integer voxel coordinates),
    dist(v) = voxel_size * sqrt(d2(v)),
with d2 = +inf (no nearest site) when S is empty.  The nearest site itself
need not be unique (ties); tests compare d2, which is, and check that a
reported site is a site at that squared distance.

Arrays are [nz][ny][nx] (x fastest), the layout of the HIP path.  Work is
brute force over sites, chunked with numpy: exact integer arithmetic in
int64.
"""
from __future__ import annotations

import numpy as np

NONE = np.iinfo(np.int64).max


def sites_of(mask: np.ndarray) -> np.ndarray:
    """Coordinates (z, y, x) of every site voxel: [S, 3] int64."""
    return np.argwhere(np.asarray(mask) != 0).astype(np.int64)


def d2_at(mask: np.ndarray, points: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """Squared distance to the nearest site for points [P, 3] (z, y, x):
    [P] int64, NONE where there is no site."""
    S = sites_of(mask)
    pts = np.asarray(points, dtype=np.int64).reshape(-1, 3)
    out = np.full(pts.shape[0], NONE, dtype=np.int64)
    if S.shape[0] == 0:
        return out
    for i in range(0, pts.shape[0], chunk):
        p = pts[i:i + chunk]
        best = np.full(p.shape[0], NONE, dtype=np.int64)
        for j in range(0, S.shape[0], 4096):
            d = p[:, None, :] - S[None, j:j + 4096, :]
            best = np.minimum(best, np.einsum("psk,psk->ps", d, d).min(1))
        out[i:i + chunk] = best
    return out


def d2_grid(mask: np.ndarray) -> np.ndarray:
    """Squared distance transform of a whole (small) grid: [nz, ny, nx] int64."""
    mask = np.asarray(mask)
    pts = np.argwhere(np.ones(mask.shape, dtype=bool))
    return d2_at(mask, pts).reshape(mask.shape)


def dist(d2: np.ndarray, voxel_size: float = 1.0) -> np.ndarray:
    """Euclidean distance from squared distances (+inf where there is no site)."""
    d2 = np.asarray(d2)
    out = np.full(d2.shape, np.inf)
    ok = d2 != NONE
    out[ok] = voxel_size * np.sqrt(d2[ok].astype(np.float64))
    return out
