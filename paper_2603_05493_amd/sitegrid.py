"""Seeded synthetic site grids for the distance transform.

This module only draws inputs: uint8 grids [nz][ny][nx] (x fastest) whose
nonzero voxels are surface sites.  It holds none of the distance-transform
arithmetic, so it can feed both the HIP path and the oracle.

`room` stands in for the surface band that site seeding extracts from a
fused TSDF of an indoor scene (the paper evaluates on a recorded bedroom
scan, which is not available here): a floor, two walls, a table, boxes and
spheres, voxelized as shells about 1.5 voxels thick (the band the
seven-point gather stencil produces), plus sparse isolated sites standing in
for depth noise.  At the paper's 20 mm ESDF voxel the default 256 x 256 x 128
grid covers a 5.12 m x 5.12 m x 2.56 m room.
"""
from __future__ import annotations

import numpy as np

BAND = 0.75   # half-thickness of a voxelized surface, in voxels


def random_sites(nz: int, ny: int, nx: int, p: float, seed: int = 0) -> np.ndarray:
    """Independent Bernoulli(p) sites."""
    rng = np.random.default_rng(seed)
    return (rng.random((nz, ny, nx)) < p).astype(np.uint8)


def _coords(shape):
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    return z, y, x


def _shell_box(z, y, x, lo, hi):
    """Voxels within BAND of the surface of the axis-aligned box [lo, hi] (z, y, x)."""
    inside_grown = np.ones(z.shape, bool)
    inside_shrunk = np.ones(z.shape, bool)
    for c, a, b in zip((z, y, x), lo, hi):
        inside_grown &= (c >= a - BAND) & (c <= b + BAND)
        inside_shrunk &= (c > a + BAND) & (c < b - BAND)
    return inside_grown & ~inside_shrunk


def room(nx: int = 256, ny: int = 256, nz: int = 128, seed: int = 0, n_boxes: int = 6, n_spheres: int = 6,
         noise: float = 1e-4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    z, y, x = _coords((nz, ny, nx))
    m = np.zeros((nz, ny, nx), bool)
    m |= np.abs(z - 2.0) <= BAND                       # floor
    m |= np.abs(x - 1.0) <= BAND                       # two walls
    m |= np.abs(y - 1.0) <= BAND
    # a table: top slab and four legs
    tz = 0.3 * nz
    t0, t1 = (0.35 * ny, 0.35 * nx), (0.6 * ny, 0.7 * nx)
    m |= _shell_box(z, y, x, (tz - 1.5, t0[0], t0[1]), (tz + 1.5, t1[0], t1[1]))
    for ly in (t0[0] + 2, t1[0] - 2):
        for lx in (t0[1] + 2, t1[1] - 2):
            m |= _shell_box(z, y, x, (2.0, ly - 1.5, lx - 1.5), (tz, ly + 1.5, lx + 1.5))
    for _ in range(n_boxes):                            # boxes on the floor and the table
        size = rng.uniform(0.04, 0.15, 3) * np.array([nz, ny, nx])
        base = tz + 1.5 if rng.random() < 0.5 else 2.0
        cy, cx = rng.uniform(0.15, 0.85) * ny, rng.uniform(0.15, 0.85) * nx
        m |= _shell_box(z, y, x, (base, cy - size[1] / 2, cx - size[2] / 2),
                        (base + size[0], cy + size[1] / 2, cx + size[2] / 2))
    for _ in range(n_spheres):                          # round objects
        r = rng.uniform(0.02, 0.08) * nx
        c = np.array([rng.uniform(r + 3, nz - r - 1), rng.uniform(r, ny - r), rng.uniform(r, nx - r)])
        d = np.sqrt((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2)
        m |= np.abs(d - r) <= BAND
    m |= rng.random(m.shape) < noise
    return m.astype(np.uint8)
