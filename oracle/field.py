"""MERF feature field: trilinear grid + three bilinear planes (TEST INFRASTRUCTURE).

Follows Oblique-MERF Sec. 3, Eq. 2: t(p) = V(p) + P_x(p) + P_y(p) + P_z(p),
with V a low-resolution 3D grid (trilinear) and the P's high-resolution 2D
planes (bilinear), 8 channels each; and Eq. 3 for the activations.

Readings (the paper gives no alignment or axis naming):

* Vertex-aligned samples: an axis with N points spans the box faces
  inclusively, u = (p - lo) / (hi - lo) * (N - 1), i0 = min(floor(u), N - 2),
  f = u - i0.  (The same convention as grid_sample with align_corners=True.)
* Planes: P_z is the XY plane indexed (x, y), P_y the XZ plane indexed
  (x, z), P_x the YZ plane indexed (y, z).  Memory order is
  [second][first][channel]; the grid is [z][y][x][channel].
* Channel order: 0 = density pre-activation, 1..3 = diffuse colour,
  4..7 = specular features (Eq. 3 split [tau, c^d, f]).

All arithmetic is float64 on the exact float64 promotion of the binary32
sample points.
"""
from __future__ import annotations

import numpy as np
import torch


def corner_weights_1d(c: np.ndarray, lo: float, hi: float, n: int):
    """Left vertex index and fractional weight along one axis (vertex-aligned)."""
    u = (np.asarray(c, dtype=np.float64) - lo) / (hi - lo) * (n - 1)
    i0 = np.clip(np.floor(u), 0, n - 2).astype(np.int64)
    f = u - i0
    return i0, f


def trilinear_corners(p: np.ndarray, box_lo, box_hi, dims):
    """Flat vertex indices [S, 8] and weights [S, 8] for grid[z][y][x].

    Corner c = (dx, dy, dz) with c = dx + 2 dy + 4 dz; weight is the product
    of (1 - f) or f per axis (trilinear interpolation)."""
    lx, ly, lz = dims
    ix, fx = corner_weights_1d(p[:, 0], box_lo[0], box_hi[0], lx)
    iy, fy = corner_weights_1d(p[:, 1], box_lo[1], box_hi[1], ly)
    iz, fz = corner_weights_1d(p[:, 2], box_lo[2], box_hi[2], lz)
    idx = np.empty((p.shape[0], 8), dtype=np.int64)
    w = np.empty((p.shape[0], 8), dtype=np.float64)
    for c in range(8):
        dx, dy, dz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        idx[:, c] = ((iz + dz) * ly + (iy + dy)) * lx + (ix + dx)
        w[:, c] = ((fx if dx else 1 - fx) * (fy if dy else 1 - fy) * (fz if dz else 1 - fz))
    return idx, w


def bilinear_corners(a: np.ndarray, b: np.ndarray, lo_a, hi_a, lo_b, hi_b, na: int, nb: int):
    """Flat texel indices [S, 4] and weights [S, 4] for plane[b][a]."""
    ia, fa = corner_weights_1d(a, lo_a, hi_a, na)
    ib, fb = corner_weights_1d(b, lo_b, hi_b, nb)
    idx = np.empty((a.shape[0], 4), dtype=np.int64)
    w = np.empty((a.shape[0], 4), dtype=np.float64)
    for c in range(4):
        da, db = c & 1, (c >> 1) & 1
        idx[:, c] = (ib + db) * na + (ia + da)
        w[:, c] = (fa if da else 1 - fa) * (fb if db else 1 - fb)
    return idx, w


SOURCES = ("grid", "plane_xy", "plane_xz", "plane_yz")


def feature_terms(p: np.ndarray, box_lo, box_hi, grid_dims, plane_dims):
    """Interpolation terms of Eq. 2 for float64 points p [S, 3]:
    {source: (flat index [S, c], weight [S, c])}."""
    nx, ny, nz = plane_dims
    return {
        "grid": trilinear_corners(p, box_lo, box_hi, grid_dims),
        "plane_xy": bilinear_corners(p[:, 0], p[:, 1], box_lo[0], box_hi[0], box_lo[1], box_hi[1], nx, ny),
        "plane_xz": bilinear_corners(p[:, 0], p[:, 2], box_lo[0], box_hi[0], box_lo[2], box_hi[2], nx, nz),
        "plane_yz": bilinear_corners(p[:, 1], p[:, 2], box_lo[1], box_hi[1], box_lo[2], box_hi[2], ny, nz),
    }


def interp_features(terms, lookup) -> torch.Tensor:
    """t = sum over sources and corners of weight * value (Eq. 2).

    ``lookup(source, corner, idx)`` returns float64 rows [len(idx), 8] of
    that source's vertices/texels for one corner column."""
    out = None
    for src in SOURCES:
        idx, w = terms[src]
        wt = torch.from_numpy(w)
        for c in range(idx.shape[1]):
            term = wt[:, c:c + 1] * lookup(src, c, idx[:, c])
            out = term if out is None else out + term
    return out


def activations(t: torch.Tensor):
    """Eq. 3: tau = exp(t0), c^d = sigmoid(t1..3), f = sigmoid(t4..7)."""
    tau = torch.exp(t[..., 0])
    cd = torch.sigmoid(t[..., 1:4])
    f = torch.sigmoid(t[..., 4:8])
    return tau, cd, f
