"""Sample placement inside the occupancy plane (TEST INFRASTRUCTURE).

Follows Oblique-MERF Sec. 4.1 (occupancy plane P_o of (z_min, z_max) per grid
point; Eq. 6 with epsilon = 0, i.e. the indicator of [z_min, z_max]; Eq. 7,
the point takes the occupancy of the grid point nearest to its xy
projection) and Sec. 4.4 (the real-time marcher samples only inside
[z_min, z_max] of the column it is in).  Rays are r(t) = o + t d (Sec. 3).

Readings where the paper is silent:

* Lattice: samples sit at t_k = k * delta, k = 0, 1, ..., measured from the
  ray origin, with delta = box height / 512 = 2^-11 (exact in binary).
  k ranges over [0, K_CAP) with K_CAP = 2^24, so t_k is exact in binary32.
* The point is evaluated in binary32 with two roundings and no fused
  multiply-add:  p = fl32(o + fl32(t_k * d)) per component.  A sample is a
  discrete decision; defining it in binary32 makes both the oracle and the
  GPU take it in the same precision.
* The nearest occupancy grid point of Eq. 7: grid points sit at cell
  centres, so the nearest one is the cell containing p.  Cells are half-open
  [lo, hi) with the far face of the box put in the last cell:
  i = clamp(floor((p_x - x_lo) * M / (x_hi - x_lo)), 0, M - 1), same for j.
  The scale M/(x_hi - x_lo) is required to be a power of two and
  x_lo * M/(x_hi - x_lo) an integer, so the floor is evaluated exactly as
  floor(p_x * scale) - x_lo * scale.
* Accept iff p lies in the closed box and z_min[j][i] <= p_z <= z_max[j][i]
  (both closed; a cell with z_min > z_max is empty).
* Keep the first n_max accepted samples in increasing k.

Completeness of the enumeration: each rounded coordinate p_a(k) is a
monotone function of k (t_k * d_a is monotone in k and rounding to nearest
is monotone), so the set of k whose point lies in [lo_a, hi_a] is one
interval of k per axis.  ``box_k_interval`` finds that interval exactly by
bisection on the binary32 predicate itself, and every k inside the
intersection is tested.
"""
from __future__ import annotations

import numpy as np

K_CAP = 1 << 24


def lattice_t(k, delta: float) -> np.ndarray:
    """t_k = k * delta as binary32 (exact for 0 <= k < 2^24, delta = 2^-11)."""
    t64 = np.asarray(k, dtype=np.float64) * float(delta)
    t32 = t64.astype(np.float32)
    return t32


def lattice_points(o: np.ndarray, d: np.ndarray, k, delta: float) -> np.ndarray:
    """p = fl32(o + fl32(t_k * d)): binary32 multiply, then binary32 add.

    ``o`` and ``d`` are float32 [..., 3]; ``k`` broadcasts against o[..., 0].
    numpy rounds each float32 operation separately (no contraction).
    """
    t = lattice_t(k, delta)[..., None]
    step = (t * d).astype(np.float32)
    return (o + step).astype(np.float32)


def _coord(o_a, d_a, k, delta):
    t = lattice_t(k, delta)
    return (o_a + (t * d_a).astype(np.float32)).astype(np.float32)


def _first_true(pred, n: int) -> np.ndarray:
    """Smallest k in [0, K_CAP] (per ray) with pred(k) true, for a predicate
    that is monotone false -> true in k; K_CAP if it never turns true."""
    lo = np.zeros(n, dtype=np.int64)
    hi = np.full(n, K_CAP, dtype=np.int64)
    while True:
        act = lo < hi
        if not act.any():
            return lo
        mid = (lo + hi) // 2
        c = pred(mid)
        hi = np.where(act & c, mid, hi)
        lo = np.where(act & ~c, mid + 1, lo)


def box_k_interval(o: np.ndarray, d: np.ndarray, box_lo, box_hi, delta: float):
    """Exact [k_first, k_last] of lattice indices whose binary32 point lies in
    the closed box, per ray (k_first > k_last when empty)."""
    o = np.asarray(o, dtype=np.float32)
    d = np.asarray(d, dtype=np.float32)
    n = o.shape[0]
    first = np.zeros(n, dtype=np.int64)
    last = np.full(n, K_CAP - 1, dtype=np.int64)
    for a in range(3):
        lo = np.float32(box_lo[a])
        hi = np.float32(box_hi[a])
        oa = o[:, a]
        da = d[:, a]
        pos = da > 0
        neg = da < 0
        zero = da == 0
        # d_a > 0: coordinate non-decreasing in k.
        enter_p = _first_true(lambda k: _coord(oa, da, k, delta) >= lo, n)
        leave_p = _first_true(lambda k: _coord(oa, da, k, delta) > hi, n) - 1
        # d_a < 0: coordinate non-increasing in k.
        enter_n = _first_true(lambda k: _coord(oa, da, k, delta) <= hi, n)
        leave_n = _first_true(lambda k: _coord(oa, da, k, delta) < lo, n) - 1
        inside0 = (oa >= lo) & (oa <= hi)
        ea = np.where(pos, enter_p, np.where(neg, enter_n, np.where(zero & inside0, 0, K_CAP)))
        la = np.where(pos, leave_p, np.where(neg, leave_n, np.where(zero & inside0, K_CAP - 1, -1)))
        first = np.maximum(first, ea)
        last = np.minimum(last, la)
    return first, last


def cell_index(p_a: np.ndarray, lo: float, hi: float, m: int) -> np.ndarray:
    """Containing cell of coordinate p_a among m half-open cells of [lo, hi]
    (far face clamped into cell m-1); exact floor (see module docstring)."""
    scale = m / (hi - lo)
    if scale <= 0 or 2.0 ** round(np.log2(scale)) != scale:
        raise ValueError("occupancy cells per unit length must be a power of two")
    off = lo * scale
    if off != round(off):
        raise ValueError("box low corner must fall on a cell boundary multiple")
    v = np.floor(np.asarray(p_a, dtype=np.float64) * scale) - off
    v = np.where(np.isfinite(v), v, 0.0)
    return np.clip(v, 0, m - 1).astype(np.int64)


def accept_mask(p: np.ndarray, occ: np.ndarray, box_lo, box_hi) -> np.ndarray:
    """Eq. 6 (epsilon = 0) with Eq. 7: p in the closed box and inside the
    closed interval [z_min, z_max] of the cell containing p's xy."""
    my, mx = occ.shape[0], occ.shape[1]
    px, py, pz = p[..., 0], p[..., 1], p[..., 2]
    inb = ((px >= np.float32(box_lo[0])) & (px <= np.float32(box_hi[0]))
           & (py >= np.float32(box_lo[1])) & (py <= np.float32(box_hi[1]))
           & (pz >= np.float32(box_lo[2])) & (pz <= np.float32(box_hi[2])))
    i = cell_index(px, box_lo[0], box_hi[0], mx)
    j = cell_index(py, box_lo[1], box_hi[1], my)
    zmin = occ[j, i, 0]
    zmax = occ[j, i, 1]
    return inb & (pz >= zmin) & (pz <= zmax)


def place_samples(o: np.ndarray, d: np.ndarray, occ: np.ndarray, box_lo, box_hi,
                  delta: float, n_max: int, chunk_elems: int = 1 << 23):
    """First n_max accepted lattice samples per ray, in increasing k.

    Returns ``k_list`` int32 [n, n_max] (padded with -1), ``n_placed`` int32
    [n] and the binary32 points ``p`` float32 [n, n_max, 3] (padding 0).
    """
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    occ = np.ascontiguousarray(occ, dtype=np.float32)
    n = o.shape[0]
    k_list = np.full((n, n_max), -1, dtype=np.int32)
    n_placed = np.zeros(n, dtype=np.int32)
    pts = np.zeros((n, n_max, 3), dtype=np.float32)
    first, last = box_k_interval(o, d, box_lo, box_hi, delta)
    length = np.maximum(last - first + 1, 0)
    r = 0
    while r < n:
        # grow the chunk while the padded candidate block stays bounded
        r1 = r + 1
        width = int(length[r])
        while r1 < n and max(width, int(length[r1])) * (r1 + 1 - r) <= chunk_elems:
            width = max(width, int(length[r1]))
            r1 += 1
        width = max(width, 1)
        idx = np.arange(width, dtype=np.int64)[None, :]
        ks = first[r:r1, None] + idx
        valid = idx < length[r:r1, None]
        ks_safe = np.where(valid, ks, 0)
        p = lattice_points(o[r:r1, None, :], d[r:r1, None, :], ks_safe, delta)
        acc = accept_mask(p, occ, box_lo, box_hi) & valid
        rank = np.cumsum(acc, axis=1)
        keep = acc & (rank <= n_max)
        rows, cols = np.nonzero(keep)
        slot = rank[rows, cols] - 1
        k_list[r + rows, slot] = ks[rows, cols].astype(np.int32)
        pts[r + rows, slot] = p[rows, cols]
        n_placed[r:r1] = np.minimum(rank[:, -1], n_max).astype(np.int32)
        r = r1
    return k_list, n_placed, pts
