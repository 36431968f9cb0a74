"""Seeded synthetic scenes and rays for the occupancy-plane ray marcher.

This module is the ONLY code shared by the CPU oracle (``oracle/``) and the
HIP path (``paper_2404_09531_amd``).  It builds inputs and nothing else: it
holds none of the renderer's arithmetic (no sample placement, no
interpolation, no activation, no compositing, no MLP evaluation).

Representation built here (the paper's Sec. 3 MERF background and Sec. 4.1):

* scene box ``[-1,1]^2 x [0,0.25]`` with z up (the ground-aligned frame the
  paper assumes in Sec. 4.1);
* a low-resolution 3D feature grid ``grid[Lz][Ly][Lx][8]`` and three
  high-resolution planes ``plane_xy[Ny][Nx][8]``, ``plane_xz[Nz][Nx][8]``,
  ``plane_yz[Nz][Ny][8]`` (Eq. 2), channels last, float32;
* an occupancy plane ``occ[M][M][2]`` holding (z_min, z_max) per grid point
  (Sec. 4.1), float32;
* the deferred MLP 10 -> 16 -> 16 -> 3 packed as one float32 vector
  ``[W1(16x10), b1(16), W2(16x16), b2(16), W3(3x16), b3(3)]`` (Eq. 4,
  appendix A: three layers, 16 hidden units).

The terrain is a seeded sum of sinusoids about height 0.12; buildings
(box-shaped solid columns) or towers (thick occupancy intervals) are added
for the larger workloads.  Channel 0 of the grid carries the density
pre-activation profile ``8 * exp(-(dist/0.02)^2)`` where ``dist`` is the
vertical distance to the solid surface/column, plus N(0, 0.05) noise in each
of the four feature sources; channels 1..7 are N(0, 0.5) in each source.

Seeds: all randomness comes from ``numpy.random.SeedSequence`` children, so a
scene is a pure function of its config and seed.  Big arrays are filled in
fixed chunks by a thread pool, so the values do not depend on thread count.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, Optional, Tuple

import numpy as np

BOX_LO = (-1.0, -1.0, 0.0)
BOX_HI = (1.0, 1.0, 0.25)
# Lattice step: box height / 512 = 2^-11, exact in binary.
DELTA = 0.25 / 512.0
CHANNELS = 8
MLP_SHAPE = (10, 16, 16, 3)
MLP_NPARAMS = 16 * 10 + 16 + 16 * 16 + 16 + 3 * 16 + 3  # 499


def mlp_inputs(dir_freqs: int) -> int:
    """Deferred-MLP input width: 7 features + the view direction, raw (3) or
    with `dir_freqs` sine/cosine frequencies per component (3 + 6 freqs)."""
    return 7 + 3 * (1 + 2 * dir_freqs)


def mlp_nparams(dir_freqs: int) -> int:
    n = mlp_inputs(dir_freqs)
    return 16 * n + 16 + 16 * 16 + 16 + 3 * 16 + 3
BASE_HEIGHT = 0.12
HEIGHT_AMP = 0.05
DENSITY_PEAK = 8.0
DENSITY_WIDTH = 0.02

_CHUNK = 1 << 22  # elements per independently seeded noise chunk


@dataclasses.dataclass(frozen=True)
class SceneConfig:
    """Shape and structure of one synthetic scene."""

    grid: Tuple[int, int, int]          # (Lx, Ly, Lz) vertices
    planes: Tuple[int, int, int]        # (Nx, Ny, Nz) texels per axis
    occ: int                            # M (occupancy plane is M x M)
    band: float = 0.03                  # half thickness of terrain interval
    n_buildings: int = 0                # box buildings (footprint 2-8 cells)
    building_max_h: float = 0.2
    tower_fraction: float = 0.0         # fraction of cells covered by towers
    dir_freqs: int = 0                  # view-direction frequencies of the deferred MLP input
    seed: int = 0
    name: str = "custom"


TINY = SceneConfig(grid=(64, 64, 16), planes=(256, 256, 64), occ=32,
                   band=0.03, name="tiny-64x64x16")
OBLIQUE = SceneConfig(grid=(1024, 1024, 128), planes=(4096, 4096, 512),
                      occ=256, band=0.03, n_buildings=200,
                      name="oblique-1024x1024x128")
TOWERS = SceneConfig(grid=(1024, 1024, 128), planes=(4096, 4096, 512),
                     occ=512, band=0.01, tower_fraction=0.10,
                     name="towers-1024x1024x128-occ512")


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def fill_normal(out: np.ndarray, std: float, seq: np.random.SeedSequence) -> None:
    """Fill a contiguous float32 array with N(0, std) in fixed seeded chunks."""
    flat = out.reshape(-1)
    n = flat.size
    nchunks = (n + _CHUNK - 1) // _CHUNK
    children = seq.spawn(nchunks)

    def work(i: int) -> None:
        lo = i * _CHUNK
        hi = min(n, lo + _CHUNK)
        g = np.random.Generator(np.random.PCG64(children[i]))
        g.standard_normal(hi - lo, dtype=np.float32, out=flat[lo:hi])
        flat[lo:hi] *= np.float32(std)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nchunks)))


def _heightfield_params(seq: np.random.SeedSequence) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(seq))
    f = g.uniform(0.5, 4.0, 8)
    psi = g.uniform(0.0, 2.0 * math.pi, 8)
    phi = g.uniform(0.0, 2.0 * math.pi, 8)
    return np.stack([f, psi, phi], axis=1)


def terrain_height(x: np.ndarray, y: np.ndarray, hp: np.ndarray) -> np.ndarray:
    """0.12 + (0.05/8) * sum_k sin(2 pi f_k (cos psi_k x + sin psi_k y) + phi_k)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    acc = np.zeros(np.broadcast(x, y).shape, dtype=np.float64)
    for f, psi, phi in hp:
        acc += np.sin(2.0 * math.pi * f * (math.cos(psi) * x + math.sin(psi) * y) + phi)
    return BASE_HEIGHT + (HEIGHT_AMP / 8.0) * acc


def _cell_centres(m: int) -> np.ndarray:
    return BOX_LO[0] + (np.arange(m, dtype=np.float64) + 0.5) * (BOX_HI[0] - BOX_LO[0]) / m


def _buildings(m: int, count: int, max_h: float, seq) -> np.ndarray:
    """Per-cell solid height above terrain from `count` random box buildings."""
    g = np.random.Generator(np.random.PCG64(seq))
    hmap = np.zeros((m, m), dtype=np.float64)
    for _ in range(count):
        w = int(g.integers(2, 9))
        h = int(g.integers(2, 9))
        i0 = int(g.integers(0, m - w + 1))
        j0 = int(g.integers(0, m - h + 1))
        height = max_h * (1.0 - g.random())  # U(0, max_h]
        blk = hmap[j0:j0 + h, i0:i0 + w]
        np.maximum(blk, height, out=blk)
    return hmap


def _towers(m: int, fraction: float, seq) -> np.ndarray:
    """Per-cell interval thickness for clustered rectangular towers.

    Rectangles of 2-8 cells per side are dropped until `fraction` of the
    cells are covered; each gets a thickness ~ U(0.02, 0.25].
    """
    g = np.random.Generator(np.random.PCG64(seq))
    thick = np.zeros((m, m), dtype=np.float64)
    covered = 0
    target = int(fraction * m * m)
    while covered < target:
        w = int(g.integers(2, 9))
        h = int(g.integers(2, 9))
        i0 = int(g.integers(0, m - w + 1))
        j0 = int(g.integers(0, m - h + 1))
        t = 0.02 + 0.23 * (1.0 - g.random())  # U(0.02, 0.25]
        blk = thick[j0:j0 + h, i0:i0 + w]
        covered += int(np.count_nonzero(blk == 0.0))
        np.maximum(blk, t, out=blk)
    return thick


def _mlp_params(seq, dir_freqs: int = 0) -> np.ndarray:
    """Xavier-uniform weights, biases U(-0.1, 0.1); packed W1 b1 W2 b2 W3 b3."""
    g = np.random.Generator(np.random.PCG64(seq))
    shape = (mlp_inputs(dir_freqs),) + MLP_SHAPE[1:]
    parts = []
    for fin, fout in zip(shape[:-1], shape[1:]):
        a = math.sqrt(6.0 / (fin + fout))
        parts.append(g.uniform(-a, a, (fout, fin)).reshape(-1))
        parts.append(g.uniform(-0.1, 0.1, fout))
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == mlp_nparams(dir_freqs)
    return out


def mlp_params(dir_freqs: int, seed: int) -> np.ndarray:
    """Stand-alone seeded deferred-MLP parameter vector (same recipe as the
    scene's), e.g. to pair a built scene with the 34-input MLP."""
    return _mlp_params(np.random.SeedSequence(seed), dir_freqs)


def make_scene(cfg: SceneConfig, seed: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Build the seeded synthetic scene for `cfg`.

    Returns a dict of C-contiguous float32 arrays: ``grid``, ``plane_xy``,
    ``plane_xz``, ``plane_yz``, ``occ``, ``mlp`` and the float64 metadata
    ``box_lo``, ``box_hi``.
    """
    seed = cfg.seed if seed is None else seed
    ss = np.random.SeedSequence(seed)
    s_height, s_struct, s_grid, s_xy, s_xz, s_yz, s_mlp = ss.spawn(7)
    Lx, Ly, Lz = cfg.grid
    Nx, Ny, Nz = cfg.planes
    m = cfg.occ
    hp = _heightfield_params(s_height)

    # Occupancy plane: interval about the terrain at each cell centre.
    cx = _cell_centres(m)
    h_cell = terrain_height(cx[None, :], cx[:, None], hp)  # [j][i]
    solid = np.zeros((m, m))
    zmin = h_cell - cfg.band
    zmax = h_cell + cfg.band
    if cfg.n_buildings:
        solid = _buildings(m, cfg.n_buildings, cfg.building_max_h, s_struct)
        zmax = np.where(solid > 0, h_cell + solid + cfg.band, zmax)
    if cfg.tower_fraction > 0:
        thick = _towers(m, cfg.tower_fraction, s_struct)
        tower = thick > 0
        zmax = np.where(tower, zmin + thick, zmax)
        solid = np.where(tower, np.maximum(zmax - cfg.band - h_cell, 0.0), 0.0)
    occ = np.empty((m, m, 2), dtype=np.float32)
    occ[..., 0] = np.clip(zmin, BOX_LO[2], BOX_HI[2])
    occ[..., 1] = np.clip(zmax, BOX_LO[2], BOX_HI[2])

    # Grid: N(0,0.5) features; channel 0 = density profile + N(0,0.05).
    grid = np.empty((Lz, Ly, Lx, CHANNELS), dtype=np.float32)
    fill_normal(grid, 0.5, s_grid)
    gx = np.linspace(BOX_LO[0], BOX_HI[0], Lx)
    gy = np.linspace(BOX_LO[1], BOX_HI[1], Ly)
    gz = np.linspace(BOX_LO[2], BOX_HI[2], Lz)
    h_v = terrain_height(gx[None, :], gy[:, None], hp)  # [Ly][Lx]
    ci = np.clip(np.floor((gx - BOX_LO[0]) / (BOX_HI[0] - BOX_LO[0]) * m).astype(np.int64), 0, m - 1)
    cj = np.clip(np.floor((gy - BOX_LO[1]) / (BOX_HI[1] - BOX_LO[1]) * m).astype(np.int64), 0, m - 1)
    top_v = h_v + solid[cj[:, None], ci[None, :]]
    h32 = h_v.astype(np.float32)
    t32 = top_v.astype(np.float32)

    def density_slice(k: int) -> None:
        z = np.float32(gz[k])
        dist = np.maximum(np.maximum(h32 - z, z - t32), np.float32(0.0))
        prof = np.float32(DENSITY_PEAK) * np.exp(-np.square(dist / np.float32(DENSITY_WIDTH)))
        sl = grid[k, :, :, 0]
        sl *= np.float32(0.1)  # N(0,0.5) -> N(0,0.05)
        sl += prof

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(density_slice, range(Lz)))

    planes = {}
    for name, shape, s in (("plane_xy", (Ny, Nx), s_xy), ("plane_xz", (Nz, Nx), s_xz),
                           ("plane_yz", (Nz, Ny), s_yz)):
        p = np.empty(shape + (CHANNELS,), dtype=np.float32)
        fill_normal(p, 0.5, s)
        p[..., 0] *= np.float32(0.1)
        planes[name] = p

    return dict(grid=grid, occ=occ, mlp=_mlp_params(s_mlp, cfg.dir_freqs), dir_freqs=cfg.dir_freqs,
                box_lo=np.array(BOX_LO), box_hi=np.array(BOX_HI), **planes)


def perturb_scene(scene: Dict[str, np.ndarray], std: float, seed: int) -> Dict[str, np.ndarray]:
    """Copy of `scene` with N(0, std) added to every feature and MLP param.

    The occupancy plane is left unchanged (it is not a trainable input of
    the render path).
    """
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(5)
    out = dict(scene)
    for key, s in zip(("grid", "plane_xy", "plane_xz", "plane_yz", "mlp"), kids):
        noise = np.empty_like(scene[key])
        fill_normal(noise, std, s)
        noise += scene[key]
        out[key] = noise
    return out


# ----------------------------------------------------------------------------
# Rays.  Built in float64, rounded to float32 once; these float32 arrays are
# the only ray input to both the oracle and the GPU path.
# ----------------------------------------------------------------------------

def _dir(pitch: np.ndarray, yaw: np.ndarray) -> np.ndarray:
    return np.stack([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), -np.sin(pitch)], axis=-1)


def oblique_rays(n: int, seed: int = 1, pitch_deg=(30.0, 60.0), origin_z: float = 1.0,
                 aim_z: float = BASE_HEIGHT) -> Tuple[np.ndarray, np.ndarray]:
    """Independent rays: aim point U([-1,1]^2) at height aim_z, pitch
    U[pitch_deg] below the horizon, yaw U[0, 2pi); origin moved back along
    the ray to z = origin_z (set exactly)."""
    g = np.random.Generator(np.random.PCG64(seed))
    aim = np.stack([g.uniform(-1, 1, n), g.uniform(-1, 1, n), np.full(n, aim_z)], axis=1)
    pitch = np.radians(g.uniform(pitch_deg[0], pitch_deg[1], n))
    yaw = g.uniform(0.0, 2.0 * math.pi, n)
    d = _dir(pitch, yaw)
    s = (origin_z - aim_z) / np.sin(pitch)
    o = aim - s[:, None] * d
    o[:, 2] = origin_z
    return o.astype(np.float32), d.astype(np.float32)


SMOOTH_SIGMA2 = 0.3  # per-component variance of the direction perturbation (Sigma = 0.3 I)


def view_perturbations(n: int, count: int, seed: int, variance: float = SMOOTH_SIGMA2) -> np.ndarray:
    """Gaussian direction perturbations delta ~ N(0, variance I), float32
    [n, count, 3], for the view-smoothness loss; the loss adds them to the
    ray directions."""
    g = np.random.Generator(np.random.PCG64(seed))
    return (g.standard_normal((n, count, 3)) * math.sqrt(variance)).astype(np.float32)


def camera_rays(width: int, height: int, pitch_deg: float, yaw_deg: float,
                aim=(0.0, 0.0, BASE_HEIGHT), origin_z: float = 1.0, hfov_deg: float = 60.0,
                pixels: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Pinhole camera looking at `aim` from height origin_z; rays through
    pixel centres, row-major.  If `pixels` (int64 flat indices) is given,
    only those rays are built."""
    pitch = math.radians(pitch_deg)
    yaw = math.radians(yaw_deg)
    fwd = _dir(np.array(pitch), np.array(yaw))
    right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    s = (origin_z - aim[2]) / math.sin(pitch)
    origin = np.asarray(aim, dtype=np.float64) - s * fwd
    origin[2] = origin_z
    if pixels is None:
        pixels = np.arange(width * height, dtype=np.int64)
    px = (pixels % width).astype(np.float64)
    py = (pixels // width).astype(np.float64)
    tx = math.tan(math.radians(hfov_deg) / 2.0)
    sx = ((px + 0.5) / width * 2.0 - 1.0) * tx
    sy = (1.0 - (py + 0.5) / height * 2.0) * tx * height / width
    d = fwd[None, :] + sx[:, None] * right[None, :] + sy[:, None] * up[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(origin, d.shape)
    return np.ascontiguousarray(o, dtype=np.float32), d.astype(np.float32)


def pixel_order(width: int, height: int, order: str = "row") -> np.ndarray:
    """Flat pixel indices in the order rays are issued.

    "row": row-major.  "tile4": 4x4 pixel tiles in row-major tile order;
    inside a tile the four 2x2 quads in row-major order, each quad
    row-major (16 consecutive rays = one 4x4 tile, 4 rays = one quad).
    Image sides must be multiples of 4 for "tile4".  "morton": Z-order of
    (x, y), so every aligned run of 4^k rays is a 2^k x 2^k square (where it
    lies inside the image)."""
    if order == "row":
        return np.arange(width * height, dtype=np.int64)
    if order == "morton":
        y, x = np.divmod(np.arange(width * height, dtype=np.int64), width)
        key = np.zeros_like(x)
        for b in range(16):
            key |= ((x >> b) & 1) << (2 * b)
            key |= ((y >> b) & 1) << (2 * b + 1)
        return np.argsort(key, kind="stable").astype(np.int64)
    if order != "tile4":
        raise KeyError(order)
    if width % 4 or height % 4:
        raise ValueError("tile4 order needs sides that are multiples of 4")
    ty, tx, qy, qx, py, px = np.meshgrid(np.arange(height // 4), np.arange(width // 4), np.arange(2),
                                         np.arange(2), np.arange(2), np.arange(2), indexing="ij")
    y = ty * 4 + qy * 2 + py
    x = tx * 4 + qx * 2 + px
    return (y * width + x).reshape(-1).astype(np.int64)


def random_cameras(count: int, seed: int, pitch_deg=(30.0, 60.0), aim_range: float = 0.8):
    """List of (pitch_deg, yaw_deg, aim) for `count` seeded oblique cameras."""
    g = np.random.Generator(np.random.PCG64(seed))
    cams = []
    for _ in range(count):
        p = float(g.uniform(*pitch_deg))
        y = float(g.uniform(0.0, 360.0))
        a = (float(g.uniform(-aim_range, aim_range)), float(g.uniform(-aim_range, aim_range)), BASE_HEIGHT)
        cams.append((p, y, a))
    return cams


def multi_camera_rays(n: int, cams, width: int, height: int, seed: int):
    """`n` rays drawn uniformly over (camera, pixel) pairs."""
    g = np.random.Generator(np.random.PCG64(seed))
    cam = g.integers(0, len(cams), n)
    pix = g.integers(0, width * height, n)
    o = np.empty((n, 3), dtype=np.float32)
    d = np.empty((n, 3), dtype=np.float32)
    for c, (p, y, a) in enumerate(cams):
        sel = np.nonzero(cam == c)[0]
        if sel.size:
            oc, dc = camera_rays(width, height, p, y, a, pixels=pix[sel])
            o[sel] = oc
            d[sel] = dc
    return o, d


def workload(name: str):
    """Named workloads: returns (scene_cfg, ray recipe dict)."""
    if name == "tiny":
        return TINY, dict(kind="oblique", n=4096, seed=1, n_max=64)
    if name == "oblique-1080p":
        return OBLIQUE, dict(kind="camera", width=1920, height=1080, pitch=45.0, yaw=90.0, n_max=256,
                             order="morton")
    if name == "train-2^18":
        return OBLIQUE, dict(kind="multi", n=1 << 18, cameras=16, width=1920, height=1080, seed=1, n_max=256)
    if name == "bf16-4k-x8":
        return OBLIQUE, dict(kind="cams", cameras=8, width=3840, height=2160, seed=1, n_max=256)
    if name == "towers-2^20":
        return TOWERS, dict(kind="multi", n=1 << 20, cameras=64, width=1920, height=1080, seed=1, n_max=512)
    raise KeyError(name)


def make_rays(recipe: dict):
    kind = recipe["kind"]
    if kind == "oblique":
        return oblique_rays(recipe["n"], recipe.get("seed", 1))
    if kind == "camera":
        px = pixel_order(recipe["width"], recipe["height"], recipe.get("order", "row"))
        return camera_rays(recipe["width"], recipe["height"], recipe["pitch"], recipe["yaw"], pixels=px)
    if kind == "multi":
        cams = random_cameras(recipe["cameras"], recipe.get("seed", 1))
        return multi_camera_rays(recipe["n"], cams, recipe["width"], recipe["height"], recipe.get("seed", 1) + 100)
    raise KeyError(kind)
