"""8-bit feature storage (TEST INFRASTRUCTURE).

Oblique-MERF bakes its features for the real-time viewer and stores them
as 8-bit images (Sec. 4.4, following MERF).  The paper gives no code
mapping; the reading used here:

* Each channel c of each feature source (grid, three planes) is stored as
  an unsigned byte q with value lo_c + q * step_c.  lo_c is the channel's
  minimum over the source and step_c = fl32((max_c - lo_c) / 255), so the
  codes span the channel's range (step 0 for a constant channel).
* Encoding rounds to the nearest code, ties to even, then clamps into
  [0, 255].  The code is an integer decided by floating point, so it is
  decided in binary32, the precision of the stored float32 features:
  q = clamp(rint(fl32(fl32(x - lo) * inv)), 0, 255) with inv = fl32(1 / step)
  (0 when step = 0).  A NaN feature encodes as 0.
* Decoding is the plain definition lo + q * step, evaluated here in float64
  (exact: q has 8 bits and step 24).

The render of an 8-bit scene is the render of its decoded scene
(``dequantize_scene`` then ``render.oracle_render``).
"""
from typing import Dict

import numpy as np

SOURCES = ("grid", "plane_xy", "plane_xz", "plane_yz")


def feature_range(x: np.ndarray) -> np.ndarray:
    """Per-channel (min, max) of a float32 feature array [..., 8] -> [8, 2]."""
    flat = np.asarray(x, dtype=np.float32).reshape(-1, 8)
    return np.stack([flat.min(axis=0), flat.max(axis=0)], axis=1)


def quant_params(minmax: np.ndarray):
    """(lo, step) float32 [8] from a channel range [8, 2]: lo = min,
    step = fl32((max - min) / 255), both in binary32 arithmetic."""
    mm = np.asarray(minmax, dtype=np.float32)
    lo = mm[:, 0].copy()
    step = ((mm[:, 1] - mm[:, 0]) / np.float32(255.0)).astype(np.float32)
    return lo, step


def _inverse(step: np.ndarray) -> np.ndarray:
    step = np.asarray(step, dtype=np.float32)
    with np.errstate(divide="ignore"):
        inv = np.float32(1.0) / step
    return np.where(step > 0, inv, np.float32(0.0)).astype(np.float32)


def quantize_u8(x: np.ndarray, lo: np.ndarray, step: np.ndarray) -> np.ndarray:
    """Codes of float32 features [..., 8] for per-channel (lo, step)."""
    x = np.asarray(x, dtype=np.float32)
    lo = np.asarray(lo, dtype=np.float32)
    inv = _inverse(step)
    with np.errstate(invalid="ignore", over="ignore"):
        y = (x - lo).astype(np.float32) * inv  # two binary32 roundings
        y = np.rint(y.astype(np.float32))      # nearest, ties to even
    y = np.where(np.isnan(y), 0.0, y)
    return np.clip(y, 0.0, 255.0).astype(np.uint8)


def dequantize(q: np.ndarray, lo: np.ndarray, step: np.ndarray) -> np.ndarray:
    """Decoded features lo + q * step (float64)."""
    return (np.asarray(lo, dtype=np.float64)
            + np.asarray(q, dtype=np.float64) * np.asarray(step, dtype=np.float64))


def quantize_scene(scene: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """8-bit copy of a float32 scene: each source's codes (uint8, same
    shape), and quant_lo / quant_step float32 [4, 8] (sources in the order
    grid, XY, XZ, YZ) from each source's own channel ranges."""
    out = dict(scene)
    lo_all = np.zeros((4, 8), np.float32)
    step_all = np.zeros((4, 8), np.float32)
    for i, src in enumerate(SOURCES):
        lo, step = quant_params(feature_range(scene[src]))
        out[src] = quantize_u8(scene[src], lo, step)
        lo_all[i], step_all[i] = lo, step
    out["quant_lo"], out["quant_step"] = lo_all, step_all
    return out


def dequantize_scene(scene_u8: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """The float64 scene an 8-bit scene stands for."""
    out = dict(scene_u8)
    for i, src in enumerate(SOURCES):
        out[src] = dequantize(scene_u8[src], scene_u8["quant_lo"][i], scene_u8["quant_step"][i])
    return out
