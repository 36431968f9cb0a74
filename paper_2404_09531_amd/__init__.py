"""MI355X-native (gfx950) occupancy-plane ray marcher of Oblique-MERF (arXiv 2404.09531).

Python surface over the C ABI (include/omerf.h, libomerf.so):

* :class:`Scene` -- a MERF scene (3D grid + XY/XZ/YZ planes, Sec. 3 Eq. 2),
  its occupancy plane (Sec. 4.1) and the deferred MLP (Eq. 4), as device
  tensors borrowed by a library handle;
* :func:`place_samples` -- the samples the marcher places (Sec. 4.1 Eq. 6-7);
* :func:`render` -- forward render (Eq. 1-4);
* :func:`render_backward` -- gradients into grid, planes and MLP;
* :class:`RenderFn` -- ``torch.autograd.Function`` over render/backward;
* :func:`l2_loss_fp64`, :func:`l2_loss_grad` -- loss kernels.

All computation runs in the library's HIP kernels on the caller's current
stream; these wrappers only check tensor metadata and marshal pointers.
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, Optional, Sequence

import torch

from . import _lib
from ._lib import OM_BF16, OM_F32, OM_MAX_SAMPLES, OM_U8, OmerfError

DELTA = 0.25 / 512  # lattice step: box height / 512 (2^-11)
MLP_NPARAMS = 499  # N = 10 inputs (no direction encoding)


def mlp_nparams(dir_freqs: int = 0) -> int:
    """Packed parameter count of the N -> 16 -> 16 -> 3 deferred MLP with
    N = 10 + 6 dir_freqs inputs (499 or 883)."""
    return 16 * (10 + 6 * dir_freqs) + 16 + 256 + 16 + 48 + 3


_FREQS_OF = {mlp_nparams(0): 0, mlp_nparams(4): 4}

__all__ = ["Scene", "place_samples", "render", "render_backward", "backward_workspace_size", "RenderFn", "SmoothFn", "smooth_loss",
           "l2_loss_fp64", "l2_loss_grad", "occ_interval_loss", "mlp_nparams", "feature_range", "quant_params",
           "quantize_u8", "quantize_features", "sparse_grid", "SparseGrid", "DELTA", "OmerfError",
           "OM_MAX_SAMPLES", "to_bf16", "mark_rows"]


def _need(t: torch.Tensor, name: str, dtype, shape=None) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def to_bf16(t: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """bfloat16 shadow of a float32 tensor, rounded to nearest even by the
    library (om_cast_bf16), into `out` (bfloat16, same shape; allocated if
    None) -- the re-cast of a bfloat16 scene after an optimiser step on its
    float32 master copy."""
    _need(t, "src", torch.float32)
    if out is None:
        out = torch.empty(t.shape, dtype=torch.bfloat16, device=t.device)
    _need(out, "out", torch.bfloat16, t.shape)
    _lib.check("om_cast_bf16", _lib.lib().om_cast_bf16(t.data_ptr(), t.numel(), out.data_ptr(), _lib.stream_of(t)))
    return out


def order_rays_workspace_size(n: int) -> int:
    """Bytes of workspace order_rays needs (om_order_rays_workspace_size)."""
    nb = _lib.lib().om_order_rays_workspace_size(n)
    if nb < 0:
        raise _lib.OmerfError("om_order_rays_workspace_size", _lib.OM_ERR_INVALID, _lib.lib().om_last_error().decode())
    return int(nb)


def order_rays(scene, o, d, out=None, workspace=None):
    """Locality order of a batch of rays (om_order_rays): returns (order
    int32 [n], o[order], d[order]).  `out` may hold preallocated
    (order, o_sorted, d_sorted) tensors; `workspace` a uint8 device tensor
    of order_rays_workspace_size(n) bytes (allocated if None)."""
    n = o.shape[0]
    _need(o, "o", torch.float32, (n, 3))
    _need(d, "d", torch.float32, (n, 3))
    if out is None:
        out = (torch.empty((n,), dtype=torch.int32, device=o.device), torch.empty_like(o), torch.empty_like(d))
    order, os_, ds_ = out
    _need(order, "order", torch.int32, (n,))
    _need(os_, "o_sorted", torch.float32, (n, 3))
    _need(ds_, "d_sorted", torch.float32, (n, 3))
    nb = order_rays_workspace_size(n)
    if workspace is None:
        workspace = torch.empty((max(nb, 1),), dtype=torch.uint8, device=o.device)
    _lib.check("om_order_rays", _lib.lib().om_order_rays(scene.handle, o.data_ptr(), d.data_ptr(), n,
                                                         order.data_ptr(), os_.data_ptr(), ds_.data_ptr(),
                                                         workspace.data_ptr(), workspace.numel(), _lib.stream_of(o)))
    return order, os_, ds_


def _rows(t, name):
    if t.dim() not in (1, 2):
        raise ValueError(f"{name}: rows of floats expected, got shape {tuple(t.shape)}")
    return t.shape[0], (t.shape[1] if t.dim() == 2 else 1)


def gather_rows(src, idx, out=None):
    """out[i] = src[idx[i]] on float32 rows (om_gather_rows)."""
    rows, cols = _rows(src, "src")
    _need(src, "src", torch.float32)
    _need(idx, "idx", torch.int32, (idx.shape[0],))
    shape = (idx.shape[0],) + tuple(src.shape[1:])
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=src.device)
    _need(out, "out", torch.float32, shape)
    _lib.check("om_gather_rows", _lib.lib().om_gather_rows(src.data_ptr(), rows, cols, idx.data_ptr(), idx.shape[0],
                                                           out.data_ptr(), _lib.stream_of(src)))
    return out


def scatter_rows(src, idx, out):
    """out[idx[i]] = src[i] on float32 rows (om_scatter_rows)."""
    n, cols = _rows(src, "src")
    _need(src, "src", torch.float32)
    _need(idx, "idx", torch.int32, (n,))
    _need(out, "out", torch.float32)
    if tuple(out.shape[1:]) != tuple(src.shape[1:]):
        raise ValueError(f"out: rows of shape {tuple(src.shape[1:])} expected, got {tuple(out.shape[1:])}")
    _lib.check("om_scatter_rows", _lib.lib().om_scatter_rows(src.data_ptr(), cols, idx.data_ptr(), n, out.data_ptr(),
                                                             out.shape[0], _lib.stream_of(src)))
    return out


class Scene:
    """Library handle over borrowed device tensors.

    grid [Lz,Ly,Lx,8], plane_xy [Ny,Nx,8], plane_xz [Nz,Nx,8], plane_yz
    [Nz,Ny,8] (all float32, all bfloat16, or all uint8 codes with
    quant=(lo, step), [4, 8] each, from quantize_features: render only),
    occ float32 [My,Mx,2], mlp float32 [499] (MLP input [F, d]) or [883]
    (input [F, d, sin/cos of 2^k d for k = 0..3], Sec. 4.2); the width
    selects the encoding.  The tensors are referenced (kept alive) by the
    Scene, never copied."""

    def __init__(self, grid, plane_xy, plane_xz, plane_yz, occ, mlp,
                 box_lo: Sequence[float] = (-1.0, -1.0, 0.0), box_hi: Sequence[float] = (1.0, 1.0, 0.25),
                 quant=None, sparse=None):
        self._handle = ctypes.c_void_p()
        self.mips, self.mip_levels = None, 0
        self._set(grid, plane_xy, plane_xz, plane_yz, occ, mlp, box_lo, box_hi, quant, sparse)
        _lib.check("om_scene_create", _lib.lib().om_scene_create(ctypes.byref(self._desc), ctypes.byref(self._handle)))

    def _set(self, grid, plane_xy, plane_xz, plane_yz, occ, mlp, box_lo, box_hi, quant=None, sparse=None):
        dt = grid.dtype
        if dt not in (torch.float32, torch.bfloat16, torch.uint8):
            raise TypeError("grid/planes must be float32, bfloat16 or uint8")
        if (dt == torch.uint8) != (quant is not None):
            raise ValueError("uint8 features need quant=(lo, step), [4, 8] each; other dtypes take none")
        if sparse is None:
            lz, ly, lx, ch = grid.shape
        else:  # atlas [n_blocks + 1, B + 1, B + 1, B + 1, 8] over a logical (Lx, Ly, Lz) grid
            lx, ly, lz = sparse.dims
            e = (1 << sparse.shift) + 1
            ch = grid.shape[-1]
            if tuple(grid.shape) != (sparse.n_blocks + 1, e, e, e, 8):
                raise ValueError(f"sparse grid atlas must be [{sparse.n_blocks + 1}, {e}, {e}, {e}, 8]")
            _need(sparse.blocks, "grid_blocks", torch.int32, sparse.index_shape())
        if ch != 8:
            raise ValueError("8 channels expected")
        ny, nx = plane_xy.shape[:2]
        nz = plane_xz.shape[0]
        _need(grid, "grid", dt)
        _need(plane_xy, "plane_xy", dt, (ny, nx, 8))
        _need(plane_xz, "plane_xz", dt, (nz, nx, 8))
        _need(plane_yz, "plane_yz", dt, (nz, ny, 8))
        my, mx = occ.shape[:2]
        _need(occ, "occ", torch.float32, (my, mx, 2))
        _need(mlp, "mlp", torch.float32)
        if mlp.dim() != 1 or mlp.numel() not in _FREQS_OF:
            raise ValueError(f"mlp must be float32 [{mlp_nparams(0)}] or [{mlp_nparams(4)}], got {tuple(mlp.shape)}")
        d = _lib.OmSceneDesc()
        d.box_lo[:] = list(box_lo)
        d.box_hi[:] = list(box_hi)
        d.grid_dims[:] = [lx, ly, lz]
        d.plane_dims[:] = [nx, ny, nz]
        d.occ_dims[:] = [mx, my]
        d.dtype = {torch.bfloat16: OM_BF16, torch.uint8: OM_U8}.get(dt, OM_F32)
        if quant is not None:
            lo, step = (torch.as_tensor(q, dtype=torch.float32).reshape(4, 8).tolist() for q in quant)
            for i in range(4):
                d.quant_lo[i][:] = lo[i]
                d.quant_step[i][:] = step[i]
        self.quant = quant
        d.grid, d.plane_xy, d.plane_xz, d.plane_yz = grid.data_ptr(), plane_xy.data_ptr(), plane_xz.data_ptr(), \
            plane_yz.data_ptr()
        d.occ, d.mlp = occ.data_ptr(), mlp.data_ptr()
        d.dir_freqs = _FREQS_OF[mlp.numel()]
        self.dir_freqs = d.dir_freqs
        if sparse is not None:
            d.grid_blocks, d.block_shift, d.n_blocks = sparse.blocks.data_ptr(), sparse.shift, sparse.n_blocks
        self.sparse = sparse
        self._desc = d
        self.tensors = dict(grid=grid, plane_xy=plane_xy, plane_xz=plane_xz, plane_yz=plane_yz, occ=occ, mlp=mlp)
        self.dtype = dt
        self.device = grid.device

    def update(self, **tensors) -> None:
        """Re-point the handle at new tensors (same keys as the constructor)."""
        quant = tensors.pop("quant", self.quant)
        sparse = tensors.pop("sparse", self.sparse)
        t = dict(self.tensors)
        t.update(tensors)
        if t["grid"].dtype != torch.uint8:
            quant = None
        old = (self._desc, self.tensors, self.dtype, self.quant, self.dir_freqs, self.sparse)
        self._set(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], t["mlp"],
                  tuple(self._desc.box_lo), tuple(self._desc.box_hi), quant, sparse)
        rc = _lib.lib().om_scene_update(self._handle, ctypes.byref(self._desc))
        if rc != 0:
            self._desc, self.tensors, self.dtype, self.quant, self.dir_freqs, self.sparse = old
            _lib.check("om_scene_update", rc)
        self.mips = None  # the library detached the pyramid; build it again if wanted
        self.mip_levels = 0

    def build_occupancy_mips(self, levels: int) -> None:
        """Compute the occupancy pyramid (levels 1..levels of pooled
        (min z_min, max z_max) blocks) into a device buffer held by this
        Scene and attach it, so placement skips empty space hierarchically;
        levels=0 detaches it."""
        L = _lib.lib()
        nbytes = L.om_occupancy_mips_size(self._handle, levels)
        if nbytes < 0:
            raise _lib.OmerfError("om_occupancy_mips_size", _lib.OM_ERR_UNSUPPORTED, L.om_last_error().decode())
        buf = torch.empty((max(nbytes, 8),), dtype=torch.uint8, device=self.device) if levels > 0 else None
        _lib.check("om_build_occupancy_mips", L.om_build_occupancy_mips(
            self._handle, _lib.ptr(buf), nbytes, levels, _lib.stream_of(self.tensors["occ"])))
        self.mips, self.mip_levels = buf, levels

    def occupancy_mips(self):
        """The attached pyramid as a list of float32 [My >> l, Mx >> l, 2]
        views, level 1 first (empty list if none)."""
        out, off = [], 0
        my, mx = self.tensors["occ"].shape[:2]
        if self.mips is None:
            return out
        flat = self.mips.view(torch.float32)
        for lvl in range(1, self.mip_levels + 1):
            h, w = my >> lvl, mx >> lvl
            out.append(flat[off:off + h * w * 2].view(h, w, 2))
            off += h * w * 2
        return out

    @property
    def handle(self):
        return self._handle

    def __del__(self):
        # may run during interpreter shutdown, when module globals are gone
        try:
            h = self._handle
            if h is not None and h.value:
                _lib.lib().om_scene_destroy(h)
                h.value = None
        except Exception:
            pass


def _params(n_max: int, delta: float, t_term: float, c_bg, mlp_bf16: int, occ_eps: float = 0.0) -> _lib.OmParams:
    p = _lib.OmParams()
    p.occ_eps = float(occ_eps)
    p.delta = delta
    p.n_max = int(n_max)
    p.t_term = float(t_term)
    p.c_bg[:] = [float(v) for v in c_bg]
    p.mlp_bf16 = int(mlp_bf16)
    return p


def _rays(scene: Scene, o: torch.Tensor, d: torch.Tensor) -> int:
    n = o.shape[0]
    _need(o, "o", torch.float32, (n, 3))
    _need(d, "d", torch.float32, (n, 3))
    if o.device != scene.device:
        raise ValueError("rays and scene must be on the same device")
    return n


def place_samples(scene: Scene, o, d, n_max: int, delta: float = DELTA):
    """Accepted lattice indices per ray (int32 [n, n_max], -1 padded) and counts."""
    n = _rays(scene, o, d)
    k = torch.empty((n, n_max), dtype=torch.int32, device=o.device)
    cnt = torch.empty((n,), dtype=torch.int32, device=o.device)
    p = _params(n_max, delta, 0.0, (0, 0, 0), -1)
    _lib.check("om_place_samples", _lib.lib().om_place_samples(scene.handle, o.data_ptr(), d.data_ptr(), n,
                                                                 ctypes.byref(p), k.data_ptr(), cnt.data_ptr(),
                                                                 _lib.stream_of(o)))
    return k, cnt


def mark_rows(scene: Scene, o, d, n_max: int, n_eval: Optional[torch.Tensor] = None, delta: float = DELTA,
              flags: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
    """uint8 flags per feature row (keys grid, plane_xy, plane_xz, plane_yz;
    one byte per vertex / texel, 1 where some evaluated sample of the rays
    reads it: the first n_eval placed samples, or all placed samples).
    `flags` (optional, zeroed by the caller) accumulates instead."""
    n = _rays(scene, o, d)
    if n_eval is not None:
        _need(n_eval, "n_eval", torch.int32, (n,))
    src = scene.tensors
    if flags is None:
        flags = {k: torch.zeros(src[k].shape[:-1], dtype=torch.uint8, device=o.device)
                 for k in ("grid", "plane_xy", "plane_xz", "plane_yz")}
    for k in ("grid", "plane_xy", "plane_xz", "plane_yz"):
        _need(flags[k], f"flags[{k}]", torch.uint8, src[k].shape[:-1])
    p = _params(n_max, delta, 0.0, (0, 0, 0), -1)
    _lib.check("om_mark_rows", _lib.lib().om_mark_rows(
        scene.handle, o.data_ptr(), d.data_ptr(), n, ctypes.byref(p), _lib.ptr(n_eval), flags["grid"].data_ptr(),
        flags["plane_xy"].data_ptr(), flags["plane_xz"].data_ptr(), flags["plane_yz"].data_ptr(), _lib.stream_of(o)))
    return flags


BATCH = 16  # samples per batch of the per-batch w v sums (OM_BATCH)


def batch_slots(n_max: int) -> int:
    """Per-ray slots of the optional `batch_wv` output (OM_BATCH_SLOTS)."""
    return (n_max + BATCH - 1) // BATCH


def render(scene: Scene, o, d, n_max: int, delta: float = DELTA, t_term: float = 0.0,
           c_bg=(0.0, 0.0, 0.0), mlp_bf16: int = -1, batch_wv: bool = False,
           occ_eps: float = 0.0) -> Dict[str, torch.Tensor]:
    """Forward render; returns C [n,3], T [n], F [n,7], n_placed [n], n_eval [n]
    and, with batch_wv=True, the per-batch sums of w v [n, batch_slots(n_max), 7]
    that let the backward skip one replay of the samples.  occ_eps > 0
    applies the soft occupancy value of Eq. 6 to the weights (Eq. 8)."""
    n = _rays(scene, o, d)
    dev = o.device
    out = dict(C=torch.empty((n, 3), dtype=torch.float32, device=dev),
               T=torch.empty((n,), dtype=torch.float32, device=dev),
               F=torch.empty((n, 7), dtype=torch.float32, device=dev),
               n_placed=torch.empty((n,), dtype=torch.int32, device=dev),
               n_eval=torch.empty((n,), dtype=torch.int32, device=dev))
    if batch_wv:
        out["batch_wv"] = torch.empty((n, batch_slots(n_max), 7), dtype=torch.float32, device=dev)
    render_into(scene, o, d, out, n_max, delta, t_term, c_bg, mlp_bf16, occ_eps=occ_eps)
    return out


def _batch_wv(out, n: int, n_max: int) -> int:
    bw = out.get("batch_wv")
    if bw is None:
        return 0
    _need(bw, "batch_wv", torch.float32, (n, batch_slots(n_max), 7))
    return bw.data_ptr()


def _fwd_out(out, n: int, n_max: int):
    return _lib.OmFwdOut(_lib.ptr(out.get("C")), out["T"].data_ptr(), out["F"].data_ptr(),
                         _lib.ptr(out.get("n_placed")), out["n_eval"].data_ptr(), _batch_wv(out, n, n_max))


def render_into(scene: Scene, o, d, out: Dict[str, torch.Tensor], n_max: int, delta: float = DELTA,
                t_term: float = 0.0, c_bg=(0.0, 0.0, 0.0), mlp_bf16: int = -1, stage: str = "all",
                occ_eps: float = 0.0) -> None:
    """Forward render into preallocated outputs (same keys as render(); an
    optional "batch_wv" entry receives the per-batch w v sums).

    stage="all" runs om_render; "march" only om_march (F, T, counts);
    "mlp" only om_deferred_mlp (C from F, T, n_eval)."""
    n = o.shape[0]
    fo = _fwd_out(out, n, n_max)
    p = _params(n_max, delta, t_term, c_bg, mlp_bf16, occ_eps)
    L = _lib.lib()
    st = _lib.stream_of(o)
    if stage == "all":
        _lib.check("om_render", L.om_render(scene.handle, o.data_ptr(), d.data_ptr(), n, ctypes.byref(p),
                                            ctypes.byref(fo), st))
    elif stage == "march":
        _lib.check("om_march", L.om_march(scene.handle, o.data_ptr(), d.data_ptr(), n, ctypes.byref(p),
                                          ctypes.byref(fo), st))
    elif stage == "mlp":
        _lib.check("om_deferred_mlp", L.om_deferred_mlp(scene.handle, d.data_ptr(), n, ctypes.byref(p),
                                                        ctypes.byref(fo), st))
    else:
        raise ValueError(stage)


def render_backward(scene: Scene, o, d, saved: Dict[str, torch.Tensor], dL_dC, grads: Dict[str, torch.Tensor],
                    n_max: int, delta: float = DELTA, t_term: float = 0.0, c_bg=(0.0, 0.0, 0.0),
                    occ_eps: float = 0.0, dL_dF: Optional[torch.Tensor] = None,
                    workspace: Optional[torch.Tensor] = None) -> None:
    """Accumulate dL/d(grid, planes, mlp) into float32 `grads` (keys grid,
    plane_xy, plane_xz, plane_yz, mlp) given dL/dC and the forward's outputs
    (with "batch_wv" among them when the forward wrote it).  With
    occ_eps > 0 an optional grads["occ"] [My, Mx, 2] receives dL/d(z_min, z_max).
    dL_dF (float32 [n, 7], optional) is an extra upstream gradient on the
    composited features, e.g. from smooth_loss.  `workspace`: optional
    device uint8 tensor of at least backward_workspace_size(n) bytes (the
    per-ray hand-over between the MLP backward and the march backward);
    allocated here when None."""
    n = _rays(scene, o, d)
    _need(dL_dC, "dL_dC", torch.float32, (n, 3))
    if dL_dF is not None:
        _need(dL_dF, "dL_dF", torch.float32, (n, 7))
    for key in ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp"):
        _need(grads[key], f"grads[{key}]", torch.float32, scene.tensors[key].shape)
    fo = _lib.OmFwdOut(saved["C"].data_ptr(), saved["T"].data_ptr(), saved["F"].data_ptr(),
                       saved["n_placed"].data_ptr(), saved["n_eval"].data_ptr(), _batch_wv(saved, n, n_max))
    g = _grads(scene, grads)
    p = _params(n_max, delta, t_term, c_bg, -1, occ_eps)
    nbytes = backward_workspace_size(n)
    if workspace is None:
        workspace = torch.empty((max(nbytes, 1),), dtype=torch.uint8, device=o.device)
    _need_workspace(workspace, nbytes, o.device)
    _lib.check("om_render_backward_ex", _lib.lib().om_render_backward_ex(
        scene.handle, o.data_ptr(), d.data_ptr(), n, ctypes.byref(p), ctypes.byref(fo), dL_dC.data_ptr(),
        _lib.ptr(dL_dF), workspace.data_ptr(), workspace.numel(), ctypes.byref(g), _lib.stream_of(o)))


def backward_workspace_size(n: int) -> int:
    """Bytes of workspace render_backward needs (om_render_backward_workspace_size)."""
    nb = _lib.lib().om_render_backward_workspace_size(n)
    if nb < 0:
        raise _lib.OmerfError("om_render_backward_workspace_size", _lib.OM_ERR_INVALID,
                              _lib.lib().om_last_error().decode())
    return int(nb)


def fwd_bwd_l2_workspace_size(n: int, n_max: int, delta: float = DELTA) -> int:
    """Bytes of workspace render_fwd_bwd_l2 needs (om_render_fwd_bwd_l2_workspace_size)."""
    p = _params(n_max, delta, 0.0, (0.0, 0.0, 0.0), -1)
    nb = _lib.lib().om_render_fwd_bwd_l2_workspace_size(n, ctypes.byref(p))
    if nb < 0:
        raise _lib.OmerfError("om_render_fwd_bwd_l2_workspace_size", _lib.OM_ERR_INVALID,
                              _lib.lib().om_last_error().decode())
    return nb


def render_fwd_bwd_l2(scene: Scene, o, d, target, out: Dict[str, torch.Tensor], grads: Dict[str, torch.Tensor],
                      n_max: int, delta: float = DELTA, t_term: float = 0.0, c_bg=(0.0, 0.0, 0.0),
                      mlp_bf16: int = -1, workspace: Optional[torch.Tensor] = None,
                      loss: Optional[torch.Tensor] = None, occ_eps: float = 0.0) -> Optional[torch.Tensor]:
    """One fused L2 training step (om_render_fwd_bwd_l2): forward into `out`
    (keys as render()), dL/dC, the loss into `loss` (a device float32 [1]
    tensor, or None to skip), and the backward ADDED into float32 `grads`.
    `workspace` is a device uint8 tensor of fwd_bwd_l2_workspace_size bytes
    (allocated here if None)."""
    n = _rays(scene, o, d)
    _need(target, "target", torch.float32, (n, 3))
    for key in ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp"):
        _need(grads[key], f"grads[{key}]", torch.float32, scene.tensors[key].shape)
    nbytes = fwd_bwd_l2_workspace_size(n, n_max, delta)
    if workspace is None:
        workspace = torch.empty((max(nbytes, 1),), dtype=torch.uint8, device=o.device)
    _need_workspace(workspace, nbytes, o.device)
    if loss is not None:
        _need(loss, "loss", torch.float32, (1,))
    fo = _lib.OmFwdOut(out["C"].data_ptr(), out["T"].data_ptr(), out["F"].data_ptr(), out["n_placed"].data_ptr(),
                       out["n_eval"].data_ptr(), 0)
    g = _grads(scene, grads)
    p = _params(n_max, delta, t_term, c_bg, mlp_bf16, occ_eps)
    _lib.check("om_render_fwd_bwd_l2", _lib.lib().om_render_fwd_bwd_l2(
        scene.handle, o.data_ptr(), d.data_ptr(), n, ctypes.byref(p), target.data_ptr(), ctypes.byref(fo),
        workspace.data_ptr(), workspace.numel(), _lib.ptr(loss), ctypes.byref(g), _lib.stream_of(o)))
    return loss


def _need_workspace(ws: torch.Tensor, nbytes: int, device) -> None:
    """A caller workspace: contiguous device uint8 of at least nbytes (the
    library checks its 256-byte alignment)."""
    if ws.dtype != torch.uint8 or not ws.is_contiguous() or ws.device != device:
        raise ValueError(f"workspace must be a contiguous uint8 tensor on {device}")
    if ws.numel() < nbytes:
        raise ValueError(f"workspace holds {ws.numel()} bytes, {nbytes} needed")


def _grads(scene: Scene, grads: Dict[str, torch.Tensor]) -> _lib.OmGrads:
    for key in ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp"):
        _need(grads[key], f"grads[{key}]", torch.float32, scene.tensors[key].shape)
    occ = grads.get("occ")
    if occ is not None:
        _need(occ, "grads[occ]", torch.float32, scene.tensors["occ"].shape)
    return _lib.OmGrads(grads["grid"].data_ptr(), grads["plane_xy"].data_ptr(), grads["plane_xz"].data_ptr(),
                        grads["plane_yz"].data_ptr(), grads["mlp"].data_ptr(), _lib.ptr(occ))


def occ_interval_loss(occ, weight: float = 1.0, grad: Optional[torch.Tensor] = None,
                      with_loss: bool = True) -> Optional[torch.Tensor]:
    """Interval-span regulariser of Eq. 5: weight * sum (z_max - z_min)^2 as a
    device float32 [1] tensor (if with_loss), and its gradient ADDED into
    `grad` (float32, shape of occ) when given."""
    _need(occ, "occ", torch.float32)
    if occ.shape[-1] != 2:
        raise ValueError("occ must end in (z_min, z_max)")
    if grad is not None:
        _need(grad, "grad", torch.float32, occ.shape)
    loss = torch.empty((1,), dtype=torch.float32, device=occ.device) if with_loss else None
    _lib.check("om_occ_interval_loss", _lib.lib().om_occ_interval_loss(
        occ.data_ptr(), occ.numel() // 2, float(weight), _lib.ptr(loss), _lib.ptr(grad), _lib.stream_of(occ)))
    return loss


def smooth_loss(scene: Scene, F, d, perturb, weight: float = 1.0, dL_dF: Optional[torch.Tensor] = None,
                grad_mlp: Optional[torch.Tensor] = None, with_loss: bool = True) -> Optional[torch.Tensor]:
    """View-smoothness regulariser of Sec. 4.2 (Eq. 9-10) on the scene's MLP
    (om_smooth_loss): weight * sum_r sum_p cos(d_r, s_rp) ||G(F_r, s_rp) -
    G(F_r, d_r)||^2 with s_rp = d_r + perturb[r, p].  F float32 [n, 7], d
    [n, 3], perturb [n, P, 3] (the caller's Gaussian draws).  Returns the
    float32 loss as a device [1] tensor (if with_loss); dL/dF and dL/dmlp
    are ADDED into dL_dF / grad_mlp when given."""
    n = F.shape[0]
    _need(F, "F", torch.float32, (n, 7))
    _need(d, "d", torch.float32, (n, 3))
    _need(perturb, "perturb", torch.float32)
    if perturb.dim() != 3 or perturb.shape[0] != n or perturb.shape[2] != 3:
        raise ValueError(f"perturb must be [n, P, 3] with n = {n}, got {tuple(perturb.shape)}")
    if dL_dF is not None:
        _need(dL_dF, "dL_dF", torch.float32, (n, 7))
    if grad_mlp is not None:
        _need(grad_mlp, "grad_mlp", torch.float32, scene.tensors["mlp"].shape)
    loss = torch.empty((1,), dtype=torch.float32, device=F.device) if with_loss else None
    _lib.check("om_smooth_loss", _lib.lib().om_smooth_loss(
        scene.handle, F.data_ptr(), d.data_ptr(), n, perturb.data_ptr(), perturb.shape[1], float(weight),
        _lib.ptr(loss), _lib.ptr(dL_dF), _lib.ptr(grad_mlp), _lib.stream_of(F)))
    return loss


class SmoothFn(torch.autograd.Function):
    """L_smooth = smooth_loss(scene, F, d, perturb, weight) as a float32
    scalar, differentiable in F and in the float32 MLP master passed last.
    ``SmoothFn.apply(scene, F, d, perturb, weight, mlp)``.  The loss and both
    gradients come out of one kernel call in the forward; the backward scales
    them by the incoming gradient."""

    @staticmethod
    def forward(ctx, scene, F, d, perturb, weight, mlp):
        F = F.detach().contiguous()
        gF = torch.zeros_like(F)
        gW = torch.zeros(mlp.shape, dtype=torch.float32, device=mlp.device)
        loss = smooth_loss(scene, F, d, perturb, weight, dL_dF=gF, grad_mlp=gW)
        ctx.save_for_backward(gF, gW)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g):
        gF, gW = ctx.saved_tensors
        s = g.to(torch.float32)
        return None, gF * s, None, None, None, gW * s


class SparseGrid:
    """Sparse voxel-block layout of a grid (Sec. 4.4): blocks of 2^shift
    cells per edge over a logical (Lx, Ly, Lz) grid; `blocks` is the int32
    block index, the atlas (the Scene's grid tensor) holds n_blocks + 1
    blocks of (B + 1)^3 vertices, block 0 all zero."""

    def __init__(self, blocks: torch.Tensor, shift: int, n_blocks: int, dims):
        self.blocks, self.shift, self.n_blocks, self.dims = blocks, int(shift), int(n_blocks), tuple(dims)

    def index_shape(self):
        b = 1 << self.shift
        lx, ly, lz = self.dims
        return ((lz - 2) // b + 1, (ly - 2) // b + 1, (lx - 2) // b + 1)


def sparse_grid(scene: "Scene", shift: int = 3):
    """Bake the dense grid of `scene` into sparse voxel blocks of 2^shift
    cells per edge (om_sparse_grid_index, om_sparse_grid_fill).  Returns
    (atlas tensor of the scene's dtype, SparseGrid) for
    Scene(atlas, ..., sparse=SparseGrid) (with quant= for 8-bit scenes)."""
    if scene.sparse is not None:
        raise ValueError("the scene's grid is already sparse")
    lz, ly, lx, _ = scene.tensors["grid"].shape
    sg = SparseGrid(None, shift, 0, (lx, ly, lz))
    blocks = torch.empty(sg.index_shape(), dtype=torch.int32, device=scene.device)
    L = _lib.lib()
    n = L.om_sparse_grid_index(scene.handle, shift, blocks.data_ptr(), blocks.numel(),
                               _lib.stream_of(scene.tensors["grid"]))
    if n < 0:
        raise _lib.OmerfError("om_sparse_grid_index", _lib.OM_ERR_INVALID, L.om_last_error().decode())
    e = (1 << shift) + 1
    atlas = torch.empty((n + 1, e, e, e, 8), dtype=scene.dtype, device=scene.device)
    _lib.check("om_sparse_grid_fill", L.om_sparse_grid_fill(scene.handle, shift, blocks.data_ptr(), n,
                                                            atlas.data_ptr(), _lib.stream_of(atlas)))
    sg.blocks, sg.n_blocks = blocks, n
    return atlas, sg


def feature_range(x: torch.Tensor) -> torch.Tensor:
    """Per-channel (min, max) of float32 features [..., 8] (om_feature_range),
    as a device float32 [8, 2] tensor."""
    _need(x, "x", torch.float32)
    if x.shape[-1] != 8:
        raise ValueError("features must end in 8 channels")
    out = torch.empty((8, 2), dtype=torch.float32, device=x.device)
    _lib.check("om_feature_range", _lib.lib().om_feature_range(x.data_ptr(), x.numel() // 8, out.data_ptr(),
                                                               _lib.stream_of(x)))
    return out


def quant_params(minmax) -> tuple:
    """(lo, step) float32 [8] lists from a channel range [8, 2]
    (om_quant_params: lo = min, step = (max - min) / 255 in binary32)."""
    mm = (ctypes.c_float * 16)(*[float(v) for v in torch.as_tensor(minmax).reshape(-1).tolist()])
    lo, step = (ctypes.c_float * 8)(), (ctypes.c_float * 8)()
    _lib.check("om_quant_params", _lib.lib().om_quant_params(mm, lo, step))
    return list(lo), list(step)


def quantize_u8(x: torch.Tensor, lo, step, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """8-bit codes of float32 features [..., 8] (om_quantize_u8)."""
    _need(x, "x", torch.float32)
    if x.shape[-1] != 8:
        raise ValueError("features must end in 8 channels")
    if out is None:
        out = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    _need(out, "out", torch.uint8, x.shape)
    lo_c, st_c = (ctypes.c_float * 8)(*[float(v) for v in lo]), (ctypes.c_float * 8)(*[float(v) for v in step])
    _lib.check("om_quantize_u8", _lib.lib().om_quantize_u8(x.data_ptr(), x.numel() // 8, lo_c, st_c, out.data_ptr(),
                                                           _lib.stream_of(x)))
    return out


def quantize_features(tensors: Dict[str, torch.Tensor]):
    """Bake float32 grid and planes to 8-bit storage (Sec. 4.4): per source,
    its channel ranges, (lo, step) and codes.  Returns ({source: uint8
    tensor}, (lo, step) as float32 [4, 8] lists for Scene(..., quant=...))."""
    codes, los, steps = {}, [], []
    for key in ("grid", "plane_xy", "plane_xz", "plane_yz"):
        lo, step = quant_params(feature_range(tensors[key]).cpu())
        codes[key] = quantize_u8(tensors[key], lo, step)
        los.append(lo)
        steps.append(step)
    return codes, (los, steps)


def l2_loss_fp64(C, target) -> torch.Tensor:
    """float64 mean over rays x 3 of (C - target)^2, as a 1-element device tensor."""
    n = C.shape[0]
    _need(C, "C", torch.float32, (n, 3))
    _need(target, "target", torch.float32, (n, 3))
    out = torch.empty((1,), dtype=torch.float64, device=C.device)
    _lib.check("om_l2_loss_fp64", _lib.lib().om_l2_loss_fp64(C.data_ptr(), target.data_ptr(), n, out.data_ptr(),
                                                               _lib.stream_of(C)))
    return out


def l2_loss_grad(C, target, dL_dC: Optional[torch.Tensor] = None, with_loss: bool = True):
    """dL/dC of the mean L2 loss (and the loss, a float32 sum in a fixed
    order, if with_loss)."""
    n = C.shape[0]
    _need(C, "C", torch.float32, (n, 3))
    _need(target, "target", torch.float32, (n, 3))
    if dL_dC is None:
        dL_dC = torch.empty_like(C)
    loss = torch.empty((1,), dtype=torch.float32, device=C.device) if with_loss else None
    _lib.check("om_l2_loss_grad", _lib.lib().om_l2_loss_grad(C.data_ptr(), target.data_ptr(), n, dL_dC.data_ptr(),
                                                               _lib.ptr(loss), _lib.stream_of(C)))
    return dL_dC, loss


class RenderFn(torch.autograd.Function):
    """C = render(scene) with gradients into float32 master tensors.

    ``RenderFn.apply(scene, o, d, opts, grid, plane_xy, plane_xz, plane_yz, mlp[, occ])``:
    the render reads the tensors the Scene points at (the float32 masters
    themselves, or bfloat16 shadows of them); the gradients are float32 and
    are returned for the master tensors passed as the last inputs, including
    the occupancy plane when it is passed and opts["occ_eps"] > 0.  The
    composited features F (third output) are differentiable too: a loss on
    them (SmoothFn) flows back into the same master gradients.
    opts = dict(n_max=..., delta=..., t_term=..., c_bg=..., mlp_bf16=..., occ_eps=...)."""

    @staticmethod
    def forward(ctx, scene, o, d, opts, grid, plane_xy, plane_xz, plane_yz, mlp, occ=None):
        out = render(scene, o, d, batch_wv=True, **opts)
        ctx.scene, ctx.opts = scene, opts
        ctx.masters = (grid, plane_xy, plane_xz, plane_yz, mlp)
        ctx.occ = occ
        ctx.save_for_backward(o, d, out["C"], out["T"], out["F"], out["n_placed"], out["n_eval"], out["batch_wv"])
        ctx.mark_non_differentiable(out["T"], out["n_placed"], out["n_eval"])
        return out["C"], out["T"], out["F"], out["n_placed"], out["n_eval"]

    @staticmethod
    def backward(ctx, gC, _gT, gF, *_unused):
        o, d, C, T, F, npl, nev, bwv = ctx.saved_tensors
        saved = dict(C=C, T=T, F=F, n_placed=npl, n_eval=nev, batch_wv=bwv)
        grads = {k: torch.zeros(m.shape, dtype=torch.float32, device=m.device)
                 for k, m in zip(("grid", "plane_xy", "plane_xz", "plane_yz", "mlp"), ctx.masters)}
        if ctx.occ is not None and ctx.opts.get("occ_eps", 0.0) > 0:
            grads["occ"] = torch.zeros(ctx.occ.shape, dtype=torch.float32, device=ctx.occ.device)
        opts = {k: v for k, v in ctx.opts.items() if k != "mlp_bf16"}
        if gC is None:
            gC = torch.zeros_like(C)
        dF = gF.contiguous().float() if gF is not None else None
        render_backward(ctx.scene, o, d, saved, gC.contiguous().float(), grads, dL_dF=dF, **opts)
        return (None, None, None, None, grads["grid"], grads["plane_xy"], grads["plane_xz"], grads["plane_yz"],
                grads["mlp"], grads.get("occ"))
