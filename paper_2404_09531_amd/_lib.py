"""ctypes binding of libomerf.so (the C ABI in include/omerf.h).

Argument marshalling only: every step of the render runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  If the
shared library is missing this module raises on first use; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_void_p

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libomerf.so")

OM_OK, OM_ERR_INVALID, OM_ERR_UNSUPPORTED, OM_ERR_HIP = 0, -1, -2, -3
OM_F32, OM_BF16, OM_U8 = 0, 1, 2
OM_MAX_SAMPLES = 1024
EXPORTS = ("om_scene_create", "om_scene_update", "om_scene_destroy", "om_occupancy_mips_size",
           "om_build_occupancy_mips", "om_place_samples", "om_march",
           "om_deferred_mlp", "om_render",
           "om_render_backward", "om_render_backward_ex", "om_render_backward_workspace_size", "om_smooth_loss", "om_render_fwd_bwd_l2", "om_render_fwd_bwd_l2_workspace_size",
           "om_render_fwd_bwd_l2_noalloc", "om_render_fwd_bwd_l2_noalloc_max_bytes",
           "om_occ_interval_loss", "om_feature_range", "om_quant_params", "om_quantize_u8",
           "om_sparse_grid_index", "om_sparse_grid_fill",
           "om_cast_bf16", "om_order_rays", "om_order_rays_workspace_size", "om_gather_rows", "om_scatter_rows",
           "om_mark_rows", "om_l2_loss_fp64", "om_l2_loss_grad", "om_last_error", "om_status_str",
           "om_version")


class OmSceneDesc(ctypes.Structure):
    _fields_ = [("box_lo", c_float * 3), ("box_hi", c_float * 3), ("grid_dims", c_int32 * 3),
                ("plane_dims", c_int32 * 3), ("occ_dims", c_int32 * 2), ("dtype", c_int32),
                ("grid", c_void_p), ("plane_xy", c_void_p), ("plane_xz", c_void_p), ("plane_yz", c_void_p),
                ("occ", c_void_p), ("mlp", c_void_p), ("dir_freqs", c_int32),
                ("quant_lo", (c_float * 8) * 4), ("quant_step", (c_float * 8) * 4),
                ("grid_blocks", c_void_p), ("block_shift", c_int32), ("n_blocks", c_int32)]


class OmParams(ctypes.Structure):
    _fields_ = [("delta", c_float), ("n_max", c_int32), ("t_term", c_float), ("c_bg", c_float * 3),
                ("mlp_bf16", c_int32), ("occ_eps", c_float)]


class OmFwdOut(ctypes.Structure):
    _fields_ = [("C", c_void_p), ("T", c_void_p), ("F", c_void_p), ("n_placed", c_void_p), ("n_eval", c_void_p),
                ("batch_wv", c_void_p)]


class OmGrads(ctypes.Structure):
    _fields_ = [("grid", c_void_p), ("plane_xy", c_void_p), ("plane_xz", c_void_p), ("plane_yz", c_void_p),
                ("mlp", c_void_p), ("occ", c_void_p)]


_lib = None


class OmerfError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libomerf.so (after torch, so it binds to torch's HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2404_09531_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.om_scene_create.argtypes = [POINTER(OmSceneDesc), POINTER(c_void_p)]
        L.om_scene_update.argtypes = [c_void_p, POINTER(OmSceneDesc)]
        L.om_scene_destroy.argtypes = [c_void_p]
        L.om_place_samples.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams), c_void_p, c_void_p,
                                       c_void_p]
        L.om_render.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams), POINTER(OmFwdOut), c_void_p]
        L.om_march.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams), POINTER(OmFwdOut), c_void_p]
        L.om_deferred_mlp.argtypes = [c_void_p, c_void_p, c_int64, POINTER(OmParams), POINTER(OmFwdOut), c_void_p]
        L.om_render_backward.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams),
                                         POINTER(OmFwdOut), c_void_p, c_void_p, c_int64, POINTER(OmGrads), c_void_p]
        L.om_render_backward_ex.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams),
                                            POINTER(OmFwdOut), c_void_p, c_void_p, c_void_p, c_int64,
                                            POINTER(OmGrads), c_void_p]
        L.om_render_backward_workspace_size.argtypes = [c_int64]
        L.om_render_backward_workspace_size.restype = c_int64
        L.om_smooth_loss.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_float, c_void_p,
                                     c_void_p, c_void_p, c_void_p]
        L.om_feature_range.argtypes = [c_void_p, c_int64, c_void_p, c_void_p]
        L.om_quant_params.argtypes = [POINTER(c_float), POINTER(c_float), POINTER(c_float)]
        L.om_quantize_u8.argtypes = [c_void_p, c_int64, POINTER(c_float), POINTER(c_float), c_void_p, c_void_p]
        L.om_sparse_grid_index.argtypes = [c_void_p, c_int, c_void_p, c_int64, c_void_p]
        L.om_sparse_grid_fill.argtypes = [c_void_p, c_int, c_void_p, c_int64, c_void_p, c_void_p]
        L.om_cast_bf16.argtypes = [c_void_p, c_int64, c_void_p, c_void_p]
        L.om_order_rays.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_int64, c_void_p]
        L.om_order_rays_workspace_size.argtypes = [c_int64]
        L.om_order_rays_workspace_size.restype = c_int64
        L.om_gather_rows.argtypes = [c_void_p, c_int64, c_int, c_void_p, c_int64, c_void_p, c_void_p]
        L.om_scatter_rows.argtypes = [c_void_p, c_int, c_void_p, c_int64, c_void_p, c_int64, c_void_p]
        L.om_mark_rows.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams), c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p]
        L.om_l2_loss_fp64.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.om_l2_loss_grad.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
        L.om_render_fwd_bwd_l2.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams), c_void_p,
                                           POINTER(OmFwdOut), c_void_p, c_int64, c_void_p, POINTER(OmGrads),
                                           c_void_p]
        L.om_render_fwd_bwd_l2_workspace_size.argtypes = [c_int64, POINTER(OmParams)]
        L.om_render_fwd_bwd_l2_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(OmParams),
                                                   c_void_p, POINTER(OmFwdOut), c_void_p, POINTER(OmGrads), c_void_p]
        L.om_render_fwd_bwd_l2_noalloc_max_bytes.argtypes = []
        L.om_occupancy_mips_size.argtypes = [c_void_p, c_int]
        L.om_occ_interval_loss.argtypes = [c_void_p, c_int64, c_float, c_void_p, c_void_p, c_void_p]
        L.om_build_occupancy_mips.argtypes = [c_void_p, c_void_p, c_int64, c_int, c_void_p]
        L.om_last_error.restype = c_char_p
        L.om_status_str.restype = c_char_p
        L.om_status_str.argtypes = [c_int]
        for name in EXPORTS:
            if name not in ("om_last_error", "om_status_str", "om_render_fwd_bwd_l2_workspace_size",
                            "om_render_fwd_bwd_l2_noalloc_max_bytes", "om_occupancy_mips_size"):
                getattr(L, name).restype = c_int
        L.om_render_fwd_bwd_l2_workspace_size.restype = c_int64
        L.om_render_fwd_bwd_l2_noalloc_max_bytes.restype = c_int64
        L.om_occupancy_mips_size.restype = c_int64
        L.om_sparse_grid_index.restype = c_int64
        _lib = L
    return _lib


def check(fn: str, code: int) -> None:
    if code != OM_OK:
        msg = lib().om_last_error().decode()
        raise OmerfError(fn, code, msg)


def ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


def stream_of(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream
