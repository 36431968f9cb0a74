"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/omerf.h, and rejects bad arguments with status codes
before any device work (no pointer is dereferenced on these paths)."""
import ctypes
import math
import os
import re

import pytest
import torch  # noqa: F401  (load torch's HIP runtime first, as the package does)

from paper_2404_09531_amd import _lib
from paper_2404_09531_amd.build import ensure_built

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x100000  # aligned, non-NULL, never dereferenced on these paths


@pytest.fixture(scope="module")
def L():
    ensure_built()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "omerf.h")).read()
    names = set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(om_\w+)\s*\(", hdr, re.M))
    assert names == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n
    assert L.om_version() == 110
    assert L.om_status_str(-2) == b"unsupported shape or dtype"


def _desc(**kw):
    d = _lib.OmSceneDesc()
    d.box_lo[:] = [-1.0, -1.0, 0.0]
    d.box_hi[:] = [1.0, 1.0, 0.25]
    d.grid_dims[:] = [64, 64, 16]
    d.plane_dims[:] = [256, 256, 64]
    d.occ_dims[:] = [32, 32]
    d.dtype = _lib.OM_F32
    for f in ("grid", "plane_xy", "plane_xz", "plane_yz", "occ", "mlp"):
        setattr(d, f, FAKE)
    for k, v in kw.items():
        if isinstance(getattr(d, k), ctypes.Array):
            getattr(d, k)[:] = v
        else:
            setattr(d, k, v)
    return d


def _create(L, d):
    h = ctypes.c_void_p()
    rc = L.om_scene_create(ctypes.byref(d), ctypes.byref(h))
    return rc, h


def test_scene_validation(L):
    rc, h = _create(L, _desc())
    assert rc == 0 and h.value
    assert L.om_scene_destroy(h) == 0
    assert L.om_scene_destroy(None) == 0
    bad = [
        (dict(box_hi=[1.0, 1.0, 0.3]), _lib.OM_ERR_UNSUPPORTED),      # extent 0.3 not a power of two
        (dict(box_hi=[-1.0, 1.0, 0.25]), _lib.OM_ERR_INVALID),        # empty box
        (dict(grid_dims=[1, 64, 16]), _lib.OM_ERR_INVALID),
        (dict(occ_dims=[24, 32]), _lib.OM_ERR_UNSUPPORTED),           # 12 cells / unit: not a power of two
        (dict(occ_dims=[0, 32]), _lib.OM_ERR_INVALID),
        (dict(dtype=7), _lib.OM_ERR_UNSUPPORTED),
        (dict(grid=None), _lib.OM_ERR_INVALID),
        (dict(occ=FAKE + 4), _lib.OM_ERR_INVALID),                    # misaligned
        (dict(grid_dims=[2048, 2048, 1024]), _lib.OM_ERR_UNSUPPORTED),  # 2^32 vertices
        (dict(dir_freqs=2), _lib.OM_ERR_UNSUPPORTED),                 # only 0 or 4 frequencies
        (dict(dir_freqs=-4), _lib.OM_ERR_UNSUPPORTED),
    ]
    for kw, code in bad:
        rc, h = _create(L, _desc(**kw))
        assert rc == code, (kw, rc)
        assert not h.value
        assert len(L.om_last_error()) > 0
    assert L.om_scene_create(None, ctypes.byref(ctypes.c_void_p())) == _lib.OM_ERR_INVALID


def _params(**kw):
    p = _lib.OmParams()
    p.delta = 0.25 / 512
    p.n_max = 64
    p.t_term = 0.0
    p.c_bg[:] = [0, 0, 0]
    p.mlp_bf16 = -1
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_render_argument_errors(L):
    rc, h = _create(L, _desc())
    assert rc == 0
    out = _lib.OmFwdOut(FAKE, FAKE, FAKE, FAKE, FAKE)
    cases = [
        (_params(delta=0.001), 4, _lib.OM_ERR_INVALID),
        (_params(delta=-0.25), 4, _lib.OM_ERR_INVALID),
        (_params(n_max=0), 4, _lib.OM_ERR_UNSUPPORTED),
        (_params(n_max=_lib.OM_MAX_SAMPLES + 1), 4, _lib.OM_ERR_UNSUPPORTED),
        (_params(t_term=float("nan")), 4, _lib.OM_ERR_INVALID),
        (_params(t_term=-1.0), 4, _lib.OM_ERR_INVALID),
        (_params(mlp_bf16=3), 4, _lib.OM_ERR_INVALID),
        (_params(occ_eps=-0.01), 4, _lib.OM_ERR_INVALID),
        (_params(occ_eps=float("inf")), 4, _lib.OM_ERR_INVALID),
        (_params(occ_eps=1e-45), 4, _lib.OM_ERR_INVALID),  # 1/eps overflows
        (_params(), -1, _lib.OM_ERR_INVALID),
        (_params(), 1 << 31, _lib.OM_ERR_UNSUPPORTED),
    ]
    for p, n, code in cases:
        assert L.om_render(h, FAKE, FAKE, n, ctypes.byref(p), ctypes.byref(out), None) == code
    # n = 0 is a no-op that touches nothing
    assert L.om_render(h, None, None, 0, ctypes.byref(_params()), ctypes.byref(out), None) == 0
    missing = _lib.OmFwdOut(FAKE, 0, FAKE, FAKE, FAKE)
    assert L.om_render(h, FAKE, FAKE, 4, ctypes.byref(_params()), ctypes.byref(missing), None) == _lib.OM_ERR_INVALID
    assert L.om_render(None, FAKE, FAKE, 4, ctypes.byref(_params()), ctypes.byref(out), None) == _lib.OM_ERR_INVALID
    g = _lib.OmGrads(FAKE, FAKE, FAKE, 0, FAKE, 0)
    assert L.om_render_backward(h, FAKE, FAKE, 4, ctypes.byref(_params()), ctypes.byref(out), FAKE, FAKE, 1 << 20,
                                ctypes.byref(g), None) == _lib.OM_ERR_INVALID
    # the optional per-batch sums must be float-aligned when given
    bad_bw = _lib.OmFwdOut(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE + 2)
    assert L.om_render(h, FAKE, FAKE, 4, ctypes.byref(_params()), ctypes.byref(bad_bw), None) == _lib.OM_ERR_INVALID
    assert L.om_march(h, FAKE, FAKE, 4, ctypes.byref(_params()), ctypes.byref(bad_bw), None) == _lib.OM_ERR_INVALID
    g_ok = _lib.OmGrads(FAKE, FAKE, FAKE, FAKE, FAKE, 0)
    assert L.om_render_backward(h, FAKE, FAKE, 4, ctypes.byref(_params()), ctypes.byref(bad_bw), FAKE, FAKE,
                                1 << 20, ctypes.byref(g_ok), None) == _lib.OM_ERR_INVALID
    assert L.om_place_samples(h, FAKE, FAKE, 4, ctypes.byref(_params()), 0, FAKE, None) == _lib.OM_ERR_INVALID
    assert L.om_l2_loss_fp64(FAKE, FAKE, 0, FAKE, None) == _lib.OM_ERR_INVALID
    assert L.om_l2_loss_grad(FAKE, FAKE, 3, FAKE, None, None) == _lib.OM_ERR_INVALID  # aliasing
    L.om_scene_destroy(h)


def test_fused_training_step_validation(L):
    """Workspace query and the fused step's argument checks (no device work)."""
    p = _params()
    n = 1000
    ws = L.om_render_fwd_bwd_l2_workspace_size(n, ctypes.byref(p))
    # dL/dC, the backward's workspace (per-ray hand-over of 8 floats, ray
    # order, 1 KiB of scheduling words), then 4 batch slots x 7 floats per ray
    bwd = (n * 32 + 255) // 256 * 256 + (n * 4 + 255) // 256 * 256 + 1024
    assert ws == (n * 12 + 255) // 256 * 256 + bwd + n * 4 * 7 * 4
    assert L.om_render_fwd_bwd_l2_workspace_size(-1, ctypes.byref(p)) == -1
    assert L.om_render_fwd_bwd_l2_workspace_size(n, ctypes.byref(_params(n_max=0))) == -1
    rc, h = _create(L, _desc())
    out = _lib.OmFwdOut(FAKE, FAKE, FAKE, FAKE, FAKE, 0)
    g = _lib.OmGrads(FAKE, FAKE, FAKE, FAKE, FAKE, 0)
    step = lambda *a: L.om_render_fwd_bwd_l2(h, FAKE, FAKE, n, ctypes.byref(p), *a)  # noqa: E731
    assert step(FAKE, ctypes.byref(out), FAKE, ws - 1, None, ctypes.byref(g), None) == _lib.OM_ERR_INVALID
    assert step(FAKE, ctypes.byref(out), FAKE + 16, ws, None, ctypes.byref(g), None) == _lib.OM_ERR_INVALID
    assert step(None, ctypes.byref(out), FAKE, ws, None, ctypes.byref(g), None) == _lib.OM_ERR_INVALID
    bad_g = _lib.OmGrads(FAKE, 0, FAKE, FAKE, FAKE, 0)
    assert step(FAKE, ctypes.byref(out), FAKE, ws, None, ctypes.byref(bad_g), None) == _lib.OM_ERR_INVALID
    assert "workspace" in L.om_last_error().decode() or "gradient" in L.om_last_error().decode()
    L.om_scene_destroy(h)


def test_backward_workspace_validation(L):
    """Workspace query and argument checks of the two backward entry points
    (no device work): 32 bytes per ray (the hand-over) and 4 bytes per ray
    (the ray order), each rounded up to 256, plus 1 KiB of scheduling
    words; a workspace that is too small or misaligned is refused before
    anything is launched."""
    assert L.om_render_backward_workspace_size(0) == 0
    assert L.om_render_backward_workspace_size(1) == 256 + 256 + 1024
    assert L.om_render_backward_workspace_size(1000) == 32000 + 4096 + 1024  # 125 x 256, 16 x 256
    assert L.om_render_backward_workspace_size(1001) == 32256 + 4096 + 1024
    assert L.om_render_backward_workspace_size(-1) == -1
    n = 1000
    ws = L.om_render_backward_workspace_size(n)
    rc, h = _create(L, _desc())
    out = _lib.OmFwdOut(FAKE, FAKE, FAKE, FAKE, FAKE, 0)
    g = _lib.OmGrads(FAKE, FAKE, FAKE, FAKE, FAKE, 0)
    p = _params()
    ex = lambda w, nb, gg=g: L.om_render_backward_ex(h, FAKE, FAKE, n, ctypes.byref(p), ctypes.byref(out),  # noqa: E731
                                                     FAKE, None, w, nb, ctypes.byref(gg), None)
    plain = lambda w, nb: L.om_render_backward(h, FAKE, FAKE, n, ctypes.byref(p), ctypes.byref(out),  # noqa: E731
                                               FAKE, w, nb, ctypes.byref(g), None)
    for call in (ex, plain):
        assert call(FAKE, ws - 1) == _lib.OM_ERR_INVALID
        assert "workspace" in L.om_last_error().decode()
        assert call(FAKE + 16, ws) == _lib.OM_ERR_INVALID
        assert call(None, ws) == _lib.OM_ERR_INVALID
    assert ex(FAKE, ws, _lib.OmGrads(FAKE, 0, FAKE, FAKE, FAKE, 0)) == _lib.OM_ERR_INVALID
    # n = 0 is a no-op that needs no workspace
    assert L.om_render_backward_ex(h, None, None, 0, ctypes.byref(p), ctypes.byref(out), None, None, None, 0,
                                   ctypes.byref(g), None) == 0
    L.om_scene_destroy(h)


def test_order_rays_validation(L):
    """Workspace query and argument checks of the ray order and the row
    gathers (no device work): a 256 KiB key histogram plus 2 bytes per ray
    rounded up to 256; n beyond 2^31 - 1, a short or misaligned workspace,
    outputs overlapping the rays, and cols outside [1, 64] are refused
    before anything is launched; n = 0 is a no-op."""
    assert L.om_order_rays_workspace_size(0) == 0
    assert L.om_order_rays_workspace_size(1) == 262144 + 256
    assert L.om_order_rays_workspace_size(128) == 262144 + 256
    assert L.om_order_rays_workspace_size(129) == 262144 + 512
    assert L.om_order_rays_workspace_size(-1) == -1
    assert L.om_order_rays_workspace_size(1 << 31) == -1
    rc, h = _create(L, _desc())
    n = 1000
    ws = L.om_order_rays_workspace_size(n)
    o, d, order, os_, ds_ = (FAKE + k * (1 << 20) for k in range(5))
    call = lambda w, nb, a=os_, b=ds_: L.om_order_rays(h, o, d, n, order, a, b, w, nb, None)  # noqa: E731
    assert call(FAKE + (8 << 20), ws - 1) == _lib.OM_ERR_INVALID
    assert "workspace" in L.om_last_error().decode()
    assert call(FAKE + (8 << 20) + 16, ws) == _lib.OM_ERR_INVALID
    assert call(None, ws) == _lib.OM_ERR_INVALID
    assert call(FAKE + (8 << 20), ws, a=o + 4) == _lib.OM_ERR_INVALID
    assert "overlap" in L.om_last_error().decode()
    assert call(FAKE + (8 << 20), ws, b=d) == _lib.OM_ERR_INVALID
    assert L.om_order_rays(None, o, d, n, order, os_, ds_, FAKE, ws, None) == _lib.OM_ERR_INVALID
    assert L.om_order_rays(h, o, d, 1 << 31, order, os_, ds_, FAKE, 1 << 40, None) == _lib.OM_ERR_INVALID
    assert L.om_order_rays(h, None, None, 0, None, None, None, None, 0, None) == 0
    for cols in (0, 65):
        assert L.om_gather_rows(o, n, cols, order, n, os_, None) == _lib.OM_ERR_INVALID
        assert L.om_scatter_rows(o, cols, order, n, os_, n, None) == _lib.OM_ERR_INVALID
    assert L.om_gather_rows(o, n, 3, order, n, o + 12, None) == _lib.OM_ERR_INVALID
    assert "overlap" in L.om_last_error().decode()
    assert L.om_scatter_rows(o, 3, None, n, os_, n, None) == _lib.OM_ERR_INVALID
    assert L.om_gather_rows(None, 0, 3, None, 0, None, None) == 0
    assert L.om_scatter_rows(None, 3, None, 0, None, 0, None) == 0
    L.om_scene_destroy(h)


def test_occupancy_mips_validation(L):
    rc, h = _create(L, _desc())  # occupancy 32 x 32
    assert L.om_occupancy_mips_size(h, 0) == 0
    assert L.om_occupancy_mips_size(h, 2) == (16 * 16 + 8 * 8) * 8
    assert L.om_occupancy_mips_size(h, 5) == sum((32 >> lv) ** 2 for lv in range(1, 6)) * 8
    assert L.om_occupancy_mips_size(h, 6) == -1      # 32 not divisible by 64
    assert L.om_occupancy_mips_size(h, -1) == -1
    assert L.om_occupancy_mips_size(None, 1) == -1
    assert L.om_build_occupancy_mips(h, FAKE, 16 * 16 * 8 - 8, 1, None) == _lib.OM_ERR_INVALID  # too small
    assert L.om_build_occupancy_mips(h, FAKE + 4, 4096, 1, None) == _lib.OM_ERR_INVALID        # misaligned
    assert L.om_build_occupancy_mips(h, None, 0, 0, None) == 0                              # detach
    L.om_scene_destroy(h)


def test_occ_interval_loss_validation(L):
    assert L.om_occ_interval_loss(FAKE, 0, 1.0, FAKE, FAKE, None) == _lib.OM_ERR_INVALID
    assert L.om_occ_interval_loss(None, 4, 1.0, FAKE, FAKE, None) == _lib.OM_ERR_INVALID
    assert L.om_occ_interval_loss(FAKE, 4, float("nan"), FAKE, FAKE, None) == _lib.OM_ERR_INVALID
    assert L.om_occ_interval_loss(FAKE, 4, 1.0, None, None, None) == 0  # nothing requested: no device work


def test_struct_layouts_match_header():
    """om_params ends with occ_eps; om_grads with occ."""
    hdr = open(os.path.join(ROOT, "include", "omerf.h")).read()
    for name, cls in (("om_scene_desc", _lib.OmSceneDesc), ("om_params", _lib.OmParams),
                      ("om_grads", _lib.OmGrads)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), hdr, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"(\w+)(?:\[\d+\])*;", body)
        assert fields == [f for f, _ in cls._fields_], name


def test_struct_offsets_match_a_c_compiler(tmp_path):
    """Sizes and field offsets of the ABI structs as gcc lays them out."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"om_scene_desc": _lib.OmSceneDesc, "om_params": _lib.OmParams, "om_fwd_out": _lib.OmFwdOut,
               "om_grads": _lib.OmGrads}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "omerf.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_fwd_out_layout_matches_header():
    """om_fwd_out is six pointers in header order, batch_wv last."""
    hdr = open(os.path.join(ROOT, "include", "omerf.h")).read()
    body = re.search(r"typedef struct om_fwd_out \{(.*?)\} om_fwd_out;", hdr, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\*\s*(\w+);", body)
    assert fields == [f for f, _ in _lib.OmFwdOut._fields_]
    assert ctypes.sizeof(_lib.OmFwdOut) == 6 * ctypes.sizeof(ctypes.c_void_p)


def test_scene_update_keeps_handle_on_error(L):
    rc, h = _create(L, _desc())
    assert L.om_scene_update(h, ctypes.byref(_desc(occ_dims=[24, 32]))) == _lib.OM_ERR_UNSUPPORTED
    assert L.om_scene_update(h, ctypes.byref(_desc(grid_dims=[8, 8, 8]))) == 0
    L.om_scene_destroy(h)


def test_dir_freqs_accepted(L):
    rc, h = _create(L, _desc(dir_freqs=4))
    assert rc == 0 and h.value
    L.om_scene_destroy(h)


def test_smooth_loss_validation(L):
    """om_smooth_loss rejects bad arguments before touching device memory."""
    rc, h = _create(L, _desc())
    f = ctypes.c_void_p(FAKE)
    cases = [
        (dict(P=0), _lib.OM_ERR_INVALID),
        (dict(P=65), _lib.OM_ERR_INVALID),
        (dict(weight=math.nan), _lib.OM_ERR_INVALID),
        (dict(F=None), _lib.OM_ERR_INVALID),
        (dict(perturb=None), _lib.OM_ERR_INVALID),
        (dict(n=-1), _lib.OM_ERR_INVALID),
        (dict(scene=None), _lib.OM_ERR_INVALID),
    ]
    for kw, code in cases:
        a = dict(scene=h, F=f, d=f, n=16, perturb=f, P=4, weight=1.0)
        a.update(kw)
        rc = L.om_smooth_loss(a["scene"], a["F"], a["d"], a["n"], a["perturb"], a["P"], a["weight"], f, f, f, None)
        assert rc == code, (kw, rc)
    # nothing requested, or no rays and no loss: a no-op that launches nothing
    assert L.om_smooth_loss(h, f, f, 16, f, 4, 1.0, None, None, None, None) == 0
    assert L.om_smooth_loss(h, None, None, 0, None, 4, 1.0, None, f, f, None) == 0
    L.om_scene_destroy(h)


def test_u8_scene_validation(L):
    rc, h = _create(L, _desc(dtype=_lib.OM_U8))
    assert rc == 0 and h.value
    L.om_scene_destroy(h)
    d = _desc(dtype=_lib.OM_U8)
    d.quant_step[2][3] = -0.5
    rc, h = _create(L, d)
    assert rc == _lib.OM_ERR_INVALID and not h.value
    d = _desc(dtype=_lib.OM_U8)
    d.quant_lo[0][0] = math.inf
    assert _create(L, d)[0] == _lib.OM_ERR_INVALID
    d = _desc(dtype=_lib.OM_F32)
    d.quant_step[0][0] = -1.0  # ignored for float scenes
    rc, h = _create(L, d)
    assert rc == 0
    L.om_scene_destroy(h)


def test_quant_params_host_matches_oracle(L):
    """om_quant_params runs on the host: lo = min, step = fl32((max - min)/255)."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(5)
    mm = np.sort(rng.standard_normal((8, 2)).astype(np.float32), axis=1)
    mm[3] = [0.25, 0.25]  # constant channel
    lo, step = (ctypes.c_float * 8)(), (ctypes.c_float * 8)()
    assert L.om_quant_params((ctypes.c_float * 16)(*mm.reshape(-1).tolist()), lo, step) == 0
    want_lo, want_step = oracle.quant_params(mm)
    assert np.array_equal(np.array(list(lo), np.float32), want_lo)
    assert np.array_equal(np.array(list(step), np.float32), want_step)
    bad = mm.copy()
    bad[1] = [1.0, 0.0]  # max < min
    assert L.om_quant_params((ctypes.c_float * 16)(*bad.reshape(-1).tolist()), lo, step) == _lib.OM_ERR_INVALID
    bad[1] = [0.0, math.nan]
    assert L.om_quant_params((ctypes.c_float * 16)(*bad.reshape(-1).tolist()), lo, step) == _lib.OM_ERR_INVALID


def test_bake_calls_validate_before_device_work(L):
    f = ctypes.c_void_p(FAKE)
    lo = (ctypes.c_float * 8)(*[0.0] * 8)
    step = (ctypes.c_float * 8)(*[0.1] * 8)
    assert L.om_feature_range(f, 0, ctypes.c_void_p(FAKE * 4), None) == _lib.OM_ERR_INVALID
    assert L.om_feature_range(None, 10, ctypes.c_void_p(FAKE * 4), None) == _lib.OM_ERR_INVALID
    assert L.om_feature_range(f, 10, ctypes.c_void_p(FAKE + 64), None) == _lib.OM_ERR_INVALID  # aliases x
    assert L.om_feature_range(ctypes.c_void_p(FAKE + 4), 10, ctypes.c_void_p(FAKE * 4), None) == _lib.OM_ERR_INVALID
    assert L.om_quantize_u8(f, -1, lo, step, ctypes.c_void_p(FAKE * 4), None) == _lib.OM_ERR_INVALID
    neg = (ctypes.c_float * 8)(*([0.1] * 7 + [-0.1]))
    assert L.om_quantize_u8(f, 10, lo, neg, ctypes.c_void_p(FAKE * 4), None) == _lib.OM_ERR_INVALID
    tiny = (ctypes.c_float * 8)(*([0.1] * 7 + [1e-40]))
    assert L.om_quantize_u8(f, 10, lo, tiny, ctypes.c_void_p(FAKE * 4), None) == _lib.OM_ERR_UNSUPPORTED
    assert L.om_quantize_u8(f, 10, lo, step, ctypes.c_void_p(FAKE * 4 + 1), None) == _lib.OM_ERR_INVALID


def test_sparse_grid_validation(L):
    d = _desc(block_shift=6, grid_blocks=FAKE)
    assert _create(L, d)[0] == _lib.OM_ERR_INVALID
    d = _desc(block_shift=3)  # no block index
    assert _create(L, d)[0] == _lib.OM_ERR_INVALID
    d = _desc(block_shift=3, grid_blocks=FAKE, n_blocks=1 << 22)  # (n + 1) 9^3 >= 2^31
    assert _create(L, d)[0] == _lib.OM_ERR_UNSUPPORTED
    rc, h = _create(L, _desc(block_shift=3, grid_blocks=FAKE, n_blocks=100))
    assert rc == 0
    # a sparse scene cannot be sparsified again; bad shifts and lengths fail before device work
    assert L.om_sparse_grid_index(h, 3, ctypes.c_void_p(FAKE), 8 * 8 * 2, None) == -1
    L.om_scene_destroy(h)
    rc, h = _create(L, _desc())  # grid 64 x 64 x 16 -> 8 x 8 x 2 blocks of 8 cells
    assert L.om_sparse_grid_index(h, 0, ctypes.c_void_p(FAKE), 128, None) == -1
    assert L.om_sparse_grid_index(h, 3, ctypes.c_void_p(FAKE), 127, None) == -1
    assert L.om_sparse_grid_index(h, 3, None, 128, None) == -1
    assert L.om_sparse_grid_fill(h, 3, ctypes.c_void_p(FAKE), -1, ctypes.c_void_p(FAKE), None) == \
        _lib.OM_ERR_UNSUPPORTED
    assert L.om_sparse_grid_fill(h, 3, ctypes.c_void_p(FAKE), 10, ctypes.c_void_p(FAKE + 8), None) == \
        _lib.OM_ERR_INVALID
    L.om_scene_destroy(h)


def test_header_compiles_cleanly_in_c_and_cpp(tmp_path):
    """include/omerf.h compiles warning-free as C11 and C++17, and its
    parameter-count macro agrees with the library's MLP sizes."""
    import shutil
    import subprocess
    src = tmp_path / "h.c"
    src.write_text('#include "omerf.h"\n'
                   '#ifdef __cplusplus\n#define SA static_assert\n#else\n#define SA _Static_assert\n#endif\n'
                   'SA(OM_MLP_NPARAMS(0) == 499, "10 inputs");\n'
                   'SA(OM_MLP_NPARAMS(4) == 883, "34 inputs");\n'
                   'SA(OM_BATCH_SLOTS(17) == 2, "slots");\n'
                   'int main(void) { return 0; }\n')
    for cc, extra in (("gcc", ["-std=c11", "-x", "c"]), ("g++", ["-std=c++17", "-x", "c++"])):
        if shutil.which(cc) is None:
            pytest.skip(f"no {cc}")
        r = subprocess.run([cc, *extra, "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                            "-fsyntax-only", str(src)], capture_output=True, text=True)
        assert r.returncode == 0, (cc, r.stderr)
