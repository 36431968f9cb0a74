"""The fused L2 training step without a caller workspace
(om_render_fwd_bwd_l2_noalloc), called through the C ABI, against the
workspace entry point (om_render_fwd_bwd_l2) on the same inputs.

Both run the same kernels; the no-alloc call keeps its workspace in the
library's fixed per-GPU array.  Forward outputs and the loss are
deterministic and must be equal bit for bit.  The gradients are float32
atomic sums whose order varies from run to run: per entry, two orders of a
float32 sum of N terms differ by at most 2 (N - 1) u A (A the sum of the
terms' absolute values, u = 2^-24), with A and N from the oracle's error
scale of the same backward; untouched entries are exactly 0 in both.

Two calls in a row on one GPU, the second with fewer rays than the first
(the array keeps the first call's contents), then a call whose workspace
would exceed the array, which must be refused.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2404_09531_amd as om
import scenegen
from oracle.fp32_bound import gradient_error_scale
from paper_2404_09531_amd import _lib
from tests.gpu_util import log, rays_to, upload_scene

BG = (0.25, 0.5, 0.75)
SOURCES = ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp")
KEYS = ("C", "T", "F", "n_placed", "n_eval")
U32 = 2.0 ** -24


def _outs(n, dev):
    return dict(C=torch.empty((n, 3), device=dev), T=torch.empty((n,), device=dev), F=torch.empty((n, 7), device=dev),
                n_placed=torch.empty((n,), dtype=torch.int32, device=dev),
                n_eval=torch.empty((n,), dtype=torch.int32, device=dev))


def _step(L, scene, og, dg, tg, n_max, noalloc):
    """One fused step through the C ABI; returns (outputs, loss, grads)."""
    n = og.shape[0]
    dev = og.device
    out = _outs(n, dev)
    grads = {k: torch.zeros(scene.tensors[k].shape, dtype=torch.float32, device=dev) for k in SOURCES}
    loss = torch.full((1,), -1.0, dtype=torch.float32, device=dev)
    p = om._params(n_max, om.DELTA, 0.0, BG, -1, 0.0)
    fo = _lib.OmFwdOut(out["C"].data_ptr(), out["T"].data_ptr(), out["F"].data_ptr(), out["n_placed"].data_ptr(),
                       out["n_eval"].data_ptr(), 0)
    g = _lib.OmGrads(*[grads[k].data_ptr() for k in SOURCES], 0)
    st = torch.cuda.current_stream(dev).cuda_stream
    if noalloc:
        rc = L.om_render_fwd_bwd_l2_noalloc(scene.handle, og.data_ptr(), dg.data_ptr(), n, ctypes.byref(p),
                                            tg.data_ptr(), ctypes.byref(fo), loss.data_ptr(), ctypes.byref(g), st)
    else:
        nb = L.om_render_fwd_bwd_l2_workspace_size(n, ctypes.byref(p))
        ws = torch.empty((nb,), dtype=torch.uint8, device=dev)
        rc = L.om_render_fwd_bwd_l2(scene.handle, og.data_ptr(), dg.data_ptr(), n, ctypes.byref(p), tg.data_ptr(),
                                    ctypes.byref(fo), ws.data_ptr(), nb, loss.data_ptr(), ctypes.byref(g), st)
    assert rc == 0, L.om_last_error().decode()
    torch.cuda.synchronize()
    return out, loss.item(), {k: v.double().cpu().numpy() for k, v in grads.items()}


def _grads_agree(ga, gb, sc, o, d, up, n_max, tag):
    """|ga - gb| <= 2 (N - 1) u A per entry (two summation orders of the same
    float32 terms), untouched entries 0 in both."""
    scale = gradient_error_scale(sc, o, d, oracle.RenderParams(n_max=n_max, c_bg=BG), up.astype(np.float64))
    for k in SOURCES:
        if k == "mlp":
            A, N = scale[k][0], scale[k][2]
            a, b = ga[k], gb[k]
            bar = 2.0 * np.maximum(N - 1, 0) * U32 * A
            err = np.abs(a - b)
            assert np.all(err <= bar), (tag, k, float((err - bar).max()))
        else:
            idx, A, N = scale[k][0], scale[k][1], scale[k][3]
            a = ga[k].reshape(-1, 8)
            b = gb[k].reshape(-1, 8)
            outside = np.ones(a.shape[0], bool)
            outside[idx] = False
            assert np.all(a[outside] == 0) and np.all(b[outside] == 0), (tag, k)
            bar = 2.0 * np.maximum(N - 1, 0)[:, None] * U32 * A
            err = np.abs(a[idx] - b[idx])
            assert np.all(err <= bar), (tag, k, float((err - bar).max()))
        log(f"  [{tag}] {k}: max |noalloc - workspace| {float(np.abs(ga[k] - gb[k]).max()):.3e}")


@pytest.mark.gpu
def test_noalloc_step_matches_workspace_step():
    L = _lib.lib()
    sc = scenegen.make_scene(scenegen.TINY)
    scene, t = upload_scene(sc)
    n_max = 64
    cap = L.om_render_fwd_bwd_l2_noalloc_max_bytes()
    assert cap == 64 << 20
    pert = scenegen.perturb_scene(sc, 0.05, seed=2)
    o_all, d_all = scenegen.oblique_rays(4096, seed=1)
    target_all = oracle.oracle_render(pert, o_all, d_all, oracle.RenderParams(n_max=n_max, c_bg=BG),
                                      keep_k=False)["C"].astype(np.float32)
    # first call: all 4096 rays; second call: 1000 other rays (fewer)
    for tag, sl in (("4096 rays", slice(0, 4096)), ("1000 rays after 4096", slice(3000, 4000))):
        o, d, target = o_all[sl], d_all[sl], target_all[sl]
        log(f"test_noalloc_step_matches_workspace_step: {tag}, n_max {n_max}")
        og, dg = rays_to(o, d)
        tg = torch.from_numpy(np.ascontiguousarray(target)).to(og.device)
        out_na, loss_na, g_na = _step(L, scene, og, dg, tg, n_max, noalloc=True)
        out_ws, loss_ws, g_ws = _step(L, scene, og, dg, tg, n_max, noalloc=False)
        for k in KEYS:
            assert torch.equal(out_na[k], out_ws[k]), (tag, k)
        assert loss_na == loss_ws and loss_na > 0, (tag, loss_na, loss_ws)
        # the backward of both took dL/dC = 2 (C - target) / (3 n) in float32
        up = ((2.0 / (3.0 * o.shape[0])) * (out_ws["C"].double().cpu().numpy() - target.astype(np.float64)))
        _grads_agree(g_na, g_ws, sc, o, d, up, n_max, tag)


@pytest.mark.gpu
def test_noalloc_step_refuses_more_than_its_array():
    L = _lib.lib()
    sc = scenegen.make_scene(scenegen.TINY)
    scene, _ = upload_scene(sc)
    p = om._params(64, om.DELTA, 0.0, BG, -1, 0.0)
    cap = L.om_render_fwd_bwd_l2_noalloc_max_bytes()
    n = 1
    while L.om_render_fwd_bwd_l2_workspace_size(n, ctypes.byref(p)) <= cap:
        n *= 2
    log(f"test_noalloc_step_refuses_more_than_its_array: {n} rays at n_max 64")
    dev = torch.device("cuda:0")
    o, d = scenegen.oblique_rays(n, seed=5)
    og, dg = rays_to(o, d)
    out = _outs(n, dev)
    tg = torch.zeros((n, 3), device=dev)
    grads = {k: torch.zeros(scene.tensors[k].shape, dtype=torch.float32, device=dev) for k in SOURCES}
    fo = _lib.OmFwdOut(out["C"].data_ptr(), out["T"].data_ptr(), out["F"].data_ptr(), out["n_placed"].data_ptr(),
                       out["n_eval"].data_ptr(), 0)
    g = _lib.OmGrads(*[grads[k].data_ptr() for k in SOURCES], 0)
    rc = L.om_render_fwd_bwd_l2_noalloc(scene.handle, og.data_ptr(), dg.data_ptr(), n, ctypes.byref(p),
                                        tg.data_ptr(), ctypes.byref(fo), None, ctypes.byref(g),
                                        torch.cuda.current_stream(dev).cuda_stream)
    assert rc == _lib.OM_ERR_UNSUPPORTED
    assert "om_render_fwd_bwd_l2_noalloc" in L.om_last_error().decode()
    torch.cuda.synchronize()
    assert all(float(v.abs().max()) == 0.0 for v in grads.values())  # nothing ran
