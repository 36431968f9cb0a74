"""GPU: the frequency-encoded view direction of the deferred MLP (34 inputs,
Sec. 4.2 / appendix) and the view-smoothness loss (Eq. 9-10), against the
float64 oracle, through the C ABI.

Bars: FP32 colours and features within 1e-5 absolute (as the forward
tests); the bfloat16 MFMA MLP within the bf16-rounding bars of the forward
tests; parameter gradients for the oracle's float32 dL/dC per entry within
1e-3 relative + the entry's float32 rounding floor (tests/gradcheck.py, as
the backward tests); the smoothness loss within 1e-5 relative,
its dL/dF and dL/dW per entry within 1e-4 relative + 1e-6 of the largest
(float32 evaluation of an MLP whose float64 value is the reference).
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import paper_2404_09531_amd as om
import scenegen
from tests.gradcheck import check, oracle_reference, oracle_upstream
from tests.gpu_util import log, rays_to, upload_scene

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)
SOURCES = ("grid", "plane_xy", "plane_xz", "plane_yz")
TOL = 1e-5
ENC = dataclasses.replace(scenegen.TINY, dir_freqs=4)


@pytest.fixture(scope="module")
def enc_scene():
    sc = scenegen.make_scene(ENC)
    assert sc["mlp"].size == om.mlp_nparams(4) == 883
    scene, t = upload_scene(sc)
    assert scene.dir_freqs == 4
    o, d = scenegen.oblique_rays(1000, seed=5)  # 62.5 groups of 16: a ragged tail
    return sc, scene, t, o, d


def test_forward_encoded_fp32_vs_oracle(enc_scene):
    sc, scene, t, o, d = enc_scene
    log("test_forward_encoded_fp32_vs_oracle: 1000 rays, 34 MLP inputs")
    og, dg = rays_to(o, d)
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, mlp_bf16=0)
    ref = oracle.oracle_render(sc, o, d, oracle.RenderParams(n_max=64, c_bg=BG), keep_k=False)
    np.testing.assert_array_equal(res["n_placed"].cpu().numpy(), ref["n_placed"])
    np.testing.assert_allclose(res["F"].double().cpu().numpy(), ref["F"], atol=TOL, rtol=0)
    np.testing.assert_allclose(res["C"].double().cpu().numpy(), ref["C"], atol=TOL, rtol=0)
    # the encoding changes the colour: a 10-input MLP reading the same F differs
    assert (ref["n_placed"] > 0).sum() > 500


def test_forward_encoded_bf16_mlp(enc_scene):
    """bfloat16 MFMA MLP with three k-tiles in layer 1 (34 inputs padded to 48)."""
    sc, scene, t, o, d = enc_scene
    log("test_forward_encoded_bf16_mlp")
    og, dg = rays_to(o, d)
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, mlp_bf16=1)
    ref = oracle.oracle_render(sc, o, d, oracle.RenderParams(n_max=64, c_bg=BG), keep_k=False)
    err = np.abs(res["C"].double().cpu().numpy() - ref["C"])
    assert err.max() < 2e-2 and err.mean() < 3e-3, (err.max(), err.mean())
    np.testing.assert_allclose(res["F"].double().cpu().numpy(), ref["F"], atol=TOL, rtol=0)


def _target(sc, o, d):
    pert = scenegen.perturb_scene(sc, 0.05, seed=2)
    pert["dir_freqs"] = sc["dir_freqs"]
    return oracle.oracle_render(pert, o, d, oracle.RenderParams(n_max=64, c_bg=BG), keep_k=False)["C"]


def _vjp(scene, t, og, dg, up, batch_wv, dL_dF=None):
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, mlp_bf16=0, batch_wv=batch_wv)
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}
    om.render_backward(scene, og, dg, res, torch.from_numpy(up).to(og.device), grads, n_max=64, c_bg=BG,
                       dL_dF=dL_dF)
    torch.cuda.synchronize()
    return res, {k: v.double().cpu().numpy() for k, v in grads.items()}


def test_backward_encoded_vs_oracle(enc_scene):
    sc, scene, t, o, d = enc_scene
    o, d = o[:256], d[:256]
    log("test_backward_encoded_vs_oracle: 256 rays")
    target = _target(sc, o, d).astype(np.float32)
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target).to(og.device)
    prm = oracle.RenderParams(n_max=64, c_bg=BG)
    up, ref_loss = oracle_upstream(sc, o, d, prm, target)
    ref, scale = oracle_reference(sc, o, d, prm, up)
    for bw in (False, True):
        res, grads = _vjp(scene, t, og, dg, up, bw)
        assert abs(om.l2_loss_fp64(res["C"], tg).item() - ref_loss) <= 1e-4 * ref_loss
        check(grads, ref, scale, f"encoded batch_wv={bw}")


def _smooth_inputs(n, p, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    F = g.uniform(0.0, 1.0, (n, 7)).astype(np.float32)
    _, d = scenegen.oblique_rays(n, seed=seed + 1)
    return F, d, scenegen.view_perturbations(n, p, seed=seed + 2)


def _check_close(got, ref, rel, floor):
    excess = np.abs(got - ref) - (rel * np.abs(ref) + floor * max(np.abs(ref).max(), 1e-30))
    assert excess.max() <= 0, float(excess.max())


@pytest.mark.parametrize("freqs", [0, 4])
@pytest.mark.parametrize("n,p", [(1037, 4), (16, 1), (5, 64)])
def test_smooth_loss_vs_oracle(freqs, n, p):
    log(f"test_smooth_loss_vs_oracle: freqs={freqs} n={n} P={p}")
    cfg = dataclasses.replace(scenegen.TINY, dir_freqs=freqs)
    sc = scenegen.make_scene(cfg)
    scene, t = upload_scene(sc)
    F, d, pert = _smooth_inputs(n, p, seed=11 + n)
    w = float(np.float32(0.1))
    ref_loss, ref_dF, ref_dW = oracle.smooth_loss(F, d, pert, sc["mlp"], freqs, w)
    dev = t["mlp"].device
    Fg, dg, pg = (torch.from_numpy(a).to(dev) for a in (F, d, pert))
    dF = torch.zeros_like(Fg)
    dW = torch.zeros_like(t["mlp"])
    loss = om.smooth_loss(scene, Fg, dg, pg, w, dL_dF=dF, grad_mlp=dW)
    torch.cuda.synchronize()
    assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss), (loss.item(), ref_loss)
    _check_close(dF.double().cpu().numpy(), ref_dF, 1e-4, 1e-6)
    _check_close(dW.double().cpu().numpy(), ref_dW, 1e-4, 1e-6)
    # the gradients are ADDED: a second call doubles them
    om.smooth_loss(scene, Fg, dg, pg, w, dL_dF=dF, grad_mlp=dW, with_loss=False)
    torch.cuda.synchronize()
    _check_close(dF.double().cpu().numpy(), 2 * ref_dF, 1e-4, 1e-6)


def test_smooth_loss_zero_cases():
    """No rays: loss 0.  Zero perturbations: s = d, so every term is 0."""
    log("test_smooth_loss_zero_cases")
    sc = scenegen.make_scene(ENC)
    scene, t = upload_scene(sc)
    dev = t["mlp"].device
    e = torch.zeros((0, 7), dtype=torch.float32, device=dev)
    loss = om.smooth_loss(scene, e, torch.zeros((0, 3), dtype=torch.float32, device=dev),
                          torch.zeros((0, 2, 3), dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    assert loss.item() == 0.0
    F, d, _ = _smooth_inputs(40, 3, seed=3)
    Fg, dg = torch.from_numpy(F).to(dev), torch.from_numpy(d).to(dev)
    dF = torch.zeros_like(Fg)
    dW = torch.zeros_like(t["mlp"])
    loss = om.smooth_loss(scene, Fg, dg, torch.zeros((40, 3, 3), dtype=torch.float32, device=dev), 1.0,
                          dL_dF=dF, grad_mlp=dW)
    torch.cuda.synchronize()
    assert loss.item() == 0.0
    assert dF.abs().max().item() == 0.0 and dW.abs().max().item() == 0.0


@pytest.mark.parametrize("freqs", [0, 4])
def test_l2_plus_smooth_gradients_vs_oracle(freqs):
    """The features' gradient path: dL/dF of the smoothness loss fed to the
    render backward (om_render_backward_ex) and through torch autograd
    (RenderFn + SmoothFn) equals the float64 gradient of
    sum(dL/dC * C) + L_smooth for the oracle's L2 dL/dC."""
    log(f"test_l2_plus_smooth_gradients_vs_oracle: freqs={freqs}")
    sc = scenegen.make_scene(dataclasses.replace(scenegen.TINY, dir_freqs=freqs))
    scene, t = upload_scene(sc)
    o, d = scenegen.oblique_rays(256, seed=9)
    target = _target(sc, o, d).astype(np.float32)
    pert = scenegen.view_perturbations(256, 4, seed=10)
    w = float(np.float32(0.05))
    smooth = dict(perturb=pert, weight=w)
    prm = oracle.RenderParams(n_max=64, c_bg=BG)
    up, _ = oracle_upstream(sc, o, d, prm, target)
    ref, scale = oracle_reference(sc, o, d, prm, up, smooth=smooth)
    og, dg = rays_to(o, d)
    pg = torch.from_numpy(pert).to(og.device)
    upg = torch.from_numpy(up).to(og.device)
    # explicit calls
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, mlp_bf16=0, batch_wv=True)
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}
    dF = torch.zeros_like(res["F"])
    om.smooth_loss(scene, res["F"], dg, pg, w, dL_dF=dF, grad_mlp=grads["mlp"], with_loss=False)
    om.render_backward(scene, og, dg, res, upg, grads, n_max=64, c_bg=BG, dL_dF=dF)
    torch.cuda.synchronize()
    check({k: v.double().cpu().numpy() for k, v in grads.items()}, ref, scale, f"L2 + smooth freqs={freqs}")
    # autograd
    masters = [t[k].clone().requires_grad_(True) for k in (*SOURCES, "mlp")]
    opts = dict(n_max=64, delta=om.DELTA, t_term=0.0, c_bg=BG, mlp_bf16=0)
    C, _, F, _, _ = om.RenderFn.apply(scene, og, dg, opts, *masters)
    loss = (C * upg).sum() + om.SmoothFn.apply(scene, F, dg, pg, w, masters[4]).float()
    loss.backward()
    torch.cuda.synchronize()
    check({k: m.grad.double().cpu().numpy() for k, m in zip((*SOURCES, "mlp"), masters)}, ref, scale,
          f"autograd L2 + smooth freqs={freqs}")


def test_backward_encoded_bf16_storage_vs_oracle(enc_scene):
    """bfloat16 storage with the 34-input MLP: float32 arithmetic and master
    gradients must match the float64 oracle on the bfloat16-rounded scene."""
    sc, _, _, o, d = enc_scene
    o, d = o[:256], d[:256]
    log("test_backward_encoded_bf16_storage_vs_oracle: 256 rays")
    rsc = dict(sc)
    for k in SOURCES:
        rsc[k] = torch.from_numpy(sc[k]).to(torch.bfloat16).float().numpy()
    scene, t = upload_scene(sc, dtype=torch.bfloat16)
    target = _target(sc, o, d).astype(np.float32)
    og, dg = rays_to(o, d)
    prm = oracle.RenderParams(n_max=64, c_bg=BG)
    up, _ = oracle_upstream(rsc, o, d, prm, target)
    ref, scale = oracle_reference(rsc, o, d, prm, up)
    _, grads = _vjp(scene, t, og, dg, up, True)
    check(grads, ref, scale, "encoded bf16 storage")
