"""Soft occupancy (Sec. 4.1, Eq. 5, 6, 8 with epsilon > 0) on the GPU
against the float64 oracle: forward colours, features and transmittance
(float32 bar 1e-5, bfloat16 storage against the oracle of the rounded
scene), gradients into features, MLP and the occupancy bounds (the
per-entry bar of tests/gradcheck.py), and the interval-span loss.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2404_09531_amd as om
import scenegen
from tests.gpu_util import bf16_round, log, rays_to, upload_scene
from tests.gradcheck import SOURCES, check, oracle_reference, oracle_upstream

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)
EPS = 0.01  # the tiny scene's intervals are 0.06 wide: a third of each lies in a buffer zone


@pytest.fixture(scope="module")
def tiny_soft():
    sc = scenegen.make_scene(scenegen.TINY)
    pert = scenegen.perturb_scene(sc, 0.05, seed=2)
    o, d = scenegen.oblique_rays(512, seed=3)
    target = oracle.oracle_render(pert, o, d, oracle.RenderParams(n_max=64, c_bg=BG, occ_eps=EPS),
                                  keep_k=False)["C"].astype(np.float32)
    return sc, o, d, target


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_soft_forward_matches_oracle(tiny_soft, dtype):
    sc, o, d, _ = tiny_soft
    log(f"test_soft_forward_matches_oracle: {dtype}, eps={EPS}")
    ref_sc = sc if dtype == torch.float32 else {**sc, **{k: bf16_round(sc[k]) for k in SOURCES}}
    scene, _ = upload_scene(sc, dtype=dtype)
    og, dg = rays_to(o, d)
    for t_term in (0.0, 1e-2):
        res = om.render(scene, og, dg, n_max=64, c_bg=BG, mlp_bf16=0, occ_eps=EPS, t_term=t_term)
        ref = oracle.oracle_render(ref_sc, o, d, oracle.RenderParams(n_max=64, c_bg=BG, occ_eps=EPS, t_term=t_term),
                                   keep_k=False)
        ne = res["n_eval"].cpu().numpy()
        same = ne == ref["n_eval"]
        assert same.mean() > 0.99
        for key in ("C", "F", "T"):
            err = np.abs(res[key].double().cpu().numpy()[same] - ref[key][same]).max()
            log(f"  t_term={t_term}: max |{key} - oracle| = {err:.2e}")
            assert err <= 1e-5, key
    # the soft mask changes the colours (it is not a no-op)
    hard = oracle.oracle_render(ref_sc, o, d, oracle.RenderParams(n_max=64, c_bg=BG), keep_k=False)
    assert np.abs(hard["C"] - ref["C"]).max() > 1e-3


@pytest.mark.parametrize("dtype,batch_wv", [(torch.float32, False), (torch.float32, True), (torch.bfloat16, True)])
def test_soft_backward_matches_oracle(tiny_soft, dtype, batch_wv):
    """float32 storage with and without the per-batch sums, and bfloat16
    storage (float32 master gradients) against the oracle of the rounded
    scene."""
    sc, o, d, target = tiny_soft
    log(f"test_soft_backward_matches_oracle: {dtype}, batch sums {batch_wv}")
    ref_sc = sc if dtype == torch.float32 else {**sc, **{k: bf16_round(sc[k]) for k in SOURCES}}
    scene, t = upload_scene(sc, dtype=dtype)
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target).to(og.device)
    prm = oracle.RenderParams(n_max=64, c_bg=BG, occ_eps=EPS)
    up, ref_loss = oracle_upstream(ref_sc, o, d, prm, target)
    ref, scale = oracle_reference(ref_sc, o, d, prm, up)
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, occ_eps=EPS, batch_wv=batch_wv, mlp_bf16=0)
    loss = om.l2_loss_fp64(res["C"], tg).item()
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp", "occ")}
    om.render_backward(scene, og, dg, res, torch.from_numpy(up).to(og.device), grads, n_max=64, c_bg=BG,
                       occ_eps=EPS)
    g = {k: v.double().cpu().numpy() for k, v in grads.items()}
    assert np.abs(ref["occ"][1]).max() > 0
    check(g, ref, scale, f"tiny soft occupancy {dtype} batch_wv={batch_wv}")


def test_soft_render_fn_returns_occupancy_gradient(tiny_soft):
    """RenderFn hands the occupancy gradient to autograd: the loss
    sum(dL/dC * C) with the oracle's dL/dC gives the oracle's gradient."""
    sc, o, d, target = tiny_soft
    log("test_soft_render_fn_returns_occupancy_gradient")
    scene, t = upload_scene(sc)
    og, dg = rays_to(o, d)
    prm = oracle.RenderParams(n_max=64, c_bg=BG, occ_eps=EPS)
    up, _ = oracle_upstream(sc, o, d, prm, target)
    ref, scale = oracle_reference(sc, o, d, prm, up)
    masters = [t[k].clone().requires_grad_(True) for k in (*SOURCES, "mlp", "occ")]
    C, *_ = om.RenderFn.apply(scene, og, dg, dict(n_max=64, c_bg=BG, occ_eps=EPS), *masters)
    (C * torch.from_numpy(up).to(og.device)).sum().backward()
    torch.cuda.synchronize()
    g = {k: m.grad.double().cpu().numpy() for k, m in zip((*SOURCES, "mlp", "occ"), masters)}
    check(g, ref, scale, "RenderFn soft occupancy")


def test_occ_interval_loss_matches_eq5():
    sc = scenegen.make_scene(scenegen.TOWERS)
    occ = torch.from_numpy(sc["occ"]).cuda()
    log("test_occ_interval_loss_matches_eq5: 512 x 512 cells")
    grad = torch.full_like(occ, 0.5)
    w = float(np.float32(0.3))  # the weight crosses the boundary as a float32
    loss = om.occ_interval_loss(occ, weight=w, grad=grad)
    ref_loss, ref_grad = oracle.occ_interval_loss(sc["occ"])
    # float32 sum of nonnegative terms by 1024 lanes: k = ceil(cells / 1024)
    # serial additions per lane, a 6-step butterfly, 16 wave partials, the
    # weight; each term (z_max - z_min)^2 rounds twice (3 u with the weight's
    # own rounding already in w): relative error <= (k + 6 + 16 + 4) u.
    k = -(-occ.shape[0] * occ.shape[1] // 1024)
    assert loss.item() == pytest.approx(w * ref_loss, rel=(k + 26) * 2.0 ** -24)
    np.testing.assert_allclose(grad.double().cpu().numpy(), 0.5 + w * ref_grad, rtol=1e-6, atol=1e-7)
