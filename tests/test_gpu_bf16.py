"""BF16 form: bfloat16 grid/plane storage with float32 arithmetic, and the
bfloat16 MFMA deferred MLP.

* The march computes in float32 on bfloat16-stored features, so its outputs
  (F, T, counts) must match the float64 oracle run on the bfloat16-rounded
  scene to the float32 bar (1e-5).
* Fidelity of the full BF16 form against the float64 oracle of the float32
  scene is reported (max-abs, PSNR) and bounded.
* Quality gate: PSNR of the BF16 render minus PSNR of the FP32 render, both
  against the float64 oracle render of the perturbed scene (a ground-truth
  stand-in), must not fall by more than 0.1 dB.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2404_09531_amd as om
import scenegen
from tests.gpu_util import bf16_round, log, rays_to, upload_scene

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)


def psnr(a, b):
    mse = np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2)
    return 10.0 * np.log10(1.0 / mse)


def _rounded(sc):
    r = dict(sc)
    for k in ("grid", "plane_xy", "plane_xz", "plane_yz"):
        r[k] = bf16_round(sc[k])
    return r


def test_bf16_march_matches_oracle_on_rounded_scene():
    sc = scenegen.make_scene(scenegen.TINY)
    o, d = scenegen.oblique_rays(4096, seed=1)
    log("test_bf16_march_matches_oracle_on_rounded_scene")
    scene, t = upload_scene(sc, dtype=torch.bfloat16)
    og, dg = rays_to(o, d)
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, mlp_bf16=0)
    ref = oracle.oracle_render(_rounded(sc), o, d, oracle.RenderParams(n_max=64, c_bg=BG), keep_k=False)
    assert np.array_equal(res["n_eval"].cpu().numpy(), ref["n_eval"])
    for key in ("F", "T", "C"):
        err = np.abs(res[key].double().cpu().numpy() - ref[key]).max()
        log(f"  bf16 storage, fp32 MLP: max |{key} - oracle(rounded)| = {err:.2e}")
        assert err <= 1e-5, key
    # full BF16 form (MFMA MLP): bounded by bfloat16 rounding of the MLP
    res2 = om.render(scene, og, dg, n_max=64, c_bg=BG)
    err2 = np.abs(res2["C"].double().cpu().numpy() - ref["C"]).max()
    err2m = np.abs(res2["C"].double().cpu().numpy() - ref["C"]).mean()
    log(f"  bf16 storage + bf16 MFMA MLP: max |C - oracle(rounded)| = {err2:.2e}, mean {err2m:.2e}")
    assert err2 < 4e-3 and err2m < 7e-4  # about 3x the measured 1.24e-3 / 2.2e-4


def test_bf16_ert_rule():
    """Early termination in the bfloat16 kernel: counts agree with the oracle
    on the rounded scene except, by one, where the transmittance at the
    crossing is within 1e-4 (relative) of t_term; equal counts give colours
    within the float32 bar."""
    sc = scenegen.make_scene(scenegen.TINY)
    o, d = scenegen.oblique_rays(4096, seed=1)
    t_term = 1e-2
    log("test_bf16_ert_rule: t_term=1e-2")
    scene, t = upload_scene(sc, dtype=torch.bfloat16)
    og, dg = rays_to(o, d)
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, t_term=t_term, mlp_bf16=0)
    ref = oracle.oracle_render(_rounded(sc), o, d, oracle.RenderParams(n_max=64, c_bg=BG, t_term=t_term),
                               keep_k=False)
    nev = res["n_eval"].cpu().numpy()
    same = nev == ref["n_eval"]
    assert same.mean() > 0.99
    if (~same).any():
        assert np.all(np.abs(nev[~same] - ref["n_eval"][~same]) == 1)
        near = np.abs(ref["T"][~same] - t_term) / t_term
        assert np.all(near <= 1e-4), near
    assert np.abs(res["C"].double().cpu().numpy()[same] - ref["C"][same]).max() <= 1e-5
    assert (nev < 64).any()


@pytest.fixture(scope="module")
def oblique_crop():
    log("building oblique scene and its perturbed copy")
    sc = scenegen.make_scene(scenegen.OBLIQUE)
    pert = scenegen.perturb_scene(sc, 0.05, seed=2)
    w, h, c = 1920, 1080, 256
    pix = np.array([(h // 2 - c // 2 + j) * w + (w // 2 - c // 2 + i) for j in range(c) for i in range(c)])
    o, d = scenegen.camera_rays(w, h, 45.0, 90.0, pixels=pix)
    prm = oracle.RenderParams(n_max=256, c_bg=BG)
    log("oracle renders of the 256x256 crop (scene, perturbed scene)")
    ref = oracle.oracle_render(sc, o, d, prm, keep_k=False)["C"]
    gt = oracle.oracle_render(pert, o, d, prm, keep_k=False)["C"]
    return sc, o, d, ref, gt


def test_bf16_psnr_gate_and_fidelity(oblique_crop):
    sc, o, d, ref, gt = oblique_crop
    log("test_bf16_psnr_gate_and_fidelity: 256x256 crop of the oblique 1080p image")
    og, dg = rays_to(o, d)
    s32, _ = upload_scene(sc)
    c32 = om.render(s32, og, dg, n_max=256, c_bg=BG)["C"].double().cpu().numpy()
    del s32
    torch.cuda.empty_cache()
    s16, _ = upload_scene(sc, dtype=torch.bfloat16)
    c16 = om.render(s16, og, dg, n_max=256, c_bg=BG)["C"].double().cpu().numpy()
    e32, e16 = np.abs(c32 - ref).max(), np.abs(c16 - ref).max()
    p32, p16 = psnr(c32, ref), psnr(c16, ref)
    g32, g16 = psnr(c32, gt), psnr(c16, gt)
    log(f"  fidelity vs FP64 oracle: FP32 max-abs {e32:.2e} PSNR {p32:.1f} dB; "
        f"BF16 max-abs {e16:.2e} PSNR {p16:.1f} dB")
    log(f"  vs perturbed-scene target: FP32 {g32:.3f} dB, BF16 {g16:.3f} dB, loss {g32 - g16:.4f} dB")
    # about 3x the measured 2.65e-3 / 70.2 dB (one MI355X)
    assert e32 <= 1e-5
    assert e16 < 8e-3 and p16 > 61.0
    assert g32 - g16 <= 0.1


def test_u8_psnr_gate_and_fidelity(oblique_crop):
    """The 8-bit form (features baked on the GPU, float32 MLP) under the same
    quality gate as bfloat16: at most 0.1 dB below the float32 render against
    the perturbed-scene target."""
    sc, o, d, ref, gt = oblique_crop
    log("test_u8_psnr_gate_and_fidelity: 256x256 crop of the oblique 1080p image")
    og, dg = rays_to(o, d)
    s32, t = upload_scene(sc)
    c32 = om.render(s32, og, dg, n_max=256, c_bg=BG)["C"].double().cpu().numpy()
    codes, quant = om.quantize_features(t)
    s8 = om.Scene(codes["grid"], codes["plane_xy"], codes["plane_xz"], codes["plane_yz"], t["occ"], t["mlp"],
                  quant=quant)
    c8 = om.render(s8, og, dg, n_max=256, c_bg=BG)["C"].double().cpu().numpy()
    e8, p8 = np.abs(c8 - ref).max(), psnr(c8, ref)
    g32, g8 = psnr(c32, gt), psnr(c8, gt)
    log(f"  fidelity vs FP64 oracle: 8-bit max-abs {e8:.2e} PSNR {p8:.1f} dB")
    log(f"  vs perturbed-scene target: FP32 {g32:.3f} dB, 8-bit {g8:.3f} dB, loss {g32 - g8:.4f} dB")
    # about 3x the measured 5.3e-3 / 64.3 dB
    assert e8 < 1.6e-2 and p8 > 55.0
    assert g32 - g8 <= 0.1


def test_bf16_4k_image0_crop_fidelity():
    """The 8 x 3840x2160 bfloat16 form, image 0 (the bench's first camera):
    on its centre 256x256 crop the float32 render matches the float64 oracle
    to 1e-5; bfloat16 storage with the float32 MLP matches the oracle run on
    the bfloat16-rounded scene to 1e-5 (the compute error alone); the full
    bfloat16 form (MFMA MLP) is reported and bounded against the oracle."""
    log("test_bf16_4k_image0_crop_fidelity: building the oblique scene")
    sc = scenegen.make_scene(scenegen.OBLIQUE)
    pitch, yaw, aim = scenegen.random_cameras(8, seed=3)[0]
    w, h, c = 3840, 2160, 256
    pix = np.array([(h // 2 - c // 2 + j) * w + (w // 2 - c // 2 + i) for j in range(c) for i in range(c)])
    o, d = scenegen.camera_rays(w, h, pitch, yaw, aim, pixels=pix)
    prm = oracle.RenderParams(n_max=256, c_bg=BG)
    log("  oracle renders of the crop (scene, bf16-rounded scene)")
    ref = oracle.oracle_render(sc, o, d, prm, keep_k=False)
    ref16 = oracle.oracle_render(_rounded(sc), o, d, prm, keep_k=False)
    og, dg = rays_to(o, d)
    s32, _ = upload_scene(sc)
    r32 = om.render(s32, og, dg, n_max=256, c_bg=BG)
    e32 = np.abs(r32["C"].double().cpu().numpy() - ref["C"]).max()
    del s32, r32
    torch.cuda.empty_cache()
    s16, _ = upload_scene(sc, dtype=torch.bfloat16)
    r16 = om.render(s16, og, dg, n_max=256, c_bg=BG, mlp_bf16=0)
    e16s = np.abs(r16["C"].double().cpu().numpy() - ref16["C"]).max()
    full = om.render(s16, og, dg, n_max=256, c_bg=BG)["C"].double().cpu().numpy()
    e16, p16 = np.abs(full - ref["C"]).max(), psnr(full, ref["C"])
    log(f"  FP32 max-abs {e32:.2e}; bf16 storage vs rounded-scene oracle {e16s:.2e}; "
        f"full BF16 max-abs {e16:.2e} PSNR {p16:.1f} dB; {int((ref['n_placed'] > 0).sum())} rays hit")
    assert e32 <= 1e-5 and e16s <= 1e-5
    assert e16 < 1.05e-2 and p16 > 60.0  # about 3x the measured 3.5e-3 / 69.2 dB


def test_bf16_oblique_1080p_sampled_parity():
    """The bfloat16 form in the benchmark's launch configuration: the full
    1920x1080 oblique frame in Morton order from bfloat16 storage.  Sampled
    rays against the oracle on the bfloat16-rounded scene: with the float32
    MLP at the float32 bars; with the bf16 MFMA MLP the march outputs are
    unchanged and C stays within the bf16 bars."""
    log("test_bf16_oblique_1080p_sampled_parity: building the oblique scene")
    cfg, recipe = scenegen.workload("oblique-1080p")
    sc = scenegen.make_scene(cfg)
    o, d = scenegen.make_rays(recipe)
    scene, _ = upload_scene(sc, dtype=torch.bfloat16)
    og, dg = rays_to(o, d)
    res = om.render(scene, og, dg, n_max=256, c_bg=BG, mlp_bf16=0)
    full = om.render(scene, og, dg, n_max=256, c_bg=BG)
    torch.cuda.synchronize()
    for key in ("F", "T", "n_placed", "n_eval"):
        assert torch.equal(res[key], full[key]), key
    rng = np.random.default_rng(11)
    n = o.shape[0]
    rows = np.unique(np.concatenate([rng.choice(n, 800, replace=False), np.arange(16), np.arange(n - 21, n)]))
    ref = oracle.oracle_render(_rounded(sc), o[rows], d[rows], oracle.RenderParams(n_max=256, c_bg=BG),
                               keep_k=False)
    assert np.array_equal(res["n_placed"].cpu().numpy()[rows], ref["n_placed"])
    assert np.array_equal(res["n_eval"].cpu().numpy()[rows], ref["n_eval"])
    for key in ("F", "T", "C"):
        err = np.abs(res[key].double().cpu().numpy()[rows] - ref[key]).max()
        log(f"  bf16 storage, fp32 MLP: max |{key} - oracle(rounded)| = {err:.2e}")
        assert err <= 1e-5, key
    err = np.abs(full["C"].double().cpu().numpy()[rows] - ref["C"])
    log(f"  full bf16 form: max |C - oracle(rounded)| = {err.max():.2e}, mean {err.mean():.2e}")
    assert err.max() < 3e-3 and err.mean() < 6e-4  # about 3x the measured 1.0e-3 / 2.0e-4


def _bits_f32(u):
    return np.asarray(u, dtype=np.uint32).view(np.float32)


def test_cast_bf16_bit_exact():
    """om_cast_bf16 (the bfloat16 shadow refresh) rounds to nearest even
    exactly as the CPU conversion does: ties to even at both parities, the
    round-up into infinity above the largest bfloat16, subnormals, signed
    zeros and infinities; NaN stays NaN.  Random values over the whole
    exponent range, with a ragged tail (n mod 8 = 3)."""
    log("test_cast_bf16_bit_exact")
    special = _bits_f32([0x00000000, 0x80000000, 0x3f800000, 0xbf800000, 0x3f808000, 0x3f818000, 0x3f80ffff,
                         0x3f817fff, 0x7f7f0000, 0x7f7f7fff, 0x7f7f8000, 0x7f7fffff, 0xff7f8000, 0x7f800000,
                         0xff800000, 0x00000001, 0x00008000, 0x00018000, 0x807fffff, 0x00800000, 0x7fc00000,
                         0x7f800001, 0xffc00001])
    rng = np.random.default_rng(12)
    rand = rng.integers(0, 2 ** 32, size=1_000_003, dtype=np.uint64).astype(np.uint32).view(np.float32)
    for x in (special, rand):
        xg = torch.from_numpy(x.copy()).cuda()
        got = om.to_bf16(xg).view(torch.int16).cpu().numpy().view(np.uint16)
        want = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        nan = np.isnan(x)
        back = got.astype(np.uint32) << 16
        assert np.all(np.isnan(back.view(np.float32)[nan]))
        mism = np.nonzero(got[~nan] != want[~nan])[0]
        log(f"  {x.size} values, {int(nan.sum())} NaN, {mism.size} mismatches")
        assert mism.size == 0, [(hex(x[~nan].view(np.uint32)[i]), hex(got[~nan][i]), hex(want[~nan][i]))
                                for i in mism[:5]]


def test_cast_bf16_shadow_refresh_and_errors():
    """The re-cast after an optimiser step writes into the existing shadow
    (no new tensor), and the call rejects misaligned or overlapping buffers;
    n = 0 is a no-op."""
    log("test_cast_bf16_shadow_refresh_and_errors")
    master = torch.randn(4096, 8, device="cuda")
    shadow = om.to_bf16(master)
    ptr = shadow.data_ptr()
    master -= 0.01 * torch.randn_like(master)  # an optimiser step
    om.to_bf16(master, out=shadow)
    assert shadow.data_ptr() == ptr
    assert torch.equal(shadow.cpu(), master.cpu().to(torch.bfloat16))
    L = om._lib.lib()
    base = torch.zeros(64, device="cuda")
    out = torch.zeros(64, dtype=torch.bfloat16, device="cuda")
    assert L.om_cast_bf16(base.data_ptr() + 4, 8, out.data_ptr(), None) == om._lib.OM_ERR_INVALID
    assert L.om_cast_bf16(base.data_ptr(), 8, base.data_ptr() + 16, None) == om._lib.OM_ERR_INVALID
    assert L.om_cast_bf16(base.data_ptr(), 0, out.data_ptr(), None) == om._lib.OM_OK
    assert L.om_cast_bf16(0, 8, out.data_ptr(), None) == om._lib.OM_ERR_INVALID
