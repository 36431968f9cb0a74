"""Occupancy pyramid (hierarchical empty-space skipping over blocks of
2^l x 2^l columns): the pyramid equals min/max pooling of the occupancy
plane, and attaching it changes no sample: k-lists and counts stay
bit-exact against the oracle and renders are identical with and without it.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2404_09531_amd as om
import scenegen
from tests.gpu_util import log, rays_to, upload_scene

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)


def _pool(z):
    """Plain 2 x 2 pooling: (min z_min, max z_max) over the non-empty cells
    (z_min <= z_max); (+inf, -inf) when there is none."""
    h, w = z.shape[0] // 2, z.shape[1] // 2
    q = z[:2 * h, :2 * w].reshape(h, 2, w, 2, 2).transpose(0, 2, 1, 3, 4).reshape(h, w, 4, 2)
    ok = q[..., 0] <= q[..., 1]
    lo = np.where(ok, q[..., 0], np.inf).min(axis=2)
    hi = np.where(ok, q[..., 1], -np.inf).max(axis=2)
    return np.stack([lo, hi], axis=-1).astype(np.float32)


@pytest.mark.parametrize("name,levels", [("tiny", 5), ("towers-2^20", 4)])
def test_pyramid_equals_pooling(name, levels):
    log(f"test_pyramid_equals_pooling: {name}, {levels} levels")
    cfg, _ = scenegen.workload(name)
    sc = scenegen.make_scene(cfg)
    scene, _ = upload_scene(sc)
    scene.build_occupancy_mips(levels)
    got = [m.cpu().numpy() for m in scene.occupancy_mips()]
    z = sc["occ"].astype(np.float32)
    for lvl in range(levels):
        z = _pool(z)
        assert np.array_equal(got[lvl], z), lvl
    assert got[-1].shape[:2] == (sc["occ"].shape[0] >> levels, sc["occ"].shape[1] >> levels)


def _placement_with_and_without(sc, o, d, n_max, levels, rows=None):
    scene, _ = upload_scene(sc)
    if not np.array_equal(sc["box_hi"], scenegen.BOX_HI):  # same tensors over another box
        t = scene.tensors
        scene = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], t["mlp"],
                         box_lo=tuple(sc["box_lo"]), box_hi=tuple(sc["box_hi"]))
    og, dg = rays_to(o, d)
    k0, c0 = om.place_samples(scene, og, dg, n_max=n_max)
    r0 = om.render(scene, og, dg, n_max=n_max, c_bg=BG)
    scene.build_occupancy_mips(levels)
    k1, c1 = om.place_samples(scene, og, dg, n_max=n_max)
    r1 = om.render(scene, og, dg, n_max=n_max, c_bg=BG)
    torch.cuda.synchronize()
    assert torch.equal(k0, k1) and torch.equal(c0, c1)
    for key in r0:
        assert torch.equal(r0[key], r1[key]), key
    sel = slice(None) if rows is None else rows
    kr, nr, _ = oracle.place_samples(o[sel], d[sel], sc["occ"], sc["box_lo"], sc["box_hi"], om.DELTA, n_max)
    assert np.array_equal(c1.cpu().numpy()[sel], nr)
    assert np.array_equal(k1.cpu().numpy()[sel], kr)


def test_tiny_placement_unchanged_by_pyramid():
    log("test_tiny_placement_unchanged_by_pyramid: 4096 rays, 5 levels")
    sc = scenegen.make_scene(scenegen.TINY)
    o, d = scenegen.oblique_rays(4096, seed=1)
    _placement_with_and_without(sc, o, d, 64, 5)


def test_towers_placement_unchanged_by_pyramid():
    log("test_towers_placement_unchanged_by_pyramid: 2^20 rays (oracle on 2000), 4 levels")
    cfg, rec = scenegen.workload("towers-2^20")
    sc = scenegen.make_scene(cfg)
    o, d = scenegen.make_rays(rec)
    rows = np.unique(np.random.default_rng(5).choice(o.shape[0], 2000, replace=False))
    _placement_with_and_without(sc, o, d, rec["n_max"], 4, rows)


def test_oblique_placement_unchanged_by_pyramid():
    log("test_oblique_placement_unchanged_by_pyramid: 1080p (oracle on 1500), 5 levels")
    cfg, rec = scenegen.workload("oblique-1080p")
    sc = scenegen.make_scene(cfg)
    o, d = scenegen.make_rays(rec)
    rows = np.unique(np.random.default_rng(6).choice(o.shape[0], 1500, replace=False))
    _placement_with_and_without(sc, o, d, rec["n_max"], 5, rows)


def test_tall_box_placement_unchanged_by_pyramid():
    """A box four times taller than the terrain (a high-altitude view: the
    upper three quarters of every column are empty), where the pyramid skips
    the most."""
    log("test_tall_box_placement_unchanged_by_pyramid: tiny scene in a [0, 1] z box, 4096 rays")
    sc = dict(scenegen.make_scene(scenegen.TINY))
    sc["box_hi"] = np.array([1.0, 1.0, 1.0])
    o, d = scenegen.camera_rays(64, 64, 45.0, 30.0, origin_z=1.5)
    _placement_with_and_without(sc, o, d, 64, 4)


def test_pyramid_detached_by_update():
    sc = scenegen.make_scene(scenegen.TINY)
    scene, t = upload_scene(sc)
    scene.build_occupancy_mips(3)
    assert scene.mip_levels == 3
    scene.update(occ=t["occ"].clone())
    assert scene.mip_levels == 0 and scene.occupancy_mips() == []


def test_high_altitude_1080p_form():
    """The bench's high-altitude form: the oblique scene's tensors over a
    [0, 1] z box, one 1920x1080 camera at pitch 45 deg from z = 1.5 in Morton
    order.  The 4-level pyramid leaves placement and render unchanged, and
    sampled rays match the oracle."""
    log("test_high_altitude_1080p_form: 1080p, 4 levels (oracle on 700 rays)")
    cfg, _ = scenegen.workload("oblique-1080p")
    sc = dict(scenegen.make_scene(cfg))
    sc["box_hi"] = np.array([1.0, 1.0, 1.0])
    o, d = scenegen.camera_rays(1920, 1080, 45.0, 90.0, origin_z=1.5,
                                pixels=scenegen.pixel_order(1920, 1080, "morton"))
    rows = np.unique(np.concatenate([np.random.default_rng(12).choice(o.shape[0], 700, replace=False),
                                     np.arange(16), np.arange(o.shape[0] - 21, o.shape[0])]))
    _placement_with_and_without(sc, o, d, 256, 4, rows)
    scene, t = upload_scene(sc)
    tall = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], t["mlp"],
                    box_lo=tuple(sc["box_lo"]), box_hi=(1.0, 1.0, 1.0))
    tall.build_occupancy_mips(4)
    og, dg = rays_to(o, d)
    res = om.render(tall, og, dg, n_max=256, c_bg=BG)
    ref = oracle.oracle_render(sc, o[rows], d[rows], oracle.RenderParams(n_max=256, c_bg=BG), keep_k=False)
    assert np.array_equal(res["n_eval"].cpu().numpy()[rows], ref["n_eval"])
    for key in ("C", "T", "F"):
        err = np.abs(res[key].double().cpu().numpy()[rows] - ref[key]).max()
        log(f"  max |{key} - oracle| = {err:.2e}")
        assert err <= 1e-5, key
