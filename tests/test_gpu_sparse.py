"""GPU: sparse voxel-block storage of the grid (Sec. 4.4) through the C ABI.

The block layout changes addresses only, so a sparse scene must render bit
for bit like its dense source (float32, bfloat16 and 8-bit storage, with
the soft occupancy and early termination too), on the tiny scene and on the
full oblique 1920x1080 frame; the dense renders are the ones checked
against the oracle elsewhere, and the tiny sparse render is checked against
the oracle here as well.  The index is checked for the properties the
render relies on (every block holding a placed sample is kept, ids 1..n in
index order) and the atlas against the dense grid (copied blocks, zero
apron past the grid's last vertex, block 0 zero).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2404_09531_amd as om
import scenegen
from tests.gpu_util import DEV, log, rays_to, upload_scene

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)
KEYS = ("C", "T", "F", "n_placed", "n_eval")


def _sparse_scene(scene, t, shift, quant=None):
    atlas, sg = om.sparse_grid(scene, shift)
    src = scene.tensors
    sp = om.Scene(atlas, src["plane_xy"], src["plane_xz"], src["plane_yz"], src["occ"], src["mlp"],
                  box_lo=tuple(scene._desc.box_lo), box_hi=tuple(scene._desc.box_hi), quant=quant, sparse=sg)
    return sp, atlas, sg


def _equal(a, b):
    for k in KEYS:
        assert torch.equal(a[k], b[k]), k


@pytest.fixture(scope="module")
def tiny():
    sc = scenegen.make_scene(scenegen.TINY)
    scene, t = upload_scene(sc)
    o, d = scenegen.oblique_rays(3000, seed=31)
    return sc, scene, t, o, d


@pytest.mark.parametrize("shift", [1, 2, 3, 4, 5])
def test_index_and_atlas(tiny, shift):
    log(f"test_index_and_atlas: B = {1 << shift}")
    sc, scene, t, o, d = tiny
    sp, atlas, sg = _sparse_scene(scene, t, shift)
    idx = sg.blocks.cpu().numpy()
    kept = idx[idx > 0]
    assert np.array_equal(kept, np.arange(1, sg.n_blocks + 1))  # ids 1..n in index order
    assert 0 < sg.n_blocks <= idx.size
    # every block that holds a placed sample is kept
    _, npl, pts = oracle.place_samples(o, d, sc["occ"], sc["box_lo"], sc["box_hi"], om.DELTA, 64)
    p = pts[np.arange(pts.shape[1])[None, :] < npl[:, None]].astype(np.float64)
    lo, hi = sc["box_lo"], sc["box_hi"]
    lz, ly, lx, _ = sc["grid"].shape
    cell = [np.minimum(np.floor((p[:, a] - lo[a]) / (hi[a] - lo[a]) * (n - 1)).astype(np.int64), n - 2)
            for a, n in ((0, lx), (1, ly), (2, lz))]
    assert (idx[cell[2] >> shift, cell[1] >> shift, cell[0] >> shift] > 0).all()
    # atlas blocks against the dense grid; past the last vertex the apron is zero
    a = atlas.cpu().numpy()
    e = (1 << shift) + 1
    assert not a[0].any()
    g = sc["grid"]
    rng = np.random.default_rng(shift)
    for bz, by, bx in zip(*np.nonzero(idx)):
        if rng.random() > 0.3:
            continue
        want = np.zeros((e, e, e, 8), np.float32)
        z0, y0, x0 = bz << shift, by << shift, bx << shift
        part = g[z0:z0 + e, y0:y0 + e, x0:x0 + e]
        want[:part.shape[0], :part.shape[1], :part.shape[2]] = part
        assert np.array_equal(a[idx[bz, by, bx]], want), (bz, by, bx)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "u8"])
@pytest.mark.parametrize("t_term,occ_eps", [(0.0, 0.0), (1e-3, 0.0), (0.0, 0.01)])
def test_sparse_render_equals_dense(tiny, dtype, t_term, occ_eps):
    log(f"test_sparse_render_equals_dense: {dtype} t_term={t_term} occ_eps={occ_eps}")
    sc, scene, t, o, d = tiny
    quant = None
    if dtype == "bf16":
        tb = {k: om.to_bf16(t[k]) for k in ("grid", "plane_xy", "plane_xz", "plane_yz")}
        scene = om.Scene(tb["grid"], tb["plane_xy"], tb["plane_xz"], tb["plane_yz"], t["occ"], t["mlp"])
    elif dtype == "u8":
        codes, quant = om.quantize_features(t)
        scene = om.Scene(codes["grid"], codes["plane_xy"], codes["plane_xz"], codes["plane_yz"], t["occ"], t["mlp"],
                         quant=quant)
    sp, _, _ = _sparse_scene(scene, t, 3, quant)
    og, dg = rays_to(o, d)
    kw = dict(n_max=64, c_bg=BG, t_term=t_term, occ_eps=occ_eps)
    _equal(om.render(sp, og, dg, **kw), om.render(scene, og, dg, **kw))


def test_sparse_render_vs_oracle(tiny):
    log("test_sparse_render_vs_oracle")
    sc, scene, t, o, d = tiny
    sp, _, _ = _sparse_scene(scene, t, 2)
    og, dg = rays_to(o, d)
    res = om.render(sp, og, dg, n_max=64, c_bg=BG)
    ref = oracle.oracle_render(sc, o, d, oracle.RenderParams(n_max=64, c_bg=BG), keep_k=False)
    assert np.array_equal(res["n_placed"].cpu().numpy(), ref["n_placed"])
    for k in ("C", "T", "F"):
        assert np.abs(res[k].double().cpu().numpy() - ref[k]).max() <= 1e-5, k


def test_sparse_scene_is_render_only(tiny):
    log("test_sparse_scene_is_render_only")
    sc, scene, t, o, d = tiny
    sp, _, _ = _sparse_scene(scene, t, 3)
    og, dg = rays_to(o[:64], d[:64])
    res = om.render(sp, og, dg, n_max=64, c_bg=BG)
    grads = {k: torch.zeros(t[k].shape, device=DEV) for k in ("plane_xy", "plane_xz", "plane_yz", "mlp")}
    grads["grid"] = torch.zeros(sp.tensors["grid"].shape, device=DEV)
    with pytest.raises(om.OmerfError):
        om.render_backward(sp, og, dg, res, torch.zeros_like(res["C"]), grads, n_max=64, c_bg=BG)
    with pytest.raises(ValueError):
        om.sparse_grid(sp, 3)


def test_sparse_oblique_1080p_equals_dense():
    """The bench's sparse forms: the full 1920x1080 oblique frame, every ray,
    float32 and 8-bit."""
    log("test_sparse_oblique_1080p_equals_dense: building the oblique scene")
    cfg, recipe = scenegen.workload("oblique-1080p")
    sc = scenegen.make_scene(cfg)
    scene, t = upload_scene(sc)
    del sc
    o, d = scenegen.make_rays(recipe)
    og, dg = rays_to(o, d)
    dense = om.render(scene, og, dg, n_max=256, c_bg=BG)
    sp, atlas, sg = _sparse_scene(scene, t, 3)
    log(f"  kept {sg.n_blocks} of {sg.blocks.numel()} blocks, atlas {atlas.numel() * 4 / 2**30:.2f} GiB "
        f"vs dense {t['grid'].numel() * 4 / 2**30:.2f} GiB")
    assert sg.n_blocks < sg.blocks.numel()
    _equal(om.render(sp, og, dg, n_max=256, c_bg=BG), dense)
    del sp, atlas, dense
    # the bench's 8-bit sparse form: 8-bit codes baked on the GPU, in blocks
    codes, quant = om.quantize_features(t)
    dense8 = om.Scene(codes["grid"], codes["plane_xy"], codes["plane_xz"], codes["plane_yz"], t["occ"], t["mlp"],
                      box_lo=tuple(scene._desc.box_lo), box_hi=tuple(scene._desc.box_hi), quant=quant)
    sp8, _, sg8 = _sparse_scene(dense8, t, 3, quant)
    log(f"  8-bit: kept {sg8.n_blocks} blocks")
    _equal(om.render(sp8, og, dg, n_max=256, c_bg=BG), om.render(dense8, og, dg, n_max=256, c_bg=BG))


def test_sparse_u8_with_pyramid_equals_dense(tiny):
    """8-bit sparse blocks with the occupancy pyramid attached: the same
    render as the dense 8-bit scene without it."""
    log("test_sparse_u8_with_pyramid_equals_dense")
    sc, scene, t, o, d = tiny
    codes, quant = om.quantize_features(t)
    dense = om.Scene(codes["grid"], codes["plane_xy"], codes["plane_xz"], codes["plane_yz"], t["occ"], t["mlp"],
                     quant=quant)
    sp, _, _ = _sparse_scene(dense, t, 3, quant)
    sp.build_occupancy_mips(3)
    og, dg = rays_to(o, d)
    _equal(om.render(sp, og, dg, n_max=64, c_bg=BG), om.render(dense, og, dg, n_max=64, c_bg=BG))
