"""Ray locality order (om_order_rays) and the row gathers that apply it.

The order is scheduling, not method: the checks are that it is a
permutation, that it lists the rays by the documented key (recomputed here
in float64; rays whose key point lies within 1e-3 cells of a lattice line
are left out, since float32 may put them on either side), that the
reordered rays are exact copies, and that a render of the reordered rays,
scattered back, is bit-identical to a render in input order (each ray is
rendered on its own, Eq. 1-3)."""
import numpy as np
import pytest
import torch

import paper_2404_09531_amd as om
import scenegen
from gpu_util import DEV, log, rays_to, upload_scene

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)
CELLS = 256


def _spread(v):
    v = v.astype(np.int64) & 0xFF
    v = (v | (v << 4)) & 0x0F0F
    v = (v | (v << 2)) & 0x3333
    v = (v | (v << 1)) & 0x5555
    return v


def host_keys(o, d, lo, hi):
    """The documented key in float64, and a mask of rays whose key point is
    too close to a lattice line (or the footprint edge) to call."""
    o = o.astype(np.float64)
    d = d.astype(np.float64)
    zm = 0.5 * (np.float32(lo[2]) + np.float32(hi[2]))
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(d[:, 2] != 0, (zm - o[:, 2]) / d[:, 2], 0.0)
    t = np.where(np.isfinite(t), t, 0.0)
    cells = []
    close = np.zeros(o.shape[0], dtype=bool)
    for a in (0, 1):
        u = (o[:, a] + t * d[:, a] - lo[a]) * (CELLS / (hi[a] - lo[a]))
        u = np.where(np.isfinite(u), u, 0.0)
        frac = u - np.floor(u)
        close |= (np.minimum(frac, 1 - frac) < 1e-3) & (u > -1e-3) & (u < CELLS + 1e-3)
        cells.append(np.clip(np.floor(u), 0, CELLS - 1).astype(np.int64))
    return _spread(cells[0]) | (_spread(cells[1]) << 1), close


def _check_order(scene_box, o, d, order, os_, ds_):
    n = o.shape[0]
    order = order.cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(n, dtype=np.int32)), "not a permutation"
    assert np.array_equal(os_.cpu().numpy(), o[order])
    assert np.array_equal(ds_.cpu().numpy(), d[order])
    keys, close = host_keys(o, d, *scene_box)
    k = keys[order][~close[order]]
    assert np.all(np.diff(k) >= 0), "rays not listed by key"
    return keys[order]


@pytest.fixture(scope="module")
def tiny():
    sc = scenegen.make_scene(scenegen.TINY)
    scene, t = upload_scene(sc)
    return sc, scene, t, (sc["box_lo"], sc["box_hi"])


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4096, 4096 + 37])
def test_order_is_a_keyed_permutation(tiny, n):
    sc, scene, t, box = tiny
    log(f"test_order_is_a_keyed_permutation: {n} oblique rays")
    o, d = scenegen.oblique_rays(n, seed=3)
    og, dg = rays_to(o, d)
    order, os_, ds_ = om.order_rays(scene, og, dg)
    torch.cuda.synchronize()
    _check_order(box, o, d, order, os_, ds_)


def test_order_of_a_row_major_frame(tiny):
    """A full 1920 x 1080 frame in row-major pixel order: equal keys keep
    their input order within runs of consecutive rays, so each key's rays
    form few runs of increasing input index."""
    sc, scene, t, box = tiny
    o, d = scenegen.camera_rays(1920, 1080, 45.0, 90.0)
    log(f"test_order_of_a_row_major_frame: {o.shape[0]} rays")
    og, dg = rays_to(o, d)
    order, os_, ds_ = om.order_rays(scene, og, dg)
    torch.cuda.synchronize()
    keys = _check_order(box, o, d, order, os_, ds_)
    idx = order.cpu().numpy()
    same = keys[1:] == keys[:-1]
    rising = idx[1:] > idx[:-1]
    assert np.mean(rising[same]) > 0.85


def test_order_degenerate_rays(tiny):
    """Rays parallel to the key plane, through the footprint's corners,
    with non-finite origins, and far outside the box still get a
    permutation."""
    sc, scene, t, box = tiny
    o = np.array([[0.0, 0.0, 0.125], [-1.0, -1.0, 1.0], [1.0, 1.0, 1.0], [np.nan, 0.0, 1.0],
                  [50.0, -50.0, 1.0], [0.3, 0.2, 0.125]], dtype=np.float32)
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 0.0, -1.0], [0.0, 0.0, -1.0],
                  [0.0, 0.6, -0.8], [0.0, 0.0, 0.0]], dtype=np.float32)
    o = np.tile(o, (20, 1))
    d = np.tile(d, (20, 1))
    og, dg = rays_to(o, d)
    order, os_, ds_ = om.order_rays(scene, og, dg)
    torch.cuda.synchronize()
    idx = order.cpu().numpy()
    assert np.array_equal(np.sort(idx), np.arange(o.shape[0], dtype=np.int32))
    assert np.array_equal(os_.cpu().numpy(), o[idx], equal_nan=True)
    assert np.array_equal(ds_.cpu().numpy(), d[idx])


@pytest.mark.parametrize("n_max", [64, 200])
def test_ordered_render_is_bit_identical(tiny, n_max):
    sc, scene, t, box = tiny
    n = 4096 + 37
    log(f"test_ordered_render_is_bit_identical: {n} rays, n_max={n_max}")
    o, d = scenegen.oblique_rays(n, seed=5)
    og, dg = rays_to(o, d)
    plain = om.render(scene, og, dg, n_max=n_max, c_bg=BG)
    order, os_, ds_ = om.order_rays(scene, og, dg)
    sorted_ = om.render(scene, os_, ds_, n_max=n_max, c_bg=BG)
    for key in ("C", "T", "F", "n_placed", "n_eval"):
        back = torch.full_like(plain[key], -7)
        if back.dtype == torch.float32:
            om.scatter_rows(sorted_[key], order, back)
            torch.cuda.synchronize()
            assert torch.equal(back, plain[key]), key
        else:
            back[order.long()] = sorted_[key]
            torch.cuda.synchronize()
            assert torch.equal(back, plain[key]), key


@pytest.mark.parametrize("cols", [1, 3, 8])
def test_gather_and_scatter_rows(cols):
    n = 5000 + cols
    log(f"test_gather_and_scatter_rows: {n} rows x {cols}")
    g = np.random.default_rng(cols)
    src = g.standard_normal((n, cols)).astype(np.float32)
    perm = g.permutation(n).astype(np.int32)
    s = torch.from_numpy(src).to(DEV)
    idx = torch.from_numpy(perm).to(DEV)
    got = om.gather_rows(s, idx)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), src[perm])
    back = torch.zeros_like(s)
    om.scatter_rows(got, idx, back)
    torch.cuda.synchronize()
    assert np.array_equal(back.cpu().numpy(), src)


def test_rows_skip_indices_outside():
    src = np.arange(30, dtype=np.float32).reshape(10, 3)
    idx = np.array([2, -1, 9, 10, 0, 1 << 30], dtype=np.int32)
    s = torch.from_numpy(src).to(DEV)
    ix = torch.from_numpy(idx).to(DEV)
    got = torch.full((6, 3), -5.0, device=DEV)
    om.gather_rows(s, ix, out=got)
    dst = torch.full((10, 3), -5.0, device=DEV)
    om.scatter_rows(got, ix, dst)
    torch.cuda.synchronize()
    want = np.full((6, 3), -5.0, dtype=np.float32)
    for i, r in enumerate(idx):
        if 0 <= r < 10:
            want[i] = src[r]
    assert np.array_equal(got.cpu().numpy(), want)
    want_back = np.full((10, 3), -5.0, dtype=np.float32)
    for r in (2, 9, 0):
        want_back[r] = src[r]
    assert np.array_equal(dst.cpu().numpy(), want_back)


def test_order_and_rows_empty(tiny):
    sc, scene, t, box = tiny
    e = torch.empty((0, 3), dtype=torch.float32, device=DEV)
    order, os_, ds_ = om.order_rays(scene, e, e.clone())
    assert order.numel() == 0
    assert om.gather_rows(e, order).shape == (0, 3)
