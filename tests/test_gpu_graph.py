"""GPU: the library's launches captured in a HIP graph.

Every entry point launches on the caller's stream and does no host
synchronisation, allocation or memset, so a caller can capture a render or
a whole training step in a graph (torch.cuda.CUDAGraph records the kernels
that the library enqueues on the capturing stream) and replay it.  Each
replay here runs with eager work and synchronisations in between, and is
checked against the eager result: the forward bit for bit (it is
deterministic), the loss bit for bit (a float32 sum in a fixed order) and
the gradients (float atomics in a varying order) to 1e-5 of the largest
entry.
"""
import numpy as np
import pytest
import torch

import paper_2404_09531_amd as om
import scenegen
from tests.gpu_util import log, rays_to, upload_scene

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)
KEYS = ("C", "T", "F", "n_placed", "n_eval")
SOURCES = ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp")


@pytest.fixture(scope="module")
def tiny():
    sc = scenegen.make_scene(scenegen.TINY)
    scene, t = upload_scene(sc)
    return sc, scene, t


def _warm(fn):
    """Warm-up calls on a side stream, as graph capture expects."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()


def test_render_graph_replays_equal_eager(tiny):
    log("test_render_graph_replays_equal_eager")
    sc, scene, t = tiny
    o, d = scenegen.oblique_rays(3000, seed=41)
    og, dg = rays_to(o, d)
    o2, d2 = scenegen.oblique_rays(1000, seed=42)
    og2, dg2 = rays_to(o2, d2)
    kw = dict(n_max=64, c_bg=BG)
    eager = om.render(scene, og, dg, **kw)
    out = {k: torch.full_like(v, -7) for k, v in eager.items()}
    fn = lambda: om.render_into(scene, og, dg, out, **kw)  # noqa: E731
    _warm(fn)
    g = torch.cuda.CUDAGraph()
    for k in out:
        out[k].fill_(-7)
    with torch.cuda.graph(g):
        fn()
    for rep in range(3):
        for k in out:
            out[k].fill_(-7)
        other = om.render(scene, og2, dg2, **kw)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(out[k], eager[k]), (rep, k)
        assert torch.isfinite(other["C"]).all()


def test_training_step_graph_replays_match_eager(tiny):
    log("test_training_step_graph_replays_match_eager")
    sc, scene, t = tiny
    o, d = scenegen.oblique_rays(2048, seed=43)
    og, dg = rays_to(o, d)
    kw = dict(n_max=64, c_bg=BG)
    n = o.shape[0]
    first = om.render(scene, og, dg, **kw)
    gen = torch.Generator(device=og.device)
    gen.manual_seed(5)
    target = (first["C"] + 0.05 * torch.randn(first["C"].shape, device=og.device, generator=gen)).contiguous()
    ws = torch.empty((om.fwd_bwd_l2_workspace_size(n, 64),), dtype=torch.uint8, device=og.device)

    def fresh():
        out = {k: torch.empty_like(v) for k, v in first.items()}
        grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in SOURCES}
        loss = torch.zeros((1,), dtype=torch.float32, device=og.device)
        return out, grads, loss

    out_e, grads_e, loss_e = fresh()
    om.render_fwd_bwd_l2(scene, og, dg, target, out_e, grads_e, workspace=ws, loss=loss_e, **kw)
    torch.cuda.synchronize()

    out, grads, loss = fresh()

    def step():
        for v in grads.values():
            v.zero_()  # a fill kernel, recorded in the graph
        om.render_fwd_bwd_l2(scene, og, dg, target, out, grads, workspace=ws, loss=loss, **kw)

    _warm(step)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    scale = {k: float(grads_e[k].abs().max()) for k in SOURCES}
    assert all(v > 0 for v in scale.values())
    for rep in range(3):
        for v in grads.values():
            v.fill_(123.0)
        loss.fill_(-1.0)
        om.render(scene, og[:100], dg[:100], **kw)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(out[k], out_e[k]), (rep, k)
        assert loss.item() == loss_e.item(), rep  # a float32 sum in a fixed order
        for k in SOURCES:
            err = float((grads[k] - grads_e[k]).abs().max())
            assert err <= 1e-5 * scale[k], (rep, k, err / scale[k])
    log(f"  loss {loss.item():.9e}, 3 replays equal to the eager step")


def test_ordered_render_graph_replays_equal_eager(tiny):
    """The ray order (its histogram cleared by a fill kernel), the render of
    the reordered rays and the scatter back, captured together; between
    replays the same order workspace is used eagerly for other rays, so a
    replay that did not clear it would place rays outside their bins."""
    log("test_ordered_render_graph_replays_equal_eager")
    sc, scene, t = tiny
    o, d = scenegen.oblique_rays(3000, seed=43)
    og, dg = rays_to(o, d)
    o2, d2 = scenegen.oblique_rays(2500, seed=44)
    og2, dg2 = rays_to(o2, d2)
    kw = dict(n_max=64, c_bg=BG)
    eager = om.render(scene, og, dg, **kw)
    n = og.shape[0]
    ws = torch.empty((om.order_rays_workspace_size(n),), dtype=torch.uint8, device=og.device)
    bufs = (torch.empty((n,), dtype=torch.int32, device=og.device), torch.empty_like(og), torch.empty_like(dg))
    out = {k: torch.empty_like(v) for k, v in eager.items()}
    image = torch.full_like(eager["C"], -7)

    def fn():
        om.order_rays(scene, og, dg, out=bufs, workspace=ws)
        om.render_into(scene, bufs[1], bufs[2], out, **kw)
        om.scatter_rows(out["C"], bufs[0], image)

    _warm(fn)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for rep in range(3):
        image.fill_(-7)
        om.order_rays(scene, og2, dg2, workspace=ws)  # eager use of the same workspace
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        idx = bufs[0].cpu().numpy()
        assert np.array_equal(np.sort(idx), np.arange(n, dtype=np.int32)), rep
        assert torch.equal(image, eager["C"]), rep
