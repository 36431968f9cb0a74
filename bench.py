"""Throughput of the occupancy-plane ray marcher on one MI355X.

One step = one pass of the whole hot path over one batch: sample placement
inside the occupancy plane, feature gather, activations, compositing and the
deferred MLP (om_render), for every ray of the batch.  The default workload
is the 1920x1080 oblique render of the 1024x1024x128 grid + 4096^2/4096x512
planes scene with a 256x256 occupancy plane and 200 buildings (float32).

Prints ONE JSON line.  `value` is Mrays/s of the float32 forward render;
`forms` adds the other configurations (tiny scene, row ray order, bfloat16
and 8-bit storage, training steps, eight 4K images, towers, high altitude,
sparse blocks).  `roofline` is for the dominant kernel (the float32 march):
HBM bytes it must move at least (every feature row it reads, once, plus rays
in and results out) against the 8 TB/s peak, beside the DRAM bytes that
rocprofv3 counted; the gather's own ceiling (`roofline.l1`) is the rate at
which the vector memory path returns 16-byte lane loads from cache-resident
data, calibrated live with a kernel of the same load shape.  The float64 CPU
oracle is timed on a crop of the same image (`cpu_baseline`), and the same
oracle crops give each precision form its error against float64.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BG = (0.25, 0.5, 0.75)
ALL_FORMS = ("tiny_fp32_render,fp32_render_row_order,fp32_render_row_order_ordered,fp32_render_ert,bf16_render,"
             "u8_render,sparse_render,fp32_fwd_bwd,fp32_fwd_bwd_ordered,fp32_fwd_bwd_soft_occ,fp32_fwd_bwd_enc_smooth,"
             "bf16_render_4k_x8,high_altitude_mips,towers_bf16_fwd_bwd,towers_bf16_fwd_bwd_ordered")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--t-term", type=float, default=0.0)
    ap.add_argument("--no-forms", action="store_true", help="skip every form")
    ap.add_argument("--forms", default=ALL_FORMS, help="comma-separated subset of forms to run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--crop", type=int, default=256, help="side of the centre crop rendered by the CPU oracle")
    ap.add_argument("--order", default=None, help="ray issue order of the headline image (row | tile4 | morton)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 1 GiB device copy (HBM byte-counter calibration under rocprofv3)")
    return ap.parse_args()


# The source files each kernel family is compiled from; a committed counter
# figure is used only while the hash of its family's files is unchanged.
KERNEL_SOURCES = {
    "fwd": ("omerf_device.h", "march_fwd.hip"),
    "bwd": ("omerf_device.h", "bwd_device.h", "march_bwd.hip"),
    "mlp": ("omerf_device.h", "mlp.hip"),
}


def kernel_source_hash(family: str = "fwd") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_2404_09531_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counter(kernel: str, workload: str, key: str = "hbm_bytes_per_launch"):
    """A per-launch figure from a committed rocprofv3 counter summary
    (profiles/traffic.json), only if it was taken on the current source of
    the kernel's family."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    e = rec.get(kernel, {}).get(workload)
    if not e or e.get("source_hash") != kernel_source_hash(e.get("family", "fwd")):
        return None
    return e.get(key)


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch (see measured_counter)."""
    return measured_counter(kernel, workload)


def time_stages(step_fns, steps, warmup, torch):
    """Run `steps` steps; each step calls the stage functions in order with
    events recorded between them on the current stream (the stream the
    library launches on).  Returns (total ms, [per-stage mean ms])."""
    for _ in range(warmup):
        for f in step_fns:
            f()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(step_fns) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    for s in range(steps):
        ev[s][0].record()
        for i, f in enumerate(step_fns):
            f()
            ev[s][i + 1].record()
    torch.cuda.synchronize()
    total = ev[0][0].elapsed_time(ev[-1][-1])
    per = [float(np.mean([ev[s][i].elapsed_time(ev[s][i + 1]) for s in range(steps)])) for i in range(len(step_fns))]
    return total, per


def _outputs(torch, n, dev, batch_slots=0):
    """Forward outputs; batch_slots > 0 adds the per-batch w v sums that a
    training forward saves for the backward."""
    out = dict(C=torch.empty((n, 3), device=dev), T=torch.empty((n,), device=dev),
               F=torch.empty((n, 7), device=dev), n_placed=torch.empty((n,), dtype=torch.int32, device=dev),
               n_eval=torch.empty((n,), dtype=torch.int32, device=dev))
    if batch_slots:
        out["batch_wv"] = torch.empty((n, batch_slots, 7), device=dev)
    return out


def _bf16_scene(om, t):
    """bfloat16 shadow of the float32 scene, cast by the library."""
    tb = {k: om.to_bf16(t[k]) for k in ("grid", "plane_xy", "plane_xz", "plane_yz")}
    return om.Scene(tb["grid"], tb["plane_xy"], tb["plane_xz"], tb["plane_yz"], t["occ"], t["mlp"]), tb


# ---------------------------------------------------------------------------
# Rooflines
# ---------------------------------------------------------------------------
def l1_gather_peak(torch, span: int, blocks: int = 8192, iters: int = 64, reps: int = 5) -> dict:
    """Rate (GB/s) at which 16-byte lane loads come back to registers from
    cache-resident data, `span` lanes per contiguous span (calibration
    kernel in libomcalib.so; a 16 KiB buffer read by every block)."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2404_09531_amd", "libomcalib.so"))
    lib.omcalib_l1_gather.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p]
    nvec = 1024
    buf = torch.rand(nvec * 4, device="cuda:0")
    sink = torch.empty(blocks * 256, device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream

    def launch():
        rc = lib.omcalib_l1_gather(buf.data_ptr(), nvec, span, blocks, iters, sink.data_ptr(), st)
        if rc != 0:
            raise RuntimeError(f"omcalib_l1_gather failed ({rc})")

    ms, _ = time_stages([launch], reps, 2, torch)
    nbytes = blocks * 256 * 8 * iters * 16
    return {"span_lanes": span, "GBps": round(nbytes / (ms / reps * 1e-3) / 1e9, 1),
            "kernel": "omcalib_l1_gather (16 KiB buffer, 16-byte lane loads)"}


_ATOMIC_PEAK = {}


def atomic_segment_peak(torch, nbytes: int = 256 << 20, blocks: int = 32768, iters: int = 16, reps: int = 5) -> dict:
    """Rate (G requests/s) at which the device performs float atomics of one
    64-byte segment per 16-lane group, at random segments of a zeroed
    `nbytes` buffer (calibration kernel in libomcalib.so; the backward's
    segment flush has this shape).  The default, 256 MiB of targets, is the
    best case: the rate is flat from 4 to 256 MiB and falls beyond (the
    targets then miss the memory-side cache), so it is the ceiling of the
    unit.  Measured once per process and size."""
    if nbytes in _ATOMIC_PEAK:
        return _ATOMIC_PEAK[nbytes]
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2404_09531_amd", "libomcalib.so"))
    lib.omcalib_atomic_segments.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_void_p]
    nseg = nbytes // 64
    buf = torch.zeros(nseg * 16, device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream

    def launch():
        rc = lib.omcalib_atomic_segments(buf.data_ptr(), nseg, blocks, iters, st)
        if rc != 0:
            raise RuntimeError(f"omcalib_atomic_segments failed ({rc})")

    ms, _ = time_stages([launch], reps, 2, torch)
    del buf
    req = blocks * 16 * iters
    _ATOMIC_PEAK[nbytes] = {"G_requests_per_s": round(req / (ms / reps * 1e-3) / 1e9, 2), "buffer_bytes": nbytes,
                            "kernel": "omcalib_atomic_segments (16 lanes x 4 B per random 64-byte segment)"}
    return _ATOMIC_PEAK[nbytes]


def measured_atomic_requests(kernel: str, workload: str):
    """Float-atomic requests per launch (TCC_ATOMIC_sum) from the committed
    counter summary, only if taken on the current source of the kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        e = json.load(fh).get(kernel, {}).get(workload)
    if not e or e.get("counter_source_hash") != kernel_source_hash(e.get("family", "fwd")):
        return None
    return e.get("counters", {}).get("TCC_ATOMIC_sum")


def rows_read(om, scene, og, dg, n_max, n_eval) -> dict:
    """Feature rows the render reads (om_mark_rows), per source."""
    fl = om.mark_rows(scene, og, dg, n_max, n_eval=n_eval)
    return {k: int(v.count_nonzero().item()) for k, v in fl.items()}


def hbm_roofline(kernel, workload, kernel_ms, min_bytes, l1_bytes=None, l1_peak=None):
    """HBM roofline of one kernel launch: `min_bytes` (the bytes it must
    move at least) per launch time against the 8 TB/s peak, the measured
    DRAM bytes (rocprofv3, committed summary for this kernel source) beside
    it, and optionally the gather ceiling (algorithmic bytes returned to
    registers against the calibrated cache-resident rate).  `kernel` may be
    a tuple of kernels launched back to back by one timed call (the
    backward's MLP stage and march): their DRAM bytes add up."""
    kernels = kernel if isinstance(kernel, tuple) else (kernel,)
    parts = [measured_traffic(k, workload) for k in kernels]
    traffic = None if any(p is None for p in parts) else sum(parts)
    kernel = " + ".join(kernels)
    s = kernel_ms * 1e-3
    r = {"bound": "hbm", "achieved": round(min_bytes / s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(min_bytes / s / 1e9 / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
         "kernel_ms": round(kernel_ms, 4), "compulsory_bytes_per_launch": int(min_bytes),
         "dram_GBps": None if traffic is None else round(traffic / s / 1e9, 1),
         "dram_frac": None if traffic is None else round(traffic / s / 1e9 / HBM_PEAK_GBS, 4)}
    if l1_bytes is not None:
        r["l1"] = {"achieved": round(l1_bytes / s / 1e9, 1), "peak": l1_peak["GBps"], "unit": "GB/s",
                   "frac": round(l1_bytes / s / 1e9 / l1_peak["GBps"], 4), "bytes_per_launch": int(l1_bytes),
                   "calibration": l1_peak}
    return r


def _psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return round(10.0 * np.log10(1.0 / max(mse, 1e-30)), 2)


# ---------------------------------------------------------------------------
# Forms
# ---------------------------------------------------------------------------
def form_tiny(om, scenegen, torch, a):
    """The tiny configuration (64x64x16 grid, 256^2 planes, 32^2 occupancy,
    4096 oblique rays, n_max 64): float32 render.  Its ~5 MiB scene is
    cache-resident, so no HBM figure is claimed."""
    dev = torch.device("cuda:0")
    cfg, rec = scenegen.workload("tiny")
    sc = scenegen.make_scene(cfg)
    o, d = scenegen.make_rays(rec)
    t = {k: torch.from_numpy(sc[k]).to(dev) for k in ("grid", "plane_xy", "plane_xz", "plane_yz", "occ", "mlp")}
    scene = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], t["mlp"])
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    n = o.shape[0]
    out = _outputs(torch, n, dev)
    kw = dict(n_max=rec["n_max"], c_bg=BG)
    m = lambda: om.render_into(scene, og, dg, out, stage="march", **kw)  # noqa: E731
    ml = lambda: om.render_into(scene, og, dg, out, stage="mlp", **kw)  # noqa: E731
    steps = max(a.steps, 50)
    tot, (m_ms, l_ms) = time_stages([m, ml], steps, a.warmup, torch)
    ms = tot / steps
    s = int(out["n_eval"].sum().item())
    return {"workload": "tiny: grid 64x64x16, planes 256^2/256x64/256x64, occupancy 32^2, 4096 rays, n_max 64",
            "rays": n, "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
            "march_ms": round(m_ms, 4), "mlp_ms": round(l_ms, 4), "samples_per_ray": round(s / n, 1),
            "note": "scene cache-resident; launch-latency bound at this size, no HBM claim"}


def form_row_order(om, scenegen, torch, scene, kw, a, l1_peak):
    """The headline frame with its rays in row-major pixel order (what a
    caller that does not reorder its rays gets) instead of Morton order."""
    dev = torch.device("cuda:0")
    _, rec = scenegen.workload("oblique-1080p")
    o, d = scenegen.make_rays(dict(rec, order="row"))
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    n = o.shape[0]
    out = _outputs(torch, n, dev)
    m = lambda: om.render_into(scene, og, dg, out, stage="march", **kw)  # noqa: E731
    ml = lambda: om.render_into(scene, og, dg, out, stage="mlp", **kw)  # noqa: E731
    tot, (m_ms, l_ms) = time_stages([m, ml], a.steps, a.warmup, torch)
    ms = tot / a.steps
    s = int(out["n_eval"].sum().item())
    return {"workload": "oblique-1080p, row-major ray order", "rays": n,
            "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4), "march_ms": round(m_ms, 4),
            "l1_frac": round((s * 640 + n * 64) / (m_ms * 1e-3) / 1e9 / l1_peak["GBps"], 4)}


def form_row_order_ordered(om, scenegen, torch, scene, kw, a):
    """The row-major headline frame ordered by the library first
    (om_order_rays: rays by where they cross the scene), rendered in that
    order, and its colours scattered back into pixel order (om_scatter_rows);
    all three inside the timed step."""
    dev = torch.device("cuda:0")
    _, rec = scenegen.workload("oblique-1080p")
    o, d = scenegen.make_rays(dict(rec, order="row"))
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    n = o.shape[0]
    out = _outputs(torch, n, dev)
    bufs = (torch.empty((n,), dtype=torch.int32, device=dev), torch.empty_like(og), torch.empty_like(dg))
    ws = torch.empty((om.order_rays_workspace_size(n),), dtype=torch.uint8, device=dev)
    image = torch.empty((n, 3), dtype=torch.float32, device=dev)
    order = lambda: om.order_rays(scene, og, dg, out=bufs, workspace=ws)  # noqa: E731
    m = lambda: om.render_into(scene, bufs[1], bufs[2], out, stage="march", **kw)  # noqa: E731
    ml = lambda: om.render_into(scene, bufs[1], bufs[2], out, stage="mlp", **kw)  # noqa: E731
    back = lambda: om.scatter_rows(out["C"], bufs[0], image)  # noqa: E731
    tot, (o_ms, m_ms, l_ms, b_ms) = time_stages([order, m, ml, back], a.steps, a.warmup, torch)
    ms = tot / a.steps
    plain = _outputs(torch, n, dev)
    om.render_into(scene, og, dg, plain, **kw)
    same = bool(torch.equal(image, plain["C"]))
    return {"workload": "oblique-1080p, row-major ray order, ordered by om_order_rays", "rays": n,
            "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
            "order_ms": round(o_ms, 4), "march_ms": round(m_ms, 4), "mlp_ms": round(l_ms, 4),
            "scatter_ms": round(b_ms, 4), "image_bit_identical_to_row_order_render": same}


def form_bf16_render(om, torch, t, og, dg, out, kw, n, a, rows, l1_peak, crop_idx, crops):
    """bfloat16 grid/planes + bfloat16 MFMA MLP on the same 1080p image."""
    scene_b, tb = _bf16_scene(om, t)
    outb = {k: torch.empty_like(v) for k, v in out.items()}
    mb = lambda: om.render_into(scene_b, og, dg, outb, stage="march", **kw)  # noqa: E731
    lb = lambda: om.render_into(scene_b, og, dg, outb, stage="mlp", **kw)  # noqa: E731
    tot, (mb_ms, lb_ms) = time_stages([mb, lb], a.steps, a.warmup, torch)
    ms = tot / a.steps
    sb = int(outb["n_eval"].sum().item())
    crops["bf16_render"] = outb["C"][crop_idx].double().cpu().numpy()
    return {"Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
            "march_ms": round(mb_ms, 4), "mlp_ms": round(lb_ms, 4),
            "roofline": hbm_roofline("k_march_fwd_lane<GatherBF16>", "oblique-1080p", mb_ms,
                                     sum(rows.values()) * 16 + n * 64, sb * 320 + n * 64, l1_peak),
            "psnr_vs_fp32_render_db": _psnr(outb["C"].cpu().numpy(), out["C"].cpu().numpy()),
            "max_abs_vs_fp32_render": float((outb["C"] - out["C"]).abs().max().item())}


def form_fp32_render_ert(om, torch, scene, og, dg, out, kw, n, a, t_term=1e-4):
    """The headline float32 frame with early ray termination at T < 1e-4
    (not in the paper; reported beside the t_term = 0 value)."""
    kw = dict(kw, t_term=t_term)
    oute = {k: torch.empty_like(v) for k, v in out.items()}
    me = lambda: om.render_into(scene, og, dg, oute, stage="march", **kw)  # noqa: E731
    le = lambda: om.render_into(scene, og, dg, oute, stage="mlp", **kw)  # noqa: E731
    tot, (me_ms, le_ms) = time_stages([me, le], a.steps, a.warmup, torch)
    ms = tot / a.steps
    se = int(oute["n_eval"].sum().item())
    return {"t_term": t_term, "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
            "march_ms": round(me_ms, 4), "mlp_ms": round(le_ms, 4), "samples_per_ray": round(se / n, 2),
            "max_abs_vs_t_term_0": float((oute["C"] - out["C"]).abs().max().item())}


def form_sparse_render(om, torch, t, scene, og, dg, out, kw, n, a, shift=3):
    """Sparse voxel blocks of 2^shift cells (Sec. 4.4: the baked grid kept as
    sparse blocks chosen from the occupancy plane) on the same 1080p frame,
    float32 and 8-bit; the renders equal the dense ones bit for bit."""
    res = {}
    codes, quant = om.quantize_features(t)
    scene_q = om.Scene(codes["grid"], codes["plane_xy"], codes["plane_xz"], codes["plane_yz"], t["occ"], t["mlp"],
                       quant=quant)
    for name, sc_d, q, ref_out in (("f32", scene, None, out), ("u8", scene_q, quant, None)):
        atlas, sg = om.sparse_grid(sc_d, shift)
        src = sc_d.tensors
        sp = om.Scene(atlas, src["plane_xy"], src["plane_xz"], src["plane_yz"], t["occ"], t["mlp"], quant=q,
                      sparse=sg)
        if ref_out is None:
            ref_out = {k: torch.empty_like(v) for k, v in out.items()}
            om.render_into(sc_d, og, dg, ref_out, **kw)
        outs = {k: torch.empty_like(v) for k, v in out.items()}
        ms_ = lambda: om.render_into(sp, og, dg, outs, stage="march", **kw)  # noqa: E731
        ls_ = lambda: om.render_into(sp, og, dg, outs, stage="mlp", **kw)  # noqa: E731
        tot, (m_ms, l_ms) = time_stages([ms_, ls_], a.steps, a.warmup, torch)
        ms = tot / a.steps
        res[name] = {"Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
                     "march_ms": round(m_ms, 4), "blocks_kept": sg.n_blocks, "blocks_total": sg.blocks.numel(),
                     "grid_bytes_sparse": atlas.numel() * atlas.element_size(),
                     "grid_bytes_dense": src["grid"].numel() * src["grid"].element_size(),
                     "equal_to_dense": bool(all(torch.equal(outs[k], ref_out[k]) for k in ("C", "T", "F")))}
        del atlas, sp
    res["block_cells"] = 1 << shift
    return res


def form_u8_render(om, torch, t, og, dg, out, kw, n, a, rows, l1_peak, crop_idx, crops):
    """8-bit features (Sec. 4.4: the baked, deployed precision) baked on the
    GPU from the float32 scene, float32 MLP, the same 1080p frame."""
    codes, quant = om.quantize_features(t)
    scene_q = om.Scene(codes["grid"], codes["plane_xy"], codes["plane_xz"], codes["plane_yz"], t["occ"], t["mlp"],
                       quant=quant)
    outq = {k: torch.empty_like(v) for k, v in out.items()}
    mq = lambda: om.render_into(scene_q, og, dg, outq, stage="march", **kw)  # noqa: E731
    lq = lambda: om.render_into(scene_q, og, dg, outq, stage="mlp", **kw)  # noqa: E731
    tot, (mq_ms, lq_ms) = time_stages([mq, lq], a.steps, a.warmup, torch)
    ms = tot / a.steps
    sq = int(outq["n_eval"].sum().item())
    crops["u8_render"] = outq["C"][crop_idx].double().cpu().numpy()
    return {"Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
            "march_ms": round(mq_ms, 4), "mlp_ms": round(lq_ms, 4),
            "roofline": hbm_roofline("k_march_fwd_lane<GatherU8>", "oblique-1080p", mq_ms,
                                     sum(rows.values()) * 8 + n * 64, sq * 160 + n * 64, l1_peak),
            "psnr_vs_fp32_render_db": _psnr(outq["C"].cpu().numpy(), out["C"].cpu().numpy()),
            "max_abs_vs_fp32_render": float((outq["C"] - out["C"]).abs().max().item()),
            "feature_bytes": int(sum(c.numel() for c in codes.values()))}


def _train_rays(scenegen, torch, name, dev):
    _, rec = scenegen.workload(name)
    o, d = scenegen.make_rays(rec)
    return torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev), rec


def _train_rooflines(om, torch, scene, og, dg, out, kw, f_ms, b_ms, fwd_kernel, bwd_kernel, workload, row_bytes):
    """Forward and backward rooflines of a training step: each must read
    every row its samples touch once; the backward also reads and writes
    their float32 gradient rows once (64 B per row: read-modify-write).
    The backward also reports its float-atomic requests per second (the
    march backward's request count from the committed counters, over the
    time of the backward call) against the calibrated segment-atomic rate:
    the unit that bounds it."""
    n = og.shape[0]
    rows = rows_read(om, scene, og, dg, kw["n_max"], out["n_eval"])
    nr = sum(rows.values())
    slots = om.batch_slots(kw["n_max"])
    ne = out["n_eval"].long()
    live_slots = int(((ne + om.BATCH - 1) // om.BATCH).sum().item())
    fwd_min = nr * row_bytes + n * 64 + live_slots * 28  # rows + rays/outputs + per-batch sums
    bwd_min = nr * (row_bytes + 64) + n * (24 + 52 + 12) + live_slots * 28
    del slots
    bwd = hbm_roofline(bwd_kernel, workload, b_ms, bwd_min)
    march = bwd_kernel[-1] if isinstance(bwd_kernel, tuple) else bwd_kernel
    req = measured_atomic_requests(march, workload)
    if req is not None:
        cal = dict(atomic_segment_peak(torch))
        # context: the same pattern over 1 GiB of targets, about the span a
        # training step's gradient rows cover
        cal["G_requests_per_s_1GiB_targets"] = atomic_segment_peak(torch, nbytes=1 << 30)["G_requests_per_s"]
        got = req / (b_ms * 1e-3) / 1e9
        bwd["atomics"] = {"achieved": round(got, 2), "peak": cal["G_requests_per_s"], "unit": "G requests/s",
                          "frac": round(got / cal["G_requests_per_s"], 4), "requests_per_launch": int(req),
                          "calibration": cal}
    return {"fwd": hbm_roofline(fwd_kernel, workload, f_ms, fwd_min), "bwd": bwd, "rows_touched": rows}


def form_fp32_fwd_bwd(om, scenegen, torch, scene, t, kw, a, occ_eps=0.0):
    """float32 forward + L2 loss gradient + backward on 2^18 rays of 16 cameras
    (with occ_eps > 0: the soft occupancy of Eq. 6/8 and the gradient of
    the occupancy bounds)."""
    kw = dict(kw, occ_eps=occ_eps)
    dev = t["grid"].device
    o2g, d2g, _ = _train_rays(scenegen, torch, "train-2^18", dev)
    n2 = o2g.shape[0]
    out2 = _outputs(torch, n2, dev, om.batch_slots(kw["n_max"]))
    om.render_into(scene, o2g, d2g, out2, **kw)
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    target = (out2["C"] + 0.05 * torch.randn(out2["C"].shape, device=dev, generator=g)).contiguous()
    keys = ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp") + (("occ",) if occ_eps > 0 else ())
    grads = {k: torch.zeros(t[k].shape, device=dev) for k in keys}
    dC = torch.empty_like(out2["C"])
    fwd = lambda: om.render_into(scene, o2g, d2g, out2, **kw)  # noqa: E731
    lossg = lambda: om.l2_loss_grad(out2["C"], target, dL_dC=dC, with_loss=False)  # noqa: E731
    ws = torch.empty((om.backward_workspace_size(n2),), dtype=torch.uint8, device=dev)
    bwd = lambda: om.render_backward(scene, o2g, d2g, out2, dC, grads, workspace=ws, **kw)  # noqa: E731
    steps = max(3, a.steps // 2)
    tot, (f_ms, l_ms, b_ms) = time_stages([fwd, lossg, bwd], steps, a.warmup, torch)
    ms = tot / steps
    s2 = int(out2["n_eval"].sum().item())
    res = {"workload": "2^18 rays, 16 cameras 1920x1080, oblique scene" + (f", soft occupancy eps {occ_eps}"
                                                                            if occ_eps > 0 else ""), "rays": n2,
           "Mrays_per_s": round(n2 / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4),
           "fwd_ms": round(f_ms, 4), "loss_ms": round(l_ms, 4), "bwd_ms": round(b_ms, 4),
           "samples_per_ray": round(s2 / n2, 1), "targets": "forward colours + N(0, 0.05), seeded",
           "bwd_Msamples_per_s": round(s2 / (b_ms * 1e-3) / 1e6, 1)}
    if occ_eps == 0:
        res["roofline"] = _train_rooflines(om, torch, scene, o2g, d2g, out2, kw, f_ms, b_ms, "k_march_fwd_f32q<true>",
                                           ("k_mlp_bwd<10>", "k_march_bwd<F32Store>"), "train-2^18", 32)
    return res


def form_fp32_fwd_bwd_ordered(om, scenegen, torch, scene, t, kw, a):
    """The float32 training step of form_fp32_fwd_bwd with the batch ordered
    by the library first (om_order_rays, and the targets brought along with
    om_gather_rows), inside the timed step.  The loss and gradients are those
    of the same ray set: only the order of the float atomics differs."""
    dev = t["grid"].device
    o2g, d2g, _ = _train_rays(scenegen, torch, "train-2^18", dev)
    n2 = o2g.shape[0]
    out2 = _outputs(torch, n2, dev, om.batch_slots(kw["n_max"]))
    om.render_into(scene, o2g, d2g, out2, **kw)
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    target = (out2["C"] + 0.05 * torch.randn(out2["C"].shape, device=dev, generator=g)).contiguous()
    bufs = (torch.empty((n2,), dtype=torch.int32, device=dev), torch.empty_like(o2g), torch.empty_like(d2g))
    ows = torch.empty((om.order_rays_workspace_size(n2),), dtype=torch.uint8, device=dev)
    tgt = torch.empty_like(target)
    grads = {k: torch.zeros(t[k].shape, device=dev) for k in ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp")}
    dC = torch.empty_like(out2["C"])
    ws = torch.empty((om.backward_workspace_size(n2),), dtype=torch.uint8, device=dev)

    def order():
        om.order_rays(scene, o2g, d2g, out=bufs, workspace=ows)
        om.gather_rows(target, bufs[0], out=tgt)

    fwd = lambda: om.render_into(scene, bufs[1], bufs[2], out2, **kw)  # noqa: E731
    lossg = lambda: om.l2_loss_grad(out2["C"], tgt, dL_dC=dC, with_loss=False)  # noqa: E731
    bwd = lambda: om.render_backward(scene, bufs[1], bufs[2], out2, dC, grads, workspace=ws, **kw)  # noqa: E731
    steps = max(3, a.steps // 2)
    tot, (o_ms, f_ms, l_ms, b_ms) = time_stages([order, fwd, lossg, bwd], steps, a.warmup, torch)
    ms = tot / steps
    return {"workload": "2^18 rays, 16 cameras 1920x1080, oblique scene, ordered by om_order_rays", "rays": n2,
            "Mrays_per_s": round(n2 / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4),
            "order_ms": round(o_ms, 4), "fwd_ms": round(f_ms, 4), "loss_ms": round(l_ms, 4),
            "bwd_ms": round(b_ms, 4)}


SMOOTH_RAYS = 1 << 10  # directions per step in the view-smoothness loss
SMOOTH_P = 4  # perturbed directions per ray


def form_fp32_enc_smooth(om, scenegen, torch, t, kw, a):
    """The training step of form_fp32_fwd_bwd with the four-frequency
    direction encoding (34-input deferred MLP) and the view-smoothness loss
    of Eq. 9-10 on the first 2^10 rays of the batch (4 Gaussian
    perturbations each, Sigma = 0.3 I): forward, L2 gradient, smoothness loss
    + dL/dF, backward with dL/dF."""
    dev = t["grid"].device
    mlp = torch.from_numpy(scenegen.mlp_params(4, seed=7)).to(dev)
    scene = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], mlp)
    o2g, d2g, _ = _train_rays(scenegen, torch, "train-2^18", dev)
    n2 = o2g.shape[0]
    out2 = _outputs(torch, n2, dev, om.batch_slots(kw["n_max"]))
    om.render_into(scene, o2g, d2g, out2, **kw)
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    target = (out2["C"] + 0.05 * torch.randn(out2["C"].shape, device=dev, generator=g)).contiguous()
    pert = torch.from_numpy(scenegen.view_perturbations(SMOOTH_RAYS, SMOOTH_P, seed=4)).to(dev)
    grads = {k: torch.zeros(t[k].shape, device=dev) for k in ("grid", "plane_xy", "plane_xz", "plane_yz")}
    grads["mlp"] = torch.zeros_like(mlp)
    dC = torch.empty_like(out2["C"])
    dF = torch.zeros_like(out2["F"])
    Fs, ds, dFs = out2["F"][:SMOOTH_RAYS], d2g[:SMOOTH_RAYS], dF[:SMOOTH_RAYS]
    w = 0.1
    fwd = lambda: om.render_into(scene, o2g, d2g, out2, **kw)  # noqa: E731
    lossg = lambda: om.l2_loss_grad(out2["C"], target, dL_dC=dC, with_loss=False)  # noqa: E731
    smooth = lambda: om.smooth_loss(scene, Fs, ds, pert, w, dL_dF=dFs, grad_mlp=grads["mlp"],  # noqa: E731
                                    with_loss=False)
    ws = torch.empty((om.backward_workspace_size(n2),), dtype=torch.uint8, device=dev)
    bwd = lambda: om.render_backward(scene, o2g, d2g, out2, dC, grads, dL_dF=dF, workspace=ws, **kw)  # noqa: E731
    steps = max(3, a.steps // 2)
    tot, (f_ms, l_ms, s_ms, b_ms) = time_stages([fwd, lossg, smooth, bwd], steps, a.warmup, torch)
    ms = tot / steps
    return {"workload": "2^18 rays, 16 cameras 1920x1080, oblique scene, 34-input MLP, "
                        f"smoothness on {SMOOTH_RAYS} rays x {SMOOTH_P} perturbations", "rays": n2,
            "Mrays_per_s": round(n2 / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4),
            "fwd_ms": round(f_ms, 4), "loss_ms": round(l_ms, 4), "smooth_ms": round(s_ms, 4),
            "bwd_ms": round(b_ms, 4)}


def form_bf16_4k(om, scenegen, torch, t, kw, a, l1_peak, crops):
    """bfloat16 render of eight 3840x2160 images from seeded oblique cameras,
    with the MFMA utilisation of the bfloat16 deferred MLP."""
    dev = t["grid"].device
    cams = scenegen.random_cameras(8, seed=3)
    W, H = 3840, 2160
    n = 8 * W * H
    og = torch.empty((n, 3), device=dev)
    dg = torch.empty((n, 3), device=dev)
    px = scenegen.pixel_order(W, H, "morton")
    for i, (p, y, aim) in enumerate(cams):
        o, d = scenegen.camera_rays(W, H, p, y, aim, pixels=px)
        og[i * W * H:(i + 1) * W * H] = torch.from_numpy(o).to(dev)
        dg[i * W * H:(i + 1) * W * H] = torch.from_numpy(d).to(dev)
    scene_b, tb = _bf16_scene(om, t)
    outb = _outputs(torch, n, dev)
    mb = lambda: om.render_into(scene_b, og, dg, outb, stage="march", **kw)  # noqa: E731
    lb = lambda: om.render_into(scene_b, og, dg, outb, stage="mlp", **kw)  # noqa: E731
    steps = max(2, a.steps // 5)
    tot, (mb_ms, lb_ms) = time_stages([mb, lb], steps, 1, torch)
    ms = tot / steps
    sb = int(outb["n_eval"].sum().item())
    # centre 256x256 crop of image 0 (its rays, through the Morton order)
    c = 256
    pix = np.array([(H // 2 - c // 2 + j) * W + (W // 2 - c // 2 + i) for j in range(c) for i in range(c)])
    inv = np.empty(W * H, dtype=np.int64)
    inv[px] = np.arange(W * H)
    ci = torch.from_numpy(inv[pix]).to(dev)
    crops["bf16_render_4k_x8"] = (outb["C"][ci].double().cpu().numpy(), og[ci].cpu().numpy(), dg[ci].cpu().numpy())
    mfma_busy = measured_counter("k_mlp_bf16<10>", "bf16-4k-x8", "mfma_busy_frac")
    mlp_flop_exec = n * 1536  # three 16x16x16 MFMA tiles per 16 rays, layer 1 zero-padded to 16 inputs
    return {"workload": "8 x 3840x2160, pitch U[30,60] deg, Morton ray order", "rays": n,
            "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 3),
            "march_ms": round(mb_ms, 3), "mlp_ms": round(lb_ms, 3), "samples_per_ray": round(sb / n, 1),
            "Msamples_per_s": round(sb / (ms * 1e-3) / 1e6, 1),
            "l1_frac": round((sb * 320 + n * 64) / (mb_ms * 1e-3) / 1e9 / l1_peak["GBps"], 4),
            "mlp_mfma": {"kernel": "k_mlp_bf16<10>", "bound": "mfma", "unit": "TFLOP/s",
                         "achieved": round(mlp_flop_exec / (lb_ms * 1e-3) / 1e12, 2), "peak": 2500.0,
                         "frac": round(mlp_flop_exec / (lb_ms * 1e-3) / 1e12 / 2500.0, 4),
                         "useful_flop_per_ray": 928, "executed_flop_per_ray": 1536,
                         "mfma_busy_frac_counter": mfma_busy,
                         "hbm_GBps": round(n * 52 / (lb_ms * 1e-3) / 1e9, 1),
                         "hbm_frac": round(n * 52 / (lb_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def form_towers(om, scenegen, torch, a, ordered=False):
    """Uneven rays: 512^2 occupancy with 10% towers, 2^20 rays of 64 cameras,
    n_max 512; bfloat16 storage, float32 master gradients.  ordered=True:
    the batch is ordered by om_order_rays (targets gathered along) inside
    the timed step."""
    dev = torch.device("cuda:0")
    cfg, rec = scenegen.workload("towers-2^20")
    sc = scenegen.make_scene(cfg)
    o, d = scenegen.make_rays(rec)
    n = o.shape[0]
    t = {k: torch.from_numpy(sc[k]).to(dev) for k in ("grid", "plane_xy", "plane_xz", "plane_yz", "occ", "mlp")}
    del sc
    scene_b, tb = _bf16_scene(om, t)
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    kw = dict(n_max=rec["n_max"], c_bg=BG)
    out = _outputs(torch, n, dev, om.batch_slots(kw["n_max"]))
    om.render_into(scene_b, og, dg, out, **kw)
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    target = (out["C"] + 0.05 * torch.randn(out["C"].shape, device=dev, generator=g)).contiguous()
    grads = {k: torch.zeros(t[k].shape, device=dev) for k in ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp")}
    dC = torch.empty_like(out["C"])
    fwd = lambda: om.render_into(scene_b, og, dg, out, **kw)  # noqa: E731
    lossg = lambda: om.l2_loss_grad(out["C"], target, dL_dC=dC, with_loss=False)  # noqa: E731
    ws = torch.empty((om.backward_workspace_size(n),), dtype=torch.uint8, device=dev)
    bwd = lambda: om.render_backward(scene_b, og, dg, out, dC, grads, workspace=ws, **kw)  # noqa: E731
    steps = max(3, a.steps // 4)
    if ordered:
        bufs = (torch.empty((n,), dtype=torch.int32, device=dev), torch.empty_like(og), torch.empty_like(dg))
        ows = torch.empty((om.order_rays_workspace_size(n),), dtype=torch.uint8, device=dev)
        tgt = torch.empty_like(target)

        def order():
            om.order_rays(scene_b, og, dg, out=bufs, workspace=ows)
            om.gather_rows(target, bufs[0], out=tgt)

        fwd = lambda: om.render_into(scene_b, bufs[1], bufs[2], out, **kw)  # noqa: E731
        lossg = lambda: om.l2_loss_grad(out["C"], tgt, dL_dC=dC, with_loss=False)  # noqa: E731
        bwd = lambda: om.render_backward(scene_b, bufs[1], bufs[2], out, dC, grads, workspace=ws, **kw)  # noqa: E731
        tot, (o_ms, f_ms, l_ms, b_ms) = time_stages([order, fwd, lossg, bwd], steps, 1, torch)
        ms = tot / steps
        return {"workload": "towers: occupancy 512^2, 10% towers, 2^20 rays of 64 cameras, n_max 512, "
                            "ordered by om_order_rays", "rays": n,
                "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 3),
                "order_ms": round(o_ms, 3), "fwd_ms": round(f_ms, 3), "bwd_ms": round(b_ms, 3)}
    tot, (f_ms, l_ms, b_ms) = time_stages([fwd, lossg, bwd], steps, 1, torch)
    ms = tot / steps
    npl = out["n_placed"].cpu().numpy()
    bins = np.arange(0, 513 + 32, 32)
    hist = np.histogram(npl, bins=bins)[0]
    hist_eval = np.histogram(out["n_eval"].cpu().numpy(), bins=bins)[0]  # equal to n_placed at t_term = 0
    se = int(out["n_eval"].sum().item())
    return {"workload": "towers: occupancy 512^2, 10% towers, 2^20 rays of 64 cameras, n_max 512", "rays": n,
            "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 3),
            "fwd_ms": round(f_ms, 3), "bwd_ms": round(b_ms, 3), "bwd_Msamples_per_s": round(se / (b_ms * 1e-3) / 1e6, 1),
            "roofline": _train_rooflines(om, torch, scene_b, og, dg, out, kw, f_ms, b_ms,
                                         "k_march_fwd_lane<GatherBF16,kBW>", ("k_mlp_bwd<10>", "k_march_bwd<BF16Store>"),
                                         "towers-2^20", 16),
            "samples_per_ray": round(float(npl.mean()), 1), "max_samples": int(npl.max()),
            "n_placed_hist_bins32": hist.tolist(), "n_eval_hist_bins32": hist_eval.tolist()}


def form_high_altitude(om, scenegen, torch, t, a):
    """The oblique scene's tensors over a box four times taller than the
    terrain (z in [0, 1]: the upper three quarters of every column empty),
    one 1920x1080 camera at pitch 45 deg from z = 1.5, Morton order: render
    time without and with the 4-level occupancy pyramid."""
    dev = torch.device("cuda:0")
    scene = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], t["mlp"],
                     box_lo=(-1.0, -1.0, 0.0), box_hi=(1.0, 1.0, 1.0))
    o, d = scenegen.camera_rays(1920, 1080, 45.0, 90.0, origin_z=1.5, pixels=scenegen.pixel_order(1920, 1080, "morton"))
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    n = o.shape[0]
    out = _outputs(torch, n, dev)
    res = {"workload": "oblique scene in a [0,1] z box, 1920x1080, pitch 45 deg from z=1.5", "rays": n}
    for levels in (0, 4):
        scene.build_occupancy_mips(levels)
        ms, _ = time_stages([lambda: om.render_into(scene, og, dg, out, n_max=256, c_bg=BG)], a.steps, a.warmup, torch)
        ms /= a.steps
        res[f"levels{levels}"] = {"ms_per_step": round(ms, 4), "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2)}
    res["samples_per_ray"] = round(float(out["n_eval"].double().mean().item()), 1)
    return res


# ---------------------------------------------------------------------------
# The CPU leg: the float64 oracle on crops of the same images
# ---------------------------------------------------------------------------
def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_leg(sc, o, d, n_max, t_term, crop_px, gpu_crop, crops, forms, c):
    """The oracle (plain float64, never tuned) on the centre crop of the
    headline image in a pool of worker processes on the host's cores, timed;
    then the oracle crops that give each precision form its error against
    float64: bfloat16 and 8-bit against the float32 scene's oracle render
    (storage + arithmetic), and against the oracle of the bfloat16-rounded /
    8-bit-decoded scene (arithmetic only)."""
    import torch as _t

    import oracle
    from oracle.parallel import render_parallel

    prm = oracle.RenderParams(n_max=n_max, c_bg=BG, t_term=t_term)
    oc, dc = o[crop_px], d[crop_px]
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)  # noqa: E731
    ref = render_parallel(sc, oc, dc, prm, log=log)
    dt = ref["seconds"]
    cpu = {"value": round(len(crop_px) / dt / 1e6, 6), "unit": "Mrays/s", "cores": ref["workers"], "kind": "oracle",
           "sample": f"centre {c}x{c} crop of the 1920x1080 image ({len(crop_px)} rays), float64 oracle in "
                     f"{ref['workers']} single-threaded worker processes",
           "cpu_model": cpu_model(), "seconds": round(dt, 2),
           "Msamples_per_s": round(float(ref["n_eval"].sum()) / dt / 1e6, 4),
           "max_abs_gpu_vs_oracle_on_crop": float(np.abs(gpu_crop - ref["C"]).max()),
           "psnr_gpu_vs_oracle_on_crop_db": _psnr(gpu_crop, ref["C"])}
    fid = {}
    if "bf16_render" in crops or "bf16_render_4k_x8" in crops:
        rounded = dict(sc)
        for k in ("grid", "plane_xy", "plane_xz", "plane_yz"):
            rounded[k] = _t.from_numpy(sc[k]).to(_t.bfloat16).float().numpy()
    if "bf16_render" in crops:
        g = crops["bf16_render"]
        rr = render_parallel(rounded, oc, dc, prm, log=log)
        fid["bf16_render"] = {"max_abs_vs_fp64_oracle": float(np.abs(g - ref["C"]).max()),
                              "psnr_vs_fp64_oracle_db": _psnr(g, ref["C"]),
                              "max_abs_vs_oracle_of_rounded_scene": float(np.abs(g - rr["C"]).max()),
                              "psnr_vs_oracle_of_rounded_scene_db": _psnr(g, rr["C"])}
    if "u8_render" in crops:
        g = crops["u8_render"]
        dec = oracle.dequantize_scene(oracle.quantize_scene(sc))
        rq = render_parallel(dec, oc, dc, prm, log=log)
        del dec
        fid["u8_render"] = {"max_abs_vs_fp64_oracle": float(np.abs(g - ref["C"]).max()),
                            "psnr_vs_fp64_oracle_db": _psnr(g, ref["C"]),
                            "max_abs_vs_oracle_of_decoded_scene": float(np.abs(g - rq["C"]).max()),
                            "psnr_vs_oracle_of_decoded_scene_db": _psnr(g, rq["C"])}
    if "bf16_render_4k_x8" in crops:
        g, o4, d4 = crops["bf16_render_4k_x8"]
        r4 = render_parallel(sc, o4, d4, prm, log=log)
        r4r = render_parallel(rounded, o4, d4, prm, log=log)
        fid["bf16_render_4k_x8"] = {"crop": "centre 256x256 of image 0",
                                    "max_abs_vs_fp64_oracle": float(np.abs(g - r4["C"]).max()),
                                    "psnr_vs_fp64_oracle_db": _psnr(g, r4["C"]),
                                    "max_abs_vs_oracle_of_rounded_scene": float(np.abs(g - r4r["C"]).max()),
                                    "psnr_vs_oracle_of_rounded_scene_db": _psnr(g, r4r["C"])}
    for k, v in fid.items():
        forms[k]["fidelity"] = v
    return cpu


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import paper_2404_09531_amd as om
    import scenegen

    dev = torch.device("cuda:0")
    if a.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.time()
    cfg, recipe = scenegen.workload("oblique-1080p")
    if a.order:
        recipe = dict(recipe, order=a.order)
    sc = scenegen.make_scene(cfg)
    o, d = scenegen.make_rays(recipe)
    n = o.shape[0]
    n_max = recipe["n_max"]
    print(f"[bench] scene+rays built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    t = {k: torch.from_numpy(sc[k]).to(dev) for k in ("grid", "plane_xy", "plane_xz", "plane_yz", "occ", "mlp")}
    scene = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], t["mlp"])
    og = torch.from_numpy(o).to(dev)
    dg = torch.from_numpy(d).to(dev)
    out = _outputs(torch, n, dev)
    kw = dict(n_max=n_max, t_term=a.t_term, c_bg=BG)

    march = lambda: om.render_into(scene, og, dg, out, stage="march", **kw)  # noqa: E731
    mlp = lambda: om.render_into(scene, og, dg, out, stage="mlp", **kw)  # noqa: E731
    total_ms, (march_ms, mlp_ms) = time_stages([march, mlp], a.steps, a.warmup, torch)
    ms_step = total_ms / a.steps
    samples = int(out["n_eval"].sum().item())
    mrays = n / (ms_step * 1e-3) / 1e6
    msamples = samples / (ms_step * 1e-3) / 1e6
    print(f"[bench] fp32 render {ms_step:.3f} ms/step (march {march_ms:.3f}, mlp {mlp_ms:.3f}), "
          f"{samples / n:.1f} samples/ray", file=sys.stderr, flush=True)

    # Rooflines of the march kernel (after the timed steps):
    # - HBM: the rows it reads (each at least once) x 32 B + 24 B of rays in
    #   and 40 B of F, T and counts out per ray, per launch time;
    # - gather: 20 corners x 8 channels x 4 B per evaluated sample + 64 B per
    #   ray returned to registers, against the calibrated cache-resident rate.
    rows = rows_read(om, scene, og, dg, n_max, out["n_eval"])
    l1_quad = l1_gather_peak(torch, 4)
    l1_lane = l1_gather_peak(torch, 1)
    roofline = hbm_roofline("k_march_fwd_f32q<false>", "oblique-1080p", march_ms, sum(rows.values()) * 32 + n * 64,
                            samples * 640 + n * 64, l1_quad)
    roofline["rows_read"] = rows
    print(f"[bench] rows read {rows}, gather calibration {l1_quad['GBps']} / {l1_lane['GBps']} GB/s",
          file=sys.stderr, flush=True)

    w, h = recipe["width"], recipe["height"]
    c = a.crop
    pix = np.array([(h // 2 - c // 2 + j) * w + (w // 2 - c // 2 + i) for j in range(c) for i in range(c)])
    inv = np.empty(w * h, dtype=np.int64)
    inv[scenegen.pixel_order(w, h, recipe.get("order", "row"))] = np.arange(w * h)
    px = inv[pix]  # ray indices of the crop's pixels
    crop_idx = torch.from_numpy(px).to(dev)
    gpu_c = out["C"][crop_idx].double().cpu().numpy()

    forms, crops = {}, {}
    want = set() if a.no_forms else set(a.forms.split(","))
    if "tiny_fp32_render" in want:
        forms["tiny_fp32_render"] = form_tiny(om, scenegen, torch, a)
    if "fp32_render_row_order" in want:
        forms["fp32_render_row_order"] = form_row_order(om, scenegen, torch, scene, kw, a, l1_quad)
    if "fp32_render_row_order_ordered" in want:
        forms["fp32_render_row_order_ordered"] = form_row_order_ordered(om, scenegen, torch, scene, kw, a)
    if "bf16_render" in want:
        forms["bf16_render"] = form_bf16_render(om, torch, t, og, dg, out, kw, n, a, rows, l1_lane, crop_idx, crops)
    if "fp32_render_ert" in want:
        forms["fp32_render_ert"] = form_fp32_render_ert(om, torch, scene, og, dg, out, kw, n, a)
    if "sparse_render" in want:
        forms["sparse_render"] = form_sparse_render(om, torch, t, scene, og, dg, out, kw, n, a)
    if "u8_render" in want:
        forms["u8_render"] = form_u8_render(om, torch, t, og, dg, out, kw, n, a, rows, l1_lane, crop_idx, crops)
    if "fp32_fwd_bwd" in want:
        forms["fp32_fwd_bwd"] = form_fp32_fwd_bwd(om, scenegen, torch, scene, t, kw, a)
    if "fp32_fwd_bwd_ordered" in want:
        forms["fp32_fwd_bwd_ordered"] = form_fp32_fwd_bwd_ordered(om, scenegen, torch, scene, t, kw, a)
    if "fp32_fwd_bwd_soft_occ" in want:
        forms["fp32_fwd_bwd_soft_occ"] = form_fp32_fwd_bwd(om, scenegen, torch, scene, t, kw, a, occ_eps=0.01)
    if "fp32_fwd_bwd_enc_smooth" in want:
        forms["fp32_fwd_bwd_enc_smooth"] = form_fp32_enc_smooth(om, scenegen, torch, t, kw, a)
    if "bf16_render_4k_x8" in want:
        forms["bf16_render_4k_x8"] = form_bf16_4k(om, scenegen, torch, t, kw, a, l1_lane, crops)
    if "high_altitude_mips" in want:
        forms["high_altitude_mips"] = form_high_altitude(om, scenegen, torch, t, a)
    if "towers_bf16_fwd_bwd" in want:
        del t, scene, out, og, dg
        torch.cuda.empty_cache()
        forms["towers_bf16_fwd_bwd"] = form_towers(om, scenegen, torch, a)
    if "towers_bf16_fwd_bwd_ordered" in want:
        if "towers_bf16_fwd_bwd" not in want:
            del t, scene, out, og, dg
            torch.cuda.empty_cache()
        forms["towers_bf16_fwd_bwd_ordered"] = form_towers(om, scenegen, torch, a, ordered=True)

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_leg(sc, o, d, n_max, a.t_term, px, gpu_c, crops, forms, c)

    rec = {
        "metric": "Mrays/s render & fwd+bwd (FP32 vs BF16) at stated error; % HBM/MFMA roofline",
        "value": round(mrays, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "oblique-1080p", "rays": n, "grid": list(cfg.grid), "planes": list(cfg.planes),
                   "occupancy": cfg.occ, "buildings": cfg.n_buildings, "n_max": n_max, "t_term": a.t_term,
                   "camera": "pitch 45 deg, yaw 90 deg, 60 deg hfov", "ray_order": recipe.get("order", "row")},
        "Msamples_per_s": round(msamples, 2), "samples_per_ray": round(samples / n, 2),
        "roofline": roofline, "cpu_baseline": cpu, "forms": forms,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
