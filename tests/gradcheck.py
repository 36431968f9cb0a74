"""Gradient parity against the float64 oracle, shared by the GPU tests.

Both sides run the backward for the SAME float32 dL/dC: the oracle's own
L2 gradient 2 (C - C*)/(3n) of its float64 render, rounded to float32 once
(an oracle input, never a GPU value).  The GPU backward then replays its own
forward (F, T, n_eval), and the oracle computes the vector-Jacobian product
of its float64 render with the same dL/dC (oracle_loss_and_grads with
upstream=...).  The forward colours are checked on their own (1e-5), and the
finite-difference tests cover the loss end to end.

Bar per entry: |g - g_oracle| <= 1e-3 |g_oracle| + u (B_e + N_e A_e), the
configurations' 1e-3 relative bar plus the float32 rounding floor of the
entry's own terms (oracle.fp32_bound): A_e is the sum of the absolute values
of the terms the entry adds up, B_e the rounding inside them, N_e their
count.  Untouched entries must stay exactly 0.  Each check logs, per tensor,
the worst |err| / bar, the worst |err| / (u A), and for the entries with
|g| >= 1e-3 max |g| of their tensor: how many of them the float32 floor
resolves to 1e-3 and the worst relative error over those.
"""
import os

import numpy as np

import oracle
from oracle.fp32_bound import U32, compare, floor, gradient_error_scale
from tests.gpu_util import log

SOURCES = ("grid", "plane_xy", "plane_xz", "plane_yz")


def oracle_upstream(sc, o, d, prm, target):
    """(float32 dL/dC [n, 3] of the oracle's L2 loss, the oracle's loss)."""
    C = oracle.oracle_render(sc, o, d, prm, keep_k=False)["C"]
    t = np.asarray(target, dtype=np.float64)
    up = (2.0 * (C - t) / (3.0 * C.shape[0])).astype(np.float32)
    return up, float(np.mean((C - t) ** 2))


def oracle_reference(sc, o, d, prm, up32, smooth=None):
    """Oracle gradient for the float32 upstream dL/dC and its error scale."""
    up = up32.astype(np.float64)
    _, _, ref = oracle.oracle_loss_and_grads(sc, o, d, prm, upstream=up, smooth=smooth)
    scale = gradient_error_scale(sc, o, d, prm, up, smooth=smooth)
    return ref, scale


def check(grads, ref, scale, tag="", keys=None):
    """Assert the per-entry bar (module docstring) for every tensor in
    `keys` (default: the four sources, the MLP and, when the oracle has it,
    the occupancy bounds); grads: numpy arrays of the full tensors."""
    keys = keys or (*SOURCES, "mlp") + (("occ",) if "occ" in ref else ())
    bad = []
    for k in keys:
        s = compare(grads[k], ref[k], scale[k])
        log(f"  [grad {tag}] {k}: worst err/bar {s['worst']:.3f}, worst err/(uA) {s['err_over_uA']:.1f}; "
            f"|g| >= 1e-3 max: {s['big']}, float32-resolved {s['resolved']}, worst rel {s['worst_rel_resolved']:.2e} "
            f"(all of them {s['worst_rel_big']:.2e})")
        if not s["ok"]:
            bad.append((k, s["worst"], s["untouched_zero"]))
            _report_worst(grads[k], ref[k], scale[k], f"{tag} {k}")
    assert not bad, bad


def _report_worst(got, ref, scale, tag, k=5):
    """Log the k entries furthest beyond their bar (row, channel, GPU value,
    oracle value, A, B, N); with OM_GRADCHECK_DUMP set to a directory, also
    save them there as an .npz for analysis on the host."""
    if isinstance(ref, tuple):
        idx, rows = ref
        g = np.asarray(got, dtype=np.float64).reshape(-1, rows.shape[-1])[idx]
        row_ids = np.broadcast_to(np.asarray(idx)[:, None], rows.shape)
    else:
        rows = np.asarray(ref, dtype=np.float64)
        g = np.asarray(got, dtype=np.float64)
        row_ids = np.arange(rows.size)
    A, B, N = scale[-3], scale[-2], np.asarray(scale[-1], dtype=np.float64)
    Nb = np.broadcast_to(N[:, None], A.shape) if A.ndim == 2 else np.broadcast_to(N, A.shape)
    bar = 1e-3 * np.abs(rows) + floor(scale)
    ratio = (np.abs(g - rows) / np.maximum(bar, 1e-300)).reshape(-1)
    order = np.argsort(-ratio)[:k]
    chan = np.broadcast_to(np.arange(rows.shape[-1]) if rows.ndim == 2 else np.zeros(1, int), rows.shape).reshape(-1)
    for i in order:
        log(f"    {tag}: row {int(row_ids.reshape(-1)[i])} ch {int(chan[i])}: gpu {g.reshape(-1)[i]:.6e} "
            f"oracle {rows.reshape(-1)[i]:.6e} A {A.reshape(-1)[i]:.3e} B/A {B.reshape(-1)[i] / max(A.reshape(-1)[i], 1e-300):.1f} "
            f"N {int(Nb.reshape(-1)[i])} err/bar {ratio[i]:.2f}")
    out = os.environ.get("OM_GRADCHECK_DUMP")
    if out:
        os.makedirs(out, exist_ok=True)
        name = "".join(ch if ch.isalnum() else "_" for ch in tag)
        np.savez(os.path.join(out, f"{name}.npz"), row=row_ids.reshape(-1)[order], chan=chan[order],
                 gpu=g.reshape(-1)[order], oracle=rows.reshape(-1)[order], A=A.reshape(-1)[order],
                 B=B.reshape(-1)[order], N=Nb.reshape(-1)[order], u=U32)
