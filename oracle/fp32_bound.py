"""Float32 error scale of the backward's gradient entries (TEST INFRASTRUCTURE).

The backward of Eq. 1-4 forms every gradient entry e (a grid vertex or plane
texel channel, an MLP parameter, an interval bound of the occupancy plane)
as a sum of per-sample or per-ray terms, and each term is a short product or
sum of float32 values.  The forward error bounds of floating-point products
and sums (Higham, "Accuracy and Stability of Numerical Algorithms", 2nd ed.,
Sec. 3.1 and Sec. 4.2) give, to first order in the unit roundoff
u = 2^-24,

    |g_float32(e) - g(e)| <= u (B_e + N_e A_e)

* A_e: the sum of the absolute values of the terms the entry adds up (not
  the absolute value of their sum, which cancelling terms can make far
  smaller); every float32 addition of the accumulation rounds relative to
  a partial sum bounded by A_e, and there are fewer than N_e of them.
* N_e: the number of terms (evaluated sample x corner incidences for a
  feature entry, rays for an MLP parameter, samples for an interval bound).
* B_e: the rounding inside each term, sum over terms of |term| times rho,
  the relative error coefficient of its factors in units of u, plus the
  propagated rounding of the quantities every term depends on (dL/dC,
  which is formed from a float32 C; the soft occupancy value M).

It is a tolerance helper for the parity tests, not part of the method (the
gradient itself is ``oracle_loss_and_grads``).  All quantities are float64
values of the oracle's forward.

Per sample s of ray r (a_s = tau_s delta, exact optical depth D, weights w
of Eq. 1, activated channels v of Eq. 3):

* terms of dL/dt_0 (through tau and Eq. 1; their signed sum is the
  derivative): delta tau (T_{s+1} M gv_s, sum_{k>s} w_k gv_k, T_n gT) with
  gv = |dL/dF| . v and gT = |dL/dC| . |c_bg|; of dL/dt_c (c = 1..7):
  w |dL/dF_c| v_c (1 - v_c); |dL/dF| is the MLP's backward with every
  weight and local derivative replaced by its absolute value (ReLU masks
  and sigmoid slopes kept), plus |dL/dC| on the diffuse part;
* rho_s = 64 + phi_s + E_s with phi_s = max_c sum_corners w |row_c| (the
  interpolated t of Eq. 2, whose rounding is relative to it, enters
  tau = exp(t_0) and the sigmoids) and E_s = sum_{j<=s} a_j phi_j (T and w
  are exponentials of float32 depth sums); 64 covers the products and short
  sums of one term (16-lane scans, 7-channel dot products);
* rho_mlp = 64 + N_in + rel_F + (N_in + 32 + rel_F) z3a per ray: dot
  products of <= N_in, 16 and 3 terms, the rounding of the float32 F
  (relative rel_F = sum rho_s w v / F), and the re-evaluated sigmoid slope
  g(1 - g), whose pre-activation z3 rounds relative to its absolute-term
  sum z3a;
* dL/dC is an input (the parity tests give both sides the same float32
  dL/dC), so it carries no rounding; |dL/dF| carries the rounding of the
  MLP backward, rho_mlp |dL/dF|, which the per-sample terms propagate;
* the soft occupancy value M = min(((z - z_min)/epsilon)^2, ...) and its
  derivatives round relative to themselves (z and z_min are binary32, so
  z - z_min rounds relative to the difference): inside rho_s;
* the MLP's inputs: F is the float32 render (rel_F above); the view
  direction d is exact; the encoded direction sin(2^k d), cos(2^k d)
  (Sec. 4.2, 2^k d exact in binary32) is evaluated by a float32 sincos
  within 2 ulp, i.e. 2^-22 absolute on values of magnitude <= 1; the
  smoothness term's s = fl32(d + delta) rounds by u |s| per component,
  which the encoding scales by 2^k.  These absolute input errors e_x are
  carried through the absolute weights and the ReLU masks (e_z1 = |W1|
  e_x, e_z2 = |W2| m1 e_z1, e_z3 = |W3| m2 e_z2) and enter rho_mlp as
  max(e_h1 / h1a, e_h2 / h2a) (units of u) and the sigmoid slope as
  e_z3; the float32 cosine similarity of Eq. 10 from the rounded s is
  within 10 u |S| + 4 u of S;
* interpolation weights (Eq. 2): the GPU forms each 1-D fraction f of a
  binary32 coordinate from the exact split of p s (rounded product plus
  its exact remainder), so f and 1 - f carry an ABSOLUTE error of at most
  FRAC_ERR = 2.5 u, not a relative one; a corner weight (a product of one
  factor per axis, each <= 1) then errs by up to FRAC_ERR u omega_c, with
  omega_c the sum over axes of the product of that corner's other-axis
  factors.  A sample lying ~1e-6 of a cell from a vertex plane thus has
  corners whose weights are off by percents.  This enters each term (B
  gains FRAC_ERR omega_c |dL/dt|) and the interpolated t (phi_s gains
  FRAC_ERR sum_axes |dt/df_a|, each slope a sum over corner pairs of the
  other-axis weight times the difference of the pair's rows);
* float32 range: the GPU flushes products below the smallest normal
  binary32 value (2^-126) to zero, so far behind an opaque surface
  (transmittance below ~2^-100) whole terms vanish where the float64
  oracle keeps them.  The factors a term is multiplied by after any of its
  intermediates are bounded by 2^29 in product (tau = exp(t_0) with
  t_0 <= 12, |dL/dF| <= 2^12, delta, weights and activations <= 1), so
  every intermediate of a term of magnitude 2^-80 or more is at least
  2^-109 and none is flushed; a term below 2^-80 is counted as entirely
  uncertain (B gains |term| / u).  Results that stay subnormal round with
  an absolute error of 2^-150 per operation instead of a relative one: the
  floor gains 65 N 2^-150 (a term's ~64 operations and its addition).

Pins (tests/test_oracle_pins.py): A_e >= |g_e| for every entry of every
tensor (tiny scene, soft occupancy, smoothness term, c_bg != 0); a
constant-density ray whose channel-0 gradient cancels exactly keeps a
nonzero A; the counts N_e sum to the number of (evaluated sample, corner)
incidences of each source.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .field import SOURCES
from .placement import cell_index
from .render import RenderParams, _render_chunk, encode_dir, unpack_mlp

U32 = 2.0 ** -24  # unit roundoff of binary32


def _mlp_abs(mlp: np.ndarray, x: np.ndarray):
    """Forward of G keeping what the absolute backward needs: the ReLU masks,
    the absolute-term sums of the hidden layers and of z3, g and g(1 - g)."""
    w1, b1, w2, b2, w3, b3 = [t.numpy() for t in unpack_mlp(torch.from_numpy(np.asarray(mlp, np.float64)))]
    xa = np.abs(x)
    z1 = x @ w1.T + b1
    m1 = z1 > 0
    h1a = m1 * (xa @ np.abs(w1).T + np.abs(b1))
    z2 = np.maximum(z1, 0.0) @ w2.T + b2
    m2 = z2 > 0
    h2a = m2 * (h1a @ np.abs(w2).T + np.abs(b2))
    z3 = np.maximum(z2, 0.0) @ w3.T + b3
    g = 1.0 / (1.0 + np.exp(-z3))
    return dict(w=(w1, w2, w3), xa=xa, m1=m1, m2=m2, h1a=h1a, h2a=h2a, g=g, sg=g * (1.0 - g),
                z3a=h2a @ np.abs(w3).T + np.abs(b3))


def _mlp_abs_backprop(fw: dict, dG: np.ndarray):
    """Backward of G with absolute weights and inputs for upstream
    magnitudes dG [R, 3] >= 0: (dW [R, P] packed like the parameters,
    dx [R, N])."""
    w1, w2, w3 = fw["w"]
    dz3 = dG * fw["sg"]
    dz2 = fw["m2"] * (dz3 @ np.abs(w3))
    dz1 = fw["m1"] * (dz2 @ np.abs(w2))
    r = dG.shape[0]
    parts = [(dz1[:, :, None] * fw["xa"][:, None, :]).reshape(r, -1), dz1,
             (dz2[:, :, None] * fw["h1a"][:, None, :]).reshape(r, -1), dz2,
             (dz3[:, :, None] * fw["h2a"][:, None, :]).reshape(r, -1), dz3]
    return np.concatenate(parts, axis=1), dz1 @ np.abs(w1)


SINCOS_ERR = 2.0 ** -22  # 2 ulp of a float32 value of magnitude <= 1
FRAC_ERR = 2.5           # absolute error of a 1-D interpolation factor, units of u
SUBNORMAL_FLOOR = 65.0 * 2.0 ** -150  # per term: ~64 subnormal roundings plus its addition
TINY_TERM = 2.0 ** -80   # terms below this may be flushed whole (float32 range)


def _axis_factors(p: np.ndarray, scene) -> dict:
    """Per source, the 1-D interpolation factors of Eq. 2 (vertex-aligned,
    as in oracle.field): a list over the source's axes of (1 - f, f) [S]
    each, with corner c taking factor bit a of c on axis a."""
    from .field import corner_weights_1d

    lo = [float(v) for v in scene["box_lo"]]
    hi = [float(v) for v in scene["box_hi"]]
    lz, ly, lx = scene["grid"].shape[:3]
    ny, nx = scene["plane_xy"].shape[:2]
    nz = scene["plane_xz"].shape[0]

    def factors(axis, n):
        _, f = corner_weights_1d(p[:, axis], lo[axis], hi[axis], n)
        return 1.0 - f, f

    return {"grid": [factors(0, lx), factors(1, ly), factors(2, lz)],
            "plane_xy": [factors(0, nx), factors(1, ny)],
            "plane_xz": [factors(0, nx), factors(2, nz)],
            "plane_yz": [factors(1, ny), factors(2, nz)]}


def _other_axis_weight(fac: list, c: int, a: int) -> np.ndarray:
    """Product of corner c's factors on every axis but a."""
    w = np.ones_like(fac[0][0])
    for b, pair in enumerate(fac):
        if b != a:
            w = w * pair[(c >> b) & 1]
    return w


def _other_axis_weights(p: np.ndarray, scene) -> dict:
    """omega [S, corners] per source: for each corner, the sum over the
    interpolation axes of the product of the corner's factors on the other
    axes -- the first-order error of its weight per unit error of every
    1-D factor."""
    out = {}
    for src, fac in _axis_factors(p, scene).items():
        k = len(fac)
        om = np.zeros((p.shape[0], 1 << k))
        for c in range(1 << k):
            for a in range(k):
                om[:, c] += _other_axis_weight(fac, c, a)
        out[src] = om
    return out


def _fraction_slopes(p: np.ndarray, scene, idx_of: dict) -> np.ndarray:
    """sum over sources and axes of |dt/df_a| bounded per channel [S, 8]:
    dt/df_a = sum over corner pairs (c, c with bit a set) of the other-axis
    weight times (row_hi - row_lo).  idx_of[src] = flat row indices [S, C]."""
    out = np.zeros((p.shape[0], 8))
    for src, fac in _axis_factors(p, scene).items():
        tab = np.asarray(scene[src], dtype=np.float64).reshape(-1, 8)
        idx = idx_of[src]
        for a in range(len(fac)):
            slope = np.zeros((p.shape[0], 8))
            for c in range(1 << len(fac)):
                if (c >> a) & 1:
                    continue
                hi_c = c | (1 << a)
                slope += _other_axis_weight(fac, c, a)[:, None] * (tab[idx[:, hi_c]] - tab[idx[:, c]])
            out += np.abs(slope)
    return out


def _input_abs_err(x: np.ndarray, raw_err: np.ndarray, freqs: int) -> np.ndarray:
    """Absolute float32 error of the MLP input [F, d, sin/cos(2^k d)] given
    the absolute error raw_err [R, 3] of the direction it was built from;
    F's own error is rel_F's (here 0)."""
    e = np.zeros_like(x)
    e[:, 7:10] = raw_err
    for k in range(freqs):
        e[:, 10 + 6 * k:13 + 6 * k] = (2.0 ** k) * raw_err + SINCOS_ERR
        e[:, 13 + 6 * k:16 + 6 * k] = (2.0 ** k) * raw_err + SINCOS_ERR
    return e


def _input_err_coeffs(fw: dict, e_x: np.ndarray):
    """Carry input errors e_x [R, N] through G: (coefficient in units of u
    relative to the hidden layers' absolute-term sums, max over both
    layers [R]; the absolute error of z3 in units of u [R, 3])."""
    w1, w2, w3 = fw["w"]
    eh1 = fw["m1"] * (e_x @ np.abs(w1).T)
    eh2 = fw["m2"] * (eh1 @ np.abs(w2).T)
    ez3 = eh2 @ np.abs(w3).T
    with np.errstate(divide="ignore", invalid="ignore"):
        r1 = np.where(fw["h1a"] > 0, eh1 / (U32 * fw["h1a"]), 0.0).max(axis=1, initial=0.0)
        r2 = np.where(fw["h2a"] > 0, eh2 / (U32 * fw["h2a"]), 0.0).max(axis=1, initial=0.0)
    return np.maximum(r1, r2), ez3 / U32


def gradient_error_scale(scene, o, d, prm: RenderParams, upstream: np.ndarray, smooth: Optional[dict] = None):
    """Error scales of the gradient of ``oracle_loss_and_grads(...,
    upstream=upstream, smooth=smooth)``, the backward for a given dL/dC:
    {src: (flat row indices, A [U, 8], B [U, 8], N [U])} for the four
    feature sources (the oracle gradient's row indices), 'mlp': (A [P],
    B [P], N) and, with prm.occ_eps > 0, 'occ': (cell indices, A [U, 2],
    B [U, 2], N [U]).  See the module docstring."""
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    with torch.no_grad():
        res = _render_chunk(scene, o, d, prm, grad=False)
    smp = res["samples"]
    ray, slot = smp["rows"], smp["slots"]
    n = o.shape[0]
    delta = float(prm.delta)
    tau = smp["tau"].numpy()
    v = torch.cat([smp["cd"], smp["f"]], dim=1).numpy()  # [S, 7] in [0, 1]
    n_eval = res["n_eval"].astype(np.int64)
    live = slot < n_eval[ray]
    S = tau.shape[0]

    # phi: absolute-term sum of the interpolated features (Eq. 2) per sample
    omega = _other_axis_weights(smp["p"], scene) if S else {k: np.zeros((0, 8)) for k in SOURCES}
    tabs = np.zeros((S, 8))
    for src in SOURCES:
        idx, w = smp["terms"][src]
        tab = np.abs(np.asarray(scene[src], dtype=np.float64).reshape(-1, 8))
        for c in range(idx.shape[1]):
            tabs += w[:, c:c + 1] * tab[idx[:, c]]
    if S:  # the interpolation factors' absolute error through dt/df
        tabs += FRAC_ERR * _fraction_slopes(smp["p"], scene, {k: smp["terms"][k][0] for k in SOURCES})
    phi = tabs.max(axis=1)

    # exact depths and weights of Eq. 1, in slot order
    smax = int(slot.max()) + 1 if S else 1
    a = np.where(live, tau * delta, 0.0)

    def ray_cumsum(x, reverse=False):
        dense = np.zeros((n, smax))
        dense[ray, slot] = x
        c = np.cumsum(dense[:, ::-1], axis=1)[:, ::-1] if reverse else np.cumsum(dense, axis=1)
        return c[ray, slot], dense.sum(axis=1)

    d_after, _ = ray_cumsum(a)
    t_next = np.exp(-d_after)
    w0 = np.where(live, np.exp(-(d_after - a)) * -np.expm1(-a), 0.0)
    e_s, _ = ray_cumsum(a * phi)  # depth-rounding factor E_s
    soft = smp["mask"] is not None
    m_val = smp["mask"].numpy() if soft else np.ones(S)
    if soft:
        eps = float(prm.occ_eps)
        box_lo = tuple(float(x) for x in scene["box_lo"])
        box_hi = tuple(float(x) for x in scene["box_hi"])
        occ = np.asarray(scene["occ"], dtype=np.float64).reshape(-1, 2)
        my, mx = scene["occ"].shape[0], scene["occ"].shape[1]
        p = smp["p"]
        cell = cell_index(p[:, 1], box_lo[1], box_hi[1], my) * mx + cell_index(p[:, 0], box_lo[0], box_hi[0], mx)
        zmin, zmax, z = occ[cell, 0], occ[cell, 1], p[:, 2]
        rise = np.clip((z - zmin) / eps, 0.0, 1.0)
        fall = np.clip((zmax - z) / eps, 0.0, 1.0)
        dz_val = np.stack([2.0 * rise / eps, 2.0 * fall / eps], axis=1)  # >= |dM/dz_min|, |dM/dz_max|

    # per-term relative error coefficients (units of u): rho_s per sample,
    # rho_mlp per ray
    rho_s = 64.0 + phi + e_s
    _, e_n = ray_cumsum(a * phi)
    rho_n = 64.0 + e_n
    x = res["x"].numpy()
    nin = x.shape[1]
    mlp = np.asarray(scene["mlp"], dtype=np.float64)
    fw = _mlp_abs(mlp, x)
    gate = (np.asarray(res["n_placed"]) > 0)[:, None]
    F = res["F"].numpy()
    F_err = np.zeros((n, 7))
    np.add.at(F_err, ray, (rho_s * w0 * m_val)[:, None] * v)
    rel_F = (F_err / np.maximum(np.abs(F), 1e-300)).max(axis=1, initial=0.0)
    # the MLP backward: dot products of <= N_in, 16, 3 terms, and the
    # re-evaluated sigmoid slope g(1 - g), whose pre-activation z3 rounds
    # relative to its absolute-term sum z3a (F carrying rel_F)
    freqs = int(scene.get("dir_freqs", 0))
    rel_in, ez3_in = _input_err_coeffs(fw, _input_abs_err(x, np.zeros((n, 3)), freqs))
    rho_mlp = 64.0 + nin + rel_in + gate[:, 0] * (rel_F + ((nin + 32.0 + rel_F)[:, None] * fw["z3a"] + ez3_in).max(axis=1))
    bg = np.abs(np.asarray(prm.c_bg, dtype=np.float64))
    T_n = res["T"].numpy()
    dC_val = np.abs(np.asarray(upstream, dtype=np.float64))
    dW_val, dx_val = _mlp_abs_backprop(fw, dC_val * gate)
    g7_val = np.concatenate([dC_val, np.zeros((n, 4))], axis=1) + gate * dx_val[:, :7]
    g7_err = gate * rho_mlp[:, None] * dx_val[:, :7]
    mlp_A = dW_val.sum(axis=0)
    mlp_B = (rho_mlp[:, None] * dW_val).sum(axis=0)
    mlp_N = int(gate.sum())
    if smooth is not None:
        rho_g = nin + 32.0 + rel_F
        sm = _smooth_scale(res, d, mlp, freqs, smooth, rho_mlp, rho_g)
        mlp_A = mlp_A + sm["A"]
        mlp_B = mlp_B + sm["B"]
        mlp_N += sm["N"]
        g7_val = g7_val + sm["dF_val"]
        g7_err = g7_err + sm["dF_err"]

    def per_sample(g7, dC, mfac, rs=None, rn=None):
        """Absolute terms of dL/dt per sample [S, 8] for |dL/dF| = g7,
        |dL/dC| = dC (its c_bg term) and the occupancy factor mfac in place
        of M, each term weighted by its coefficient (rs per sample, rn per
        ray; 1 if None)."""
        rs = np.ones(S) if rs is None else rs
        rn = np.ones(n) if rn is None else rn
        gv = np.einsum("sc,sc->s", g7[ray], v)
        w = w0 * mfac
        suffix, _ = ray_cumsum(rs * w * gv, reverse=True)
        suffix -= rs * w * gv
        gT = dC @ bg
        ab = np.zeros((S, 8))
        ab[:, 0] = delta * tau * (rs * t_next * mfac * gv + suffix + (rn * T_n * gT)[ray])
        ab[:, 1:] = (rs * w)[:, None] * g7[ray] * v * (1.0 - v)
        ab[~live] = 0.0
        return ab, gv

    no_dC = np.zeros((n, 3))
    ab_val, gv_val = per_sample(g7_val, dC_val, m_val)
    ab_b = per_sample(g7_val, dC_val, m_val, rho_s, rho_n)[0] + per_sample(g7_err, no_dC, m_val)[0]
    ab_b = ab_b + np.where(ab_val < TINY_TERM, ab_val / U32, 0.0)  # float32 range (module docstring)
    gv_err = np.einsum("sc,sc->s", g7_err[ray], v)

    out = {}
    for src in SOURCES:
        idx, w = smp["terms"][src]
        uniq, inv = np.unique(idx.reshape(-1), return_inverse=True)
        inv = inv.reshape(idx.shape)
        A = np.zeros((uniq.size, 8))
        B = np.zeros((uniq.size, 8))
        N = np.zeros(uniq.size, dtype=np.int64)
        for c in range(idx.shape[1]):
            np.add.at(A, inv[:, c], w[:, c:c + 1] * ab_val)
            np.add.at(B, inv[:, c], w[:, c:c + 1] * ab_b + FRAC_ERR * omega[src][:, c:c + 1] * ab_val)
            np.add.at(N, inv[:, c], live.astype(np.int64))
        out[src] = (uniq, A, B, N)
    out["mlp"] = (mlp_A, mlp_B, mlp_N)
    if soft:
        uniq, inv = np.unique(cell, return_inverse=True)
        lw = np.where(live, w0, 0.0)[:, None]
        occ_val = lw * gv_val[:, None] * dz_val
        occ_b = rho_s[:, None] * occ_val + lw * gv_err[:, None] * dz_val
        occ_b = occ_b + np.where(occ_val < TINY_TERM, occ_val / U32, 0.0)
        A = np.zeros((uniq.size, 2))
        B = np.zeros((uniq.size, 2))
        np.add.at(A, inv, occ_val)
        np.add.at(B, inv, occ_b)
        N = np.bincount(inv, weights=live.astype(np.float64), minlength=uniq.size).astype(np.int64)
        out["occ"] = (uniq, A, B, N)
    return out


def _smooth_scale(res, d, mlp, freqs, smooth, rho_mlp, rho_g):
    """MLP and dL/dF scales of the view-smoothness term of Eq. 9-10: two
    evaluations of G per (ray, perturbation), backpropagated with
    |dL/dG| = 2 |weight cos| |G_s - G_d| (values) and the rounding scale of
    G_s - G_d (each G rounds by rho_g g(1 - g) z3a plus its input error's
    g(1 - g) e_z3, their difference by the sum of the two), plus the float32
    cosine's error (10 u |cos| + 4 u) on the whole term.  The input of G_s
    is built from s = fl32(d + delta) (u |s| per component), that of G_d
    from the exact d."""
    F = res["F"].numpy()
    d64 = np.asarray(d, dtype=np.float64)
    pert = np.asarray(smooth["perturb"], dtype=np.float64)
    r, p = pert.shape[0], pert.shape[1]
    s = d64[:, None, :] + pert
    cos = (s * d64[:, None, :]).sum(-1) / (np.linalg.norm(s, axis=-1) * np.linalg.norm(d64, axis=-1)[:, None])
    Fp = np.repeat(F, p, axis=0)
    s2 = s.reshape(-1, 3)
    d2 = np.repeat(d64, p, axis=0)
    xs = np.concatenate([Fp, encode_dir(torch.from_numpy(s2), freqs).numpy()], 1)
    xd = np.concatenate([Fp, encode_dir(torch.from_numpy(d2), freqs).numpy()], 1)
    fs = _mlp_abs(mlp, xs)
    fd = _mlp_abs(mlp, xd)
    rel_s, ez3_s = _input_err_coeffs(fs, _input_abs_err(xs, U32 * np.abs(s2), freqs))
    rel_d, ez3_d = _input_err_coeffs(fd, _input_abs_err(xd, np.zeros_like(d2), freqs))
    wabs = 2.0 * abs(float(smooth["weight"]))
    wc = wabs * np.abs(cos).reshape(-1, 1)
    rm = np.repeat(rho_mlp, p)[:, None]
    rg = np.repeat(rho_g, p)[:, None]
    dg = np.abs(fs["g"] - fd["g"])
    dG_val = wc * dg
    dG_err = (wc * (fs["g"] + fd["g"] + rg * (fs["sg"] * fs["z3a"] + fd["sg"] * fd["z3a"])
                    + fs["sg"] * ez3_s + fd["sg"] * ez3_d)
              + dg * (10.0 * wc + 4.0 * wabs))
    tot = {}
    for name, dG in (("val", dG_val), ("err", dG_err)):
        dWs, dxs = _mlp_abs_backprop(fs, dG)
        dWd, dxd = _mlp_abs_backprop(fd, dG)
        tot[name] = (dWs, dWd, dxs[:, :7], dxd[:, :7])
    vWs, vWd, vxs, vxd = tot["val"]
    eWs, eWd, exs, exd = tot["err"]
    rms, rmd = rm + rel_s[:, None], rm + rel_d[:, None]
    return {"N": 2 * r * p, "A": (vWs + vWd).sum(0),
            "B": (rms * vWs + rmd * vWd).sum(0) + (eWs + eWd).sum(0),
            "dF_val": (vxs + vxd).reshape(r, p, 7).sum(axis=1),
            "dF_err": (rms * vxs + rmd * vxd + exs + exd).reshape(r, p, 7).sum(axis=1)}


def floor(scale) -> np.ndarray:
    """The rounding floor u (B + N A) + 65 N 2^-150 of one tensor's scale
    from gradient_error_scale: (A, B, N) or (indices, A, B, N), A and B
    [U, C] or [P], N [U] or a scalar."""
    A, B, N = scale[-3], scale[-2], scale[-1]
    N = np.asarray(N, dtype=np.float64)
    if A.ndim == 2:
        N = N[:, None]
    return U32 * (B + N * A) + SUBNORMAL_FLOOR * N


def compare(got: np.ndarray, ref: tuple, scale: tuple, rel: float = 1e-3) -> dict:
    """Per-entry parity of one gradient tensor against the oracle.

    got: the full gradient tensor under test (flattened to rows of the
    oracle's channel count); ref: the oracle's (indices, rows) or dense
    vector; scale: gradient_error_scale's entry.  The bar is
    |got - ref| <= rel |ref| + floor (u (B + N A) + 65 N 2^-150) on every
    oracle entry and
    got == 0 on entries no sample touches.  Returns the statistics: 'ok',
    'worst' (largest |err| / bar), 'err_over_uA' (largest |err| / (u A)),
    and for the entries with |ref| >= 1e-3 max |ref| ('big'): their count,
    the count whose float32 floor is below rel |ref| ('resolved'), the
    worst relative error over the resolved ones and over all big ones."""
    if isinstance(ref, tuple):
        idx, rows = ref
        g = np.asarray(got, dtype=np.float64).reshape(-1, rows.shape[-1])
        outside = np.ones(g.shape[0], bool)
        outside[idx] = False
        untouched_zero = bool(np.all(g[outside] == 0))
        g = g[idx]
    else:
        rows = np.asarray(ref, dtype=np.float64)
        g = np.asarray(got, dtype=np.float64)
        untouched_zero = True
    A = scale[-3]
    fl = floor(scale)
    err = np.abs(g - rows)
    bar = rel * np.abs(rows) + fl
    big = np.abs(rows) >= 1e-3 * np.abs(rows).max()
    resolved = big & (fl <= rel * np.abs(rows))
    relerr = err / np.maximum(np.abs(rows), 1e-300)
    worst = float((err / np.maximum(bar, 1e-300)).max(initial=0.0))
    return dict(ok=bool(np.all(err <= bar)) and untouched_zero, untouched_zero=untouched_zero, worst=worst,
                err_over_uA=float((err / np.maximum(U32 * A, 1e-300)).max(initial=0.0)),
                big=int(big.sum()), resolved=int(resolved.sum()),
                worst_rel_resolved=float(relerr[resolved].max(initial=0.0)),
                worst_rel_big=float(relerr[big].max(initial=0.0)))
