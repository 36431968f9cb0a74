"""Volume rendering, deferred MLP, loss and float64 gradients (TEST INFRASTRUCTURE).

Follows Oblique-MERF Sec. 3: Eq. 1 (quadrature C = sum_i w_i c_i,
w_i = T_i alpha_i, alpha_i = 1 - exp(-tau_i delta_i), T_i = prod_{j<i}
(1 - alpha_j)), Eq. 4 (deferred shading: C = sum w c^d + G(F, d),
F = [sum w c^d, sum w f]) and Sec. 4.1, Eq. 6-8 (only samples inside the
occupancy interval contribute: with epsilon = 0 the mask is 0/1 and the
masked samples are simply not placed; with epsilon > 0 each placed
sample's weight is multiplied by the occupancy value M of Eq. 6).

Readings where the paper is silent or ambiguous:

* delta_i is the constant lattice step delta for every sample (each sample
  owns [t_i, t_i + delta)); the paper's t_{i+1} - t_i is undefined for the
  last sample and would span skipped gaps.
* Background: C = sum w c^d + [n_placed > 0] G(F, d) + T_n c_bg, where T_n
  is the transmittance after the last evaluated sample and c_bg a call
  parameter.  A ray with no sample returns exactly c_bg.
* G is N -> 16 -> 16 -> 3 with ReLU, ReLU, sigmoid; input order
  [sum w c^d (3), sum w f (4), enc(d)].  enc(d) is the raw unit direction
  d (N = 10), or, with L view-direction frequencies (the paper's deferred
  MLP uses four, as in MERF), [d, sin(2^0 d), cos(2^0 d), ...,
  sin(2^(L-1) d), cos(2^(L-1) d)] with each term a 3-vector
  (N = 7 + 3 (1 + 2 L); 34 for L = 4).  Parameters are packed
  [W1 (16xN), b1, W2 (16x16), b2, W3 (3x16), b3], weights row-major
  (out, in); N follows from the packed size.
* Early ray termination (not in the paper): with t_term > 0 a ray stops
  after the first sample whose following transmittance T_{i+1} < t_term;
  t_term = 0 never stops.
* Loss: L = mean over rays and the 3 channels of (C - C*)^2.
* Occupancy value (Eq. 6) with buffer width epsilon > 0 and exponent q:
  M = min(clamp((z - z_min)/eps, 0, 1)^q, clamp((z_max - z)/eps, 0, 1)^q),
  which equals the paper's four cases whenever z_max - z_min >= 2 eps and
  stays continuous when the two buffer zones overlap (the cases conflict
  there).  Eq. 8 multiplies the weight w_i by M_i; the transmittance T is
  left unmasked, as written.  M is read at the cell containing the
  sample's xy (Eq. 7), the same cell the placement used.

The forward and the gradient share one code path: the gradient is float64
autograd of exactly the forward below.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from .field import SOURCES, activations, feature_terms, interp_features
from .placement import cell_index, place_samples

MLP_SIZES = (10, 16, 16, 3)


@dataclasses.dataclass
class RenderParams:
    delta: float = 0.25 / 512
    n_max: int = 64
    t_term: float = 0.0
    c_bg: Sequence[float] = (0.0, 0.0, 0.0)
    occ_eps: float = 0.0  # buffer-zone width epsilon of Eq. 6 (0: the hard interval)
    occ_q: float = 2.0    # exponent q of Eq. 6


def occupancy_value(z: torch.Tensor, zmin: torch.Tensor, zmax: torch.Tensor, eps: float, q: float):
    """Occupancy function M of Sec. 4.1, Eq. 6, in the overlap-safe form of
    the module docstring."""
    rise = torch.clamp((z - zmin) / eps, 0.0, 1.0) ** q
    fall = torch.clamp((zmax - z) / eps, 0.0, 1.0) ** q
    return torch.minimum(rise, fall)


def smooth_loss(F: np.ndarray, d: np.ndarray, perturb: np.ndarray, mlp: np.ndarray, freqs: int = 0,
                weight: float = 1.0):
    """View-smoothness regulariser of Sec. 4.2, Eq. 9-10:
    L = weight * sum_r sum_p S(d_r, s_rp) ||G(F_r, s_rp) - G(F_r, d_r)||^2
    with s_rp = d_r + delta_rp and S the cosine similarity.  The Gaussian
    perturbations delta ~ N(0, Sigma) of Eq. 9 are drawn by the caller and
    passed in as `perturb` [R, P, 3]; s is used as it is (not renormalised),
    as written.  F [R, 7] (the composited features of Eq. 4), d [R, 3].
    Returns (loss, dL/dF [R, 7], dL/dmlp [n_params]) in float64."""
    Ft = torch.from_numpy(np.asarray(F, dtype=np.float64)).requires_grad_(True)
    W = torch.from_numpy(np.asarray(mlp, dtype=np.float64)).requires_grad_(True)
    loss = _smooth_term(Ft, np.asarray(d), np.asarray(perturb), W, freqs, weight)
    gF, gW = torch.autograd.grad(loss, [Ft, W])
    return float(loss.item()), gF.numpy(), gW.numpy()


def _smooth_term(Ft: torch.Tensor, d: np.ndarray, perturb: np.ndarray, W: torch.Tensor, freqs: int, weight: float):
    """The float64 graph of the smoothness loss of Eq. 9-10 (see smooth_loss)."""
    dt = torch.from_numpy(np.asarray(d, dtype=np.float64))
    st = dt[:, None, :] + torch.from_numpy(np.asarray(perturb, dtype=np.float64))
    g_d = mlp_forward(torch.cat([Ft, encode_dir(dt, freqs)], dim=1), W)
    r, p = st.shape[0], st.shape[1]
    Fp = Ft[:, None, :].expand(r, p, 7)
    g_s = mlp_forward(torch.cat([Fp, encode_dir(st, freqs)], dim=2).reshape(r * p, -1), W).reshape(r, p, 3)
    cos = (st * dt[:, None, :]).sum(-1) / (torch.linalg.norm(st, dim=-1) * torch.linalg.norm(dt, dim=-1)[:, None])
    return weight * (cos * ((g_s - g_d[:, None, :]) ** 2).sum(-1)).sum()


def occ_interval_loss(occ: np.ndarray):
    """Interval-span loss of Sec. 4.1, Eq. 5: sum over the grid points of
    (z_max - z_min)^2, and its gradient [My, Mx, 2] (float64)."""
    z = np.asarray(occ, dtype=np.float64)
    span = z[..., 1] - z[..., 0]
    grad = np.stack([-2.0 * span, 2.0 * span], axis=-1)
    return float(np.sum(span * span)), grad


def mlp_input_width(n_params: int) -> int:
    """N of the packed N -> 16 -> 16 -> 3 parameter vector."""
    rest = 16 + 16 * 16 + 16 + 3 * 16 + 3
    if (n_params - rest) % 16:
        raise ValueError(f"{n_params} is not an N x 16 x 16 x 3 parameter count")
    return (n_params - rest) // 16


def encode_dir(d: torch.Tensor, freqs: int) -> torch.Tensor:
    """View-direction input of the deferred MLP (see the module docstring)."""
    parts = [d]
    for k in range(freqs):
        parts += [torch.sin(d * 2.0 ** k), torch.cos(d * 2.0 ** k)]
    return torch.cat(parts, dim=-1)


def unpack_mlp(mlp):
    """Split the packed parameter vector into (W1, b1, W2, b2, W3, b3)."""
    out = []
    off = 0
    sizes = (mlp_input_width(mlp.shape[0]),) + MLP_SIZES[1:]
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        out.append(mlp[off:off + fout * fin].reshape(fout, fin))
        off += fout * fin
        out.append(mlp[off:off + fout])
        off += fout
    assert off == mlp.shape[0]
    return out


def mlp_forward(x: torch.Tensor, mlp: torch.Tensor) -> torch.Tensor:
    """Deferred MLP G of Eq. 4: sigmoid(W3 relu(W2 relu(W1 x + b1) + b2) + b3)."""
    w1, b1, w2, b2, w3, b3 = unpack_mlp(mlp)
    h1 = torch.relu(x @ w1.T + b1)
    h2 = torch.relu(h1 @ w2.T + b2)
    return torch.sigmoid(h2 @ w3.T + b3)


def composite(tau, cd, f, n_placed, delta: float, t_term: float = 0.0, mask=None):
    """Eq. 1 evaluated front to back, one sample slot at a time.

    tau [R, S], cd [R, S, 3], f [R, S, 4]; slot s of ray r is a sample iff
    s < n_placed[r].  mask [R, S] (optional): the occupancy value M of
    Eq. 6 applied to each weight (Eq. 8), not to T.  Returns (Cd [R,3],
    Fs [R,4], T_n [R], n_eval [R])."""
    r = tau.shape[0]
    s_max = tau.shape[1]
    T = torch.ones(r, dtype=torch.float64)
    cd_acc = torch.zeros(r, 3, dtype=torch.float64)
    f_acc = torch.zeros(r, 4, dtype=torch.float64)
    n_eval = torch.zeros(r, dtype=torch.int64)
    alive = torch.ones(r, dtype=torch.bool)
    npl = torch.as_tensor(n_placed, dtype=torch.int64)
    for s in range(s_max):
        m = (npl > s) & alive
        if not bool(m.any()):
            break
        a = tau[:, s] * delta
        alpha = -torch.expm1(-a)
        w = torch.where(m, T * alpha, torch.zeros_like(a))
        if mask is not None:
            w = w * mask[:, s]
        cd_acc = cd_acc + w[:, None] * cd[:, s]
        f_acc = f_acc + w[:, None] * f[:, s]
        T = torch.where(m, T * torch.exp(-a), T)
        n_eval = n_eval + m.to(torch.int64)
        if t_term > 0:
            alive = alive & ~(m & (T < t_term))
    return cd_acc, f_acc, T, n_eval


class _Tables:
    """Row lookup into the scene's feature sources, optionally through
    float64 leaf tensors holding only the rows touched (for gradients)."""

    def __init__(self, scene, terms: Optional[dict], grad: bool):
        self.scene = scene
        self.grad = grad
        self.leaves = {}
        self.uniq = {}
        self.inv = {}
        if grad:
            for src in SOURCES:
                idx = terms[src][0]
                u, inv = np.unique(idx.reshape(-1), return_inverse=True)
                rows = np.asarray(scene[src]).reshape(-1, 8)[u].astype(np.float64)
                leaf = torch.from_numpy(rows).requires_grad_(True)
                self.leaves[src] = leaf
                self.uniq[src] = u
                self.inv[src] = inv.reshape(idx.shape)

    def lookup(self, src, corner, idx):
        if not self.grad:
            rows = np.asarray(self.scene[src]).reshape(-1, 8)[idx]
            return torch.from_numpy(rows.astype(np.float64))
        return self.leaves[src][torch.from_numpy(self.inv[src][:, corner])]


def _render_chunk(scene, o, d, prm: RenderParams, grad: bool, mlp_leaf=None):
    box_lo = tuple(float(v) for v in scene["box_lo"])
    box_hi = tuple(float(v) for v in scene["box_hi"])
    grid_dims = scene["grid"].shape[2], scene["grid"].shape[1], scene["grid"].shape[0]
    plane_dims = scene["plane_xy"].shape[1], scene["plane_xy"].shape[0], scene["plane_xz"].shape[0]
    k_list, n_placed, pts = place_samples(o, d, scene["occ"], box_lo, box_hi, prm.delta, prm.n_max)
    r = o.shape[0]
    s_used = int(n_placed.max()) if r else 0
    rows, slots = np.nonzero(np.arange(max(s_used, 1))[None, :] < n_placed[:, None])
    p64 = pts[rows, slots].astype(np.float64)
    terms = feature_terms(p64, box_lo, box_hi, grid_dims, plane_dims)
    tables = _Tables(scene, terms, grad)
    t = interp_features(terms, tables.lookup) if rows.size else torch.zeros(0, 8, dtype=torch.float64)
    tau_s, cd_s, f_s = activations(t)
    s_dim = max(s_used, 1)
    ri = torch.from_numpy(rows)
    si = torch.from_numpy(slots)
    tau = torch.zeros(r, s_dim, dtype=torch.float64).index_put((ri, si), tau_s)
    cd = torch.zeros(r, s_dim, 3, dtype=torch.float64).index_put((ri, si), cd_s)
    f = torch.zeros(r, s_dim, 4, dtype=torch.float64).index_put((ri, si), f_s)
    mask, occ_leaf, occ_uniq = None, None, None
    if prm.occ_eps > 0:
        # Eq. 6-7: the occupancy value at the cell containing each sample's xy
        my, mx = scene["occ"].shape[0], scene["occ"].shape[1]
        cell = (cell_index(p64[:, 1], box_lo[1], box_hi[1], my) * mx
                + cell_index(p64[:, 0], box_lo[0], box_hi[0], mx))
        zz_all = np.asarray(scene["occ"], dtype=np.float64).reshape(-1, 2)
        if grad:
            occ_uniq, inv = np.unique(cell, return_inverse=True)
            occ_leaf = torch.from_numpy(zz_all[occ_uniq].copy()).requires_grad_(True)
            zz = occ_leaf[torch.from_numpy(inv.reshape(-1))]
        else:
            zz = torch.from_numpy(zz_all[cell])
        m_s = occupancy_value(torch.from_numpy(p64[:, 2]), zz[:, 0], zz[:, 1], prm.occ_eps, prm.occ_q)
        mask = torch.zeros(r, s_dim, dtype=torch.float64).index_put((ri, si), m_s)
    cd_acc, f_acc, T, n_eval = composite(tau, cd, f, n_placed, prm.delta, prm.t_term, mask)
    mlp = mlp_leaf if mlp_leaf is not None else torch.from_numpy(np.asarray(scene["mlp"], dtype=np.float64))
    freqs = int(scene.get("dir_freqs", 0))
    x = torch.cat([cd_acc, f_acc, encode_dir(torch.from_numpy(d.astype(np.float64)), freqs)], dim=1)
    gate = torch.from_numpy(n_placed > 0)
    g = mlp_forward(x, mlp)
    g = torch.where(gate[:, None], g, torch.zeros_like(g))
    bg = torch.tensor(list(prm.c_bg), dtype=torch.float64)
    C = cd_acc + g + T[:, None] * bg[None, :]
    F = torch.cat([cd_acc, f_acc], dim=1)
    return dict(C=C, T=T, F=F, n_placed=n_placed, n_eval=n_eval.numpy().astype(np.int32),
                k_list=k_list, tables=tables, occ_leaf=occ_leaf, occ_uniq=occ_uniq,
                # per-sample intermediates, for the float32 error scale of the gradient
                samples=dict(rows=rows, slots=slots, p=p64, terms=terms, tau=tau_s, cd=cd_s, f=f_s,
                             mask=None if mask is None else m_s), x=x, g=g)


def oracle_render(scene: Dict[str, np.ndarray], o: np.ndarray, d: np.ndarray, prm: RenderParams,
                  chunk: int = 1024, keep_k: bool = True):
    """Render rays (o, d) (float32 [n, 3]) through the scene.

    Returns float64 ``C`` [n,3], ``T`` [n], ``F`` [n,7] and int32
    ``n_placed``, ``n_eval`` [n] and (if keep_k) ``k_list`` [n, n_max]."""
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    n = o.shape[0]
    out = dict(C=np.zeros((n, 3)), T=np.zeros(n), F=np.zeros((n, 7)),
               n_placed=np.zeros(n, np.int32), n_eval=np.zeros(n, np.int32))
    if keep_k:
        out["k_list"] = np.full((n, prm.n_max), -1, np.int32)
    with torch.no_grad():
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            res = _render_chunk(scene, o[a:b], d[a:b], prm, grad=False)
            out["C"][a:b] = res["C"].numpy()
            out["T"][a:b] = res["T"].numpy()
            out["F"][a:b] = res["F"].numpy()
            out["n_placed"][a:b] = res["n_placed"]
            out["n_eval"][a:b] = res["n_eval"]
            if keep_k:
                out["k_list"][a:b] = res["k_list"]
    return out


def oracle_loss_and_grads(scene, o, d, prm: RenderParams, target: Optional[np.ndarray] = None,
                          smooth: Optional[dict] = None, upstream: Optional[np.ndarray] = None):
    """L2 loss (mean over rays x 3) and its float64 gradient.  With
    smooth = dict(perturb=[n, P, 3], weight=w) the loss also holds the
    view-smoothness term of Eq. 9-10 on the rays' composited features F
    (the training objective of Eq. 10 without its other regularisers).
    With upstream = [n, 3] instead of target, the colour term is the linear
    functional sum(upstream * C), whose gradient is the vector-Jacobian
    product of the render with that fixed dL/dC (the backward's input).

    Returns (loss, C, grads) where grads[src] = (flat row indices, [U, 8]
    gradient rows) for the four feature sources and grads['mlp'] is the
    dense [n_params] gradient; with prm.occ_eps > 0 also grads['occ'] = (flat
    cell indices, [U, 2] gradient of (z_min, z_max))."""
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    mlp_leaf = torch.from_numpy(np.asarray(scene["mlp"], dtype=np.float64).copy()).requires_grad_(True)
    res = _render_chunk(scene, o, d, prm, grad=True, mlp_leaf=mlp_leaf)
    C = res["C"]
    if (target is None) == (upstream is None):
        raise ValueError("pass exactly one of target and upstream")
    if upstream is not None:
        loss = torch.sum(torch.from_numpy(np.asarray(upstream, dtype=np.float64)) * C)
    else:
        loss = torch.mean((C - torch.from_numpy(np.asarray(target, dtype=np.float64))) ** 2)
    if smooth is not None:
        loss = loss + _smooth_term(res["F"], d, smooth["perturb"], mlp_leaf, int(scene.get("dir_freqs", 0)),
                                   float(smooth["weight"]))
    tables = res["tables"]
    leaves = [tables.leaves[s] for s in SOURCES] + [mlp_leaf]
    if res["occ_leaf"] is not None:
        leaves.append(res["occ_leaf"])
    gr = torch.autograd.grad(loss, leaves, allow_unused=True)
    grads = {}
    for s, g in zip(SOURCES, gr[:4]):
        grads[s] = (tables.uniq[s], (g if g is not None else torch.zeros_like(tables.leaves[s])).numpy())
    grads["mlp"] = gr[4].numpy() if gr[4] is not None else np.zeros(mlp_leaf.shape)
    if res["occ_leaf"] is not None:
        g = gr[5] if gr[5] is not None else torch.zeros_like(res["occ_leaf"])
        grads["occ"] = (res["occ_uniq"], g.numpy())
    return float(loss.item()), C.detach().numpy(), grads
