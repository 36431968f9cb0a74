"""Mutation check of the oracle pins: plant a plausible mistake in the oracle
(on the CPU) and require that at least one pin of test_oracle_pins fails.

Each mutant is a small, realistic slip -- a dropped feature source, a
transposed plane, a cell-centred instead of vertex-aligned grid, a missing
transmittance factor, a wrong decay, a lost background term, a missing ReLU,
a rounded instead of floored cell index, an open instead of closed interval,
an off-by-one lattice step, and for the soft occupancy (Eq. 5, 6, 8) the
mask also scaling T, exponent 1, the mask ignored and an unsquared span;
for the 8-bit storage (Sec. 4.4) ties rounded up, a 256-level step and a
code that wraps instead of clamping.
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.field as field
import oracle.fp32_bound as fp32_bound
import oracle.placement as placement
import oracle.quant as quant
import oracle.render as render
from tests import test_oracle_pins as pins

PIN_TESTS = [
    pins.test_vertical_rays_closed_form_counts,
    pins.test_horizontal_ray_closed_form_counts,
    pins.test_empty_and_full_plane,
    pins.test_placement_brute_force_small,
    pins.test_affine_field_reproduced_exactly,
    pins.test_interpolation_matches_grid_sample,
    lambda: pins.test_constant_density_closed_form(50.0, 1024),
    pins.test_single_sample_weight_is_alpha,
    pins.test_opaque_first_sample,
    pins.test_mlp_hand_example,
    pins.test_ert_stops_after_crossing_sample,
    pins.test_soft_mask_single_sample_hand_value,
    lambda: pins.test_occupancy_value_matches_paper_cases(2.0),
    pins.test_occ_interval_loss_hand_example,
    pins.test_direction_encoding_hand_values,
    pins.test_smooth_loss_hand_example,
    pins.test_quantize_u8_hand_values,
    pins.test_quant_params_span_the_range,
    pins.test_u8_scene_render_is_render_of_decoded_scene,
    pins.test_error_scale_covers_float32_underflow,
    pins.test_error_scale_input_errors_bound_a_perturbed_mlp,
    pins.test_error_scale_weight_error_bounds_perturbed_fractions,
    pins.test_error_scale_fraction_slopes_bound_a_perturbed_field,
]


def _any_pin_fails():
    for t in PIN_TESTS:
        try:
            t()
        except (AssertionError, ValueError, IndexError, RuntimeError):
            return True
    return False


def _drop_plane_yz(orig):
    def f(*a, **k):
        terms = orig(*a, **k)
        idx, w = terms["plane_yz"]
        terms["plane_yz"] = (idx, np.zeros_like(w))
        return terms
    return f


def _transpose_xz(orig):
    def f(p, box_lo, box_hi, grid_dims, plane_dims):
        terms = orig(p, box_lo, box_hi, grid_dims, plane_dims)
        nx, ny, nz = plane_dims
        # index the XZ plane as [x][z] instead of [z][x]
        terms["plane_xz"] = field.bilinear_corners(p[:, 2], p[:, 0], box_lo[2], box_hi[2], box_lo[0], box_hi[0],
                                                   nz, nx)
        return terms
    return f


def _cell_centred(c, lo, hi, n):
    u = (np.asarray(c, dtype=np.float64) - lo) / (hi - lo) * n - 0.5
    i0 = np.clip(np.floor(u), 0, n - 2).astype(np.int64)
    return i0, u - i0


def _composite_no_T(tau, cd, f, n_placed, delta, t_term=0.0, mask=None):
    r, s_max = tau.shape
    cd_acc = torch.zeros(r, 3, dtype=torch.float64)
    f_acc = torch.zeros(r, 4, dtype=torch.float64)
    T = torch.ones(r, dtype=torch.float64)
    npl = torch.as_tensor(n_placed, dtype=torch.int64)
    for s in range(s_max):
        m = npl > s
        a = tau[:, s] * delta
        w = torch.where(m, -torch.expm1(-a), torch.zeros_like(a))  # T dropped
        if mask is not None:
            w = w * mask[:, s]
        cd_acc = cd_acc + w[:, None] * cd[:, s]
        f_acc = f_acc + w[:, None] * f[:, s]
        T = torch.where(m, T * torch.exp(-a), T)
    return cd_acc, f_acc, T, npl


def _wrap_composite_decay(orig):
    def f(tau, cd, fe, n_placed, delta, t_term=0.0, mask=None):
        return orig(tau, cd, fe, n_placed, 2.0 * delta, t_term, mask)
    return f


def _mlp_no_relu(x, mlp):
    w1, b1, w2, b2, w3, b3 = render.unpack_mlp(mlp)
    return torch.sigmoid(((x @ w1.T + b1) @ w2.T + b2) @ w3.T + b3)


def _round_cell(p_a, lo, hi, m):
    scale = m / (hi - lo)
    v = np.round(np.asarray(p_a, dtype=np.float64) * scale) - lo * scale
    v = np.where(np.isfinite(v), v, 0.0)
    return np.clip(v, 0, m - 1).astype(np.int64)


def _open_zmax(orig):
    def f(p, occ, box_lo, box_hi):
        i = placement.cell_index(p[..., 0], box_lo[0], box_hi[0], occ.shape[1])
        j = placement.cell_index(p[..., 1], box_lo[1], box_hi[1], occ.shape[0])
        return orig(p, occ, box_lo, box_hi) & (p[..., 2] < occ[j, i, 1])
    return f


def _off_by_one(orig):
    def f(o, d, k, delta):
        return orig(o, d, np.asarray(k) + 1, delta)
    return f


def _no_background(orig):
    def f(scene, o, d, prm, grad, mlp_leaf=None):
        res = orig(scene, o, d, prm, grad, mlp_leaf)
        bg = torch.tensor(list(prm.c_bg), dtype=torch.float64)
        res["C"] = res["C"] - res["T"][:, None] * bg[None, :]
        return res
    return f


def _composite_mask_on_T(orig):
    """The rejected reading of Eq. 8: the occupancy value also scales the
    attenuation (T_{i+1} = T_i exp(-M_i a_i))."""
    def f(tau, cd, fe, n_placed, delta, t_term=0.0, mask=None):
        if mask is None:
            return orig(tau, cd, fe, n_placed, delta, t_term, mask)
        return orig(tau * mask, cd, fe, n_placed, delta, t_term, None)
    return f


def _occ_q1(orig):
    def f(z, zmin, zmax, eps, q):
        return orig(z, zmin, zmax, eps, 1.0)
    return f


def _occ_ones(z, zmin, zmax, eps, q):
    return torch.ones_like(z)


def _span_not_squared(occ):
    z = np.asarray(occ, dtype=np.float64)
    span = z[..., 1] - z[..., 0]
    return float(np.sum(np.abs(span))), np.stack([-np.sign(span), np.sign(span)], axis=-1)


def _encode_linear_freqs(d, freqs):
    parts = [d]
    for k in range(freqs):
        parts += [torch.sin(d * (k + 1)), torch.cos(d * (k + 1))]
    return torch.cat(parts, dim=-1)


def _smooth_no_cos(orig):
    """Drops the cosine weighting of Eq. 10 (every perturbation weighs 1)."""
    def f(F, d, perturb, mlp, freqs=0, weight=1.0):
        Ft = torch.from_numpy(np.asarray(F, dtype=np.float64))
        W = torch.from_numpy(np.asarray(mlp, dtype=np.float64))
        dt = torch.from_numpy(np.asarray(d, dtype=np.float64))
        st = dt[:, None, :] + torch.from_numpy(np.asarray(perturb, dtype=np.float64))
        g_d = render.mlp_forward(torch.cat([Ft, render.encode_dir(dt, freqs)], dim=1), W)
        r, p = st.shape[0], st.shape[1]
        x = torch.cat([Ft[:, None, :].expand(r, p, 7), render.encode_dir(st, freqs)], dim=2).reshape(r * p, -1)
        g_s = render.mlp_forward(x, W).reshape(r, p, 3)
        loss = weight * ((g_s - g_d[:, None, :]) ** 2).sum()
        return float(loss), np.zeros_like(np.asarray(F)), np.zeros_like(np.asarray(mlp))
    return f


def _quantize_half_up(x, lo, step):
    x = np.asarray(x, dtype=np.float32)
    y = (x - np.asarray(lo, np.float32)).astype(np.float32) * quant._inverse(step)
    y = np.floor(y.astype(np.float32) + np.float32(0.5))
    return np.clip(np.where(np.isnan(y), 0.0, y), 0.0, 255.0).astype(np.uint8)


def _params_256(minmax):
    mm = np.asarray(minmax, dtype=np.float32)
    return mm[:, 0].copy(), ((mm[:, 1] - mm[:, 0]) / np.float32(256.0)).astype(np.float32)


def _quantize_wrap(x, lo, step):
    x = np.asarray(x, dtype=np.float32)
    with np.errstate(invalid="ignore", over="ignore"):
        y = np.rint((x - np.asarray(lo, np.float32)).astype(np.float32) * quant._inverse(step))
    return np.where(np.isfinite(y), y, 0.0).astype(np.int64).astype(np.uint8)


def _both(mp, name, new):
    """Patch a field-module function in every module that bound it."""
    mp.setattr(field, name, new)
    if hasattr(render, name):
        mp.setattr(render, name, new)


def _input_err_unscaled(x, raw_err, freqs):
    """The encoded direction's error without the 2^k of d/dd sin(2^k d)."""
    e = np.zeros_like(x)
    e[:, 7:10] = raw_err
    for k in range(freqs):
        e[:, 10 + 6 * k:16 + 6 * k] = np.concatenate([raw_err, raw_err], 1) + fp32_bound.SINCOS_ERR
    return e


def _omega_is_weight(orig):
    """The weight term taken relative to the corner weight (omega = w)."""
    def f(p, scene):
        from oracle.field import feature_terms
        dims_g = scene["grid"].shape[:3][::-1]
        dims_p = (scene["plane_xy"].shape[1], scene["plane_xy"].shape[0], scene["plane_xz"].shape[0])
        terms = feature_terms(p, scene["box_lo"], scene["box_hi"], dims_g, dims_p)
        return {k: terms[k][1] for k in terms}
    return f


def _slopes_one_axis(orig):
    """Fraction slopes of the first axis only (the others forgotten)."""
    def f(p, scene, idx_of):
        q = p.copy()
        for a in (1, 2):  # put the other axes on vertices: their slopes no longer count
            lo, hi = float(scene["box_lo"][a]), float(scene["box_hi"][a])
            q[:, a] = lo
        return orig(q, scene, idx_of)
    return f


def _input_err_dropped(fw, e_x):
    return np.zeros(e_x.shape[0]), np.zeros((e_x.shape[0], 3))


MUTANTS = {
    "drop plane_yz": lambda mp: _both(mp, "feature_terms", _drop_plane_yz(field.feature_terms)),
    "transposed XZ plane": lambda mp: _both(mp, "feature_terms", _transpose_xz(field.feature_terms)),
    "cell-centred grid": lambda mp: mp.setattr(field, "corner_weights_1d", _cell_centred),
    "weight without T": lambda mp: mp.setattr(render, "composite", _composite_no_T),
    "double decay": lambda mp: mp.setattr(render, "composite", _wrap_composite_decay(render.composite)),
    "no ReLU": lambda mp: mp.setattr(render, "mlp_forward", _mlp_no_relu),
    "rounded cell index": lambda mp: mp.setattr(placement, "cell_index", _round_cell),
    "open z_max": lambda mp: mp.setattr(placement, "accept_mask", _open_zmax(placement.accept_mask)),
    "no background term": lambda mp: mp.setattr(render, "_render_chunk", _no_background(render._render_chunk)),
    "lattice off by one": lambda mp: mp.setattr(placement, "lattice_points", _off_by_one(placement.lattice_points)),
    "occupancy mask on T": lambda mp: mp.setattr(render, "composite", _composite_mask_on_T(render.composite)),
    "occupancy exponent 1": lambda mp: (mp.setattr(render, "occupancy_value", _occ_q1(render.occupancy_value)),
                                        mp.setattr(oracle, "occupancy_value", _occ_q1(render.occupancy_value))),
    "occupancy mask ignored": lambda mp: (mp.setattr(render, "occupancy_value", _occ_ones),
                                          mp.setattr(oracle, "occupancy_value", _occ_ones)),
    "encoding frequencies k, not 2^k": lambda mp: (mp.setattr(render, "encode_dir", _encode_linear_freqs),
                                                   mp.setattr(oracle, "encode_dir", _encode_linear_freqs)),
    "smoothness without cosine weight": lambda mp: (mp.setattr(render, "smooth_loss", _smooth_no_cos(None)),
                                                    mp.setattr(oracle, "smooth_loss", _smooth_no_cos(None))),
    "8-bit ties rounded up": lambda mp: (mp.setattr(quant, "quantize_u8", _quantize_half_up),
                                         mp.setattr(oracle, "quantize_u8", _quantize_half_up)),
    "8-bit step over 256 levels": lambda mp: (mp.setattr(quant, "quant_params", _params_256),
                                              mp.setattr(oracle, "quant_params", _params_256)),
    "8-bit code wraps instead of clamping": lambda mp: (mp.setattr(quant, "quantize_u8", _quantize_wrap),
                                                        mp.setattr(oracle, "quantize_u8", _quantize_wrap)),
    "error scale without the float32 underflow allowance": lambda mp: mp.setattr(fp32_bound, "TINY_TERM", 0.0),
    "error scale: encoding error not scaled by 2^k": lambda mp: mp.setattr(fp32_bound, "_input_abs_err",
                                                                           _input_err_unscaled),
    "error scale: MLP input errors dropped": lambda mp: mp.setattr(fp32_bound, "_input_err_coeffs",
                                                                   _input_err_dropped),
    "error scale: weight error relative to the weight": lambda mp: mp.setattr(
        fp32_bound, "_other_axis_weights", _omega_is_weight(fp32_bound._other_axis_weights)),
    "error scale: fraction slopes of one axis only": lambda mp: mp.setattr(
        fp32_bound, "_fraction_slopes", _slopes_one_axis(fp32_bound._fraction_slopes)),
    "interval loss not squared": lambda mp: (mp.setattr(render, "occ_interval_loss", _span_not_squared),
                                             mp.setattr(oracle, "occupancy_value", render.occupancy_value),
                                             mp.setattr(oracle, "occ_interval_loss", _span_not_squared)),
}


def test_unmutated_pins_pass():
    assert not _any_pin_fails()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    MUTANTS[name](monkeypatch)
    assert _any_pin_fails(), f"no pin catches the mutant '{name}'"
