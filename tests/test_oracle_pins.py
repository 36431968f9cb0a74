"""Pins of the CPU oracle against closed forms, library routines and brute force.

Each test checks the oracle against something other than itself: exact
rational sample counts, affine-field reproduction, torch grid_sample,
closed-form transmittance, a hand-derived MLP example (tests/golden/),
float64 finite differences and sum invariants.  Citations name the
Oblique-MERF passage the checked behaviour comes from.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
import oracle.field
import oracle.render
from tests._scenes import BOX_HI, BOX_LO, DELTA, micro_scene, vertex_coords

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _f32(x):
    return np.asarray(x, dtype=np.float32)


# ---------------------------------------------------------------------------
# Placement (Sec. 4.1 Eq. 6-7, Sec. 4.4): exact counts with rational arithmetic
# ---------------------------------------------------------------------------

def test_vertical_rays_closed_form_counts():
    """d = (0,0,-1) from z = 1: p_z = 1 - k delta exactly, so the accepted k
    are the integers in [(1 - zmax')/delta, (1 - zmin')/delta] with the
    interval clipped to the box."""
    rng = np.random.default_rng(5)
    m = 8
    occ = np.empty((m, m, 2), np.float32)
    occ[..., 0] = rng.uniform(-0.05, 0.2, (m, m))
    occ[..., 1] = occ[..., 0] + rng.uniform(-0.02, 0.12, (m, m))
    n = 300
    xy = rng.uniform(-1, 1, (n, 2)).astype(np.float32)
    xy[:4] = [[-1, -1], [1, 1], [0, 0], [-0.75, 0.5]]  # faces and cell borders
    o = np.concatenate([xy, np.ones((n, 1), np.float32)], axis=1)
    d = np.tile(_f32([0, 0, -1]), (n, 1))
    k_list, n_placed, _ = oracle.place_samples(o, d, occ, BOX_LO, BOX_HI, DELTA, 1024)
    dl = Fraction(DELTA)
    for r in range(n):
        x, y = Fraction(float(xy[r, 0])), Fraction(float(xy[r, 1]))
        i = min(int(math.floor((x + 1) * m / 2)), m - 1)
        j = min(int(math.floor((y + 1) * m / 2)), m - 1)
        lo = max(Fraction(float(occ[j, i, 0])), Fraction(0))
        hi = min(Fraction(float(occ[j, i, 1])), Fraction(1, 4))
        if lo > hi:
            want = []
        else:
            k0 = math.ceil((1 - hi) / dl)
            k1 = math.floor((1 - lo) / dl)
            want = list(range(k0, k1 + 1))
        assert n_placed[r] == len(want), r
        assert list(k_list[r, :n_placed[r]]) == want


def test_horizontal_ray_closed_form_counts():
    """d = (1,0,0) from x = -1.5 on the lattice: each occupied cell of width
    2/M holds 4096/M lattice points (half-open), plus the far face point."""
    m = 16
    rng = np.random.default_rng(7)
    occ = np.empty((m, m, 2), np.float32)
    occ[..., 0] = 0.1
    occ[..., 1] = np.where(rng.random((m, m)) < 0.5, 0.2, 0.05)
    for yv, zv in [(0.3, 0.15), (-0.9, 0.12), (0.0, 0.1)]:
        o = _f32([[-1.5, yv, zv]])
        d = _f32([[1, 0, 0]])
        k_list, n_placed, _ = oracle.place_samples(o, d, occ, BOX_LO, BOX_HI, DELTA, 8192)
        j = min(int(math.floor((Fraction(float(np.float32(yv))) + 1) * m / 2)), m - 1)
        z = np.float32(zv)
        want = []
        for i in range(m):
            if occ[j, i, 0] <= z <= occ[j, i, 1]:
                per = 4096 // m
                first = 1024 + i * per
                want.extend(range(first, first + per))
                if i == m - 1:
                    want.append(1024 + 4096)
        assert n_placed[0] == len(want)
        assert list(k_list[0, :n_placed[0]]) == want


def test_empty_and_full_plane():
    """Empty plane (z_min > z_max): no samples, C = c_bg exactly, T = 1.
    Full plane: a vertical ray from z = 1 gets every lattice point with
    0.75 <= k delta <= 1, i.e. 513 samples."""
    prm = oracle.RenderParams(n_max=4200, c_bg=(0.25, 0.5, 0.75))
    sc = micro_scene(zmin=0.2, zmax=0.1, seed=3)
    o, d = _f32([[0.1, 0.2, 1.0], [-2, 0, 0.1]]), _f32([[0, 0, -1], [1, 0, 0]])
    r = oracle.oracle_render(sc, o, d, prm)
    assert (r["n_placed"] == 0).all()
    assert np.array_equal(r["C"], np.tile([0.25, 0.5, 0.75], (2, 1)))
    assert np.array_equal(r["T"], [1.0, 1.0])
    sc = micro_scene(zmin=0.0, zmax=0.25, seed=3)
    r = oracle.oracle_render(sc, o, d, prm)
    assert r["n_placed"][0] == 513
    assert r["n_placed"][1] == 4097


def _brute_force_count(o, d, occ, n_kmax):
    """Scalar loop over every k in [0, n_kmax): independent of the oracle's
    vectorised bisection of the box range."""
    m = occ.shape[0]
    cnt = []
    for k in range(n_kmax):
        t = np.float32(k * DELTA)
        p = [np.float32(o[a] + np.float32(t * d[a])) for a in range(3)]
        if not (-1 <= p[0] <= 1 and -1 <= p[1] <= 1 and 0 <= p[2] <= 0.25):
            continue
        i = min(max(int(math.floor(float(p[0]) * (m / 2))) + m // 2, 0), m - 1)
        j = min(max(int(math.floor(float(p[1]) * (m / 2))) + m // 2, 0), m - 1)
        if occ[j, i, 0] <= p[2] <= occ[j, i, 1]:
            cnt.append(k)
    return cnt


def test_placement_brute_force_small():
    """Random oblique rays near the box vs a plain scalar loop over all k."""
    rng = np.random.default_rng(11)
    m = 4
    occ = np.empty((m, m, 2), np.float32)
    occ[..., 0] = rng.uniform(0.0, 0.15, (m, m))
    occ[..., 1] = occ[..., 0] + rng.uniform(0.0, 0.1, (m, m))
    occ[0, 0] = (0.2, 0.1)  # one empty cell
    n = 12
    a = rng.uniform(-1, 1, (n, 2))
    pitch = rng.uniform(0.2, 1.3, n)
    yaw = rng.uniform(0, 2 * np.pi, n)
    d = np.stack([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), -np.sin(pitch)], 1)
    o = np.concatenate([a, np.full((n, 1), 0.1)], 1) - 0.4 * d
    o, d = o.astype(np.float32), d.astype(np.float32)
    k_list, n_placed, _ = oracle.place_samples(o, d, occ, BOX_LO, BOX_HI, DELTA, 8192)
    for r in range(n):
        want = _brute_force_count(o[r], d[r], occ, 9000)
        assert list(k_list[r, :n_placed[r]]) == want


def test_nested_intervals_nested_sets():
    """Widening every occupancy interval can only add samples."""
    rng = np.random.default_rng(2)
    m = 8
    inner = np.empty((m, m, 2), np.float32)
    inner[..., 0] = rng.uniform(0.05, 0.15, (m, m))
    inner[..., 1] = inner[..., 0] + rng.uniform(0, 0.05, (m, m))
    outer = inner.copy()
    outer[..., 0] -= rng.uniform(0, 0.03, (m, m)).astype(np.float32)
    outer[..., 1] += rng.uniform(0, 0.03, (m, m)).astype(np.float32)
    import scenegen
    o, d = scenegen.oblique_rays(64, seed=4)
    ki, ni, _ = oracle.place_samples(o, d, inner, BOX_LO, BOX_HI, DELTA, 4096)
    ko, no, _ = oracle.place_samples(o, d, outer, BOX_LO, BOX_HI, DELTA, 4096)
    assert (ni <= no).all() and (no > ni).any()
    for r in range(64):
        assert set(ki[r, :ni[r]]) <= set(ko[r, :no[r]])


def test_n_max_keeps_first_in_k_order():
    sc = micro_scene(zmin=0.0, zmax=0.25)
    o, d = _f32([[0.3, 0.3, 1.0]]), _f32([[0, 0, -1]])
    k_all, n_all, _ = oracle.place_samples(o, d, sc["occ"], BOX_LO, BOX_HI, DELTA, 1024)
    k5, n5, _ = oracle.place_samples(o, d, sc["occ"], BOX_LO, BOX_HI, DELTA, 5)
    assert n5[0] == 5 and list(k5[0]) == list(k_all[0, :5])
    assert list(k_all[0, :3]) == [1536, 1537, 1538]


def test_nan_and_inf_rays_place_nothing():
    sc = micro_scene(zmin=0.0, zmax=0.25)
    o = _f32([[np.nan, 0, 1], [0, 0, 1], [0, 0, np.inf]])
    d = _f32([[0, 0, -1], [np.nan, 0, -1], [0, 0, -1]])
    _, n, _ = oracle.place_samples(o, d, sc["occ"], BOX_LO, BOX_HI, DELTA, 64)
    assert (n == 0).all()


# ---------------------------------------------------------------------------
# Features (Sec. 3 Eq. 2-3)
# ---------------------------------------------------------------------------

def _affine_scene(grid, planes, coef):
    """Each source holds an affine function of its own coordinates."""
    lx, ly, lz = grid
    nx, ny, nz = planes
    sc = micro_scene(grid=grid, planes=planes)
    gx, gy, gz = (vertex_coords(lx, -1, 1), vertex_coords(ly, -1, 1), vertex_coords(lz, 0, 0.25))
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    c = coef["grid"]
    sc["grid"] = (c[0] + c[1] * X[..., None] + c[2] * Y[..., None] + c[3] * Z[..., None]).astype(np.float64)
    px, py, pz = vertex_coords(nx, -1, 1), vertex_coords(ny, -1, 1), vertex_coords(nz, 0, 0.25)
    for name, (u, v) in {"plane_xy": (px, py), "plane_xz": (px, pz), "plane_yz": (py, pz)}.items():
        V, U = np.meshgrid(v, u, indexing="ij")
        c = coef[name]
        sc[name] = c[0] + c[1] * U[..., None] + c[2] * V[..., None]
    return sc


def test_affine_field_reproduced_exactly():
    rng = np.random.default_rng(9)
    grid, planes = (5, 7, 4), (9, 6, 8)
    coef = {"grid": rng.standard_normal((4, 8))}
    for name in ("plane_xy", "plane_xz", "plane_yz"):
        coef[name] = rng.standard_normal((3, 8))
    sc = _affine_scene(grid, planes, coef)
    p = np.stack([rng.uniform(-1, 1, 500), rng.uniform(-1, 1, 500), rng.uniform(0, 0.25, 500)], 1)
    p[:3] = [[-1, -1, 0], [1, 1, 0.25], [1, -1, 0.25]]  # faces
    terms = oracle.field.feature_terms(p, BOX_LO, BOX_HI, grid, planes)
    t = oracle.field.interp_features(terms, lambda s, c, idx: torch.from_numpy(sc[s].reshape(-1, 8)[idx])).numpy()
    x, y, z = p[:, 0:1], p[:, 1:2], p[:, 2:3]
    g, a, b, e = coef["grid"], coef["plane_xy"], coef["plane_xz"], coef["plane_yz"]
    want = (g[0] + g[1] * x + g[2] * y + g[3] * z + a[0] + a[1] * x + a[2] * y
            + b[0] + b[1] * x + b[2] * z + e[0] + e[1] * y + e[2] * z)
    np.testing.assert_allclose(t, want, rtol=0, atol=1e-12)


def test_interpolation_matches_grid_sample():
    """Vertex-aligned interpolation equals grid_sample(align_corners=True)."""
    import torch.nn.functional as Fn
    sc = micro_scene(grid=(6, 5, 4), planes=(7, 9, 5), seed=1)
    rng = np.random.default_rng(3)
    p = np.stack([rng.uniform(-1, 1, 300), rng.uniform(-1, 1, 300), rng.uniform(0, 0.25, 300)], 1)
    terms = oracle.field.feature_terms(p, BOX_LO, BOX_HI, (6, 5, 4), (7, 9, 5))
    src = {k: torch.from_numpy(sc[k].astype(np.float64)) for k in ("grid", "plane_xy", "plane_xz", "plane_yz")}
    t = oracle.field.interp_features(terms, lambda s, c, idx: src[s].reshape(-1, 8)[torch.from_numpy(idx)]).numpy()
    nx = torch.from_numpy(p[:, 0])
    ny = torch.from_numpy(p[:, 1])
    nz = torch.from_numpy(p[:, 2] / 0.125 - 1)
    vol = src["grid"].permute(3, 0, 1, 2)[None]
    g3 = torch.stack([nx, ny, nz], 1)[None, :, None, None, :]
    ref = Fn.grid_sample(vol, g3, mode="bilinear", align_corners=True)[0, :, :, 0, 0].T
    for name, (u, v) in {"plane_xy": (nx, ny), "plane_xz": (nx, nz), "plane_yz": (ny, nz)}.items():
        img = src[name].permute(2, 0, 1)[None]
        g2 = torch.stack([u, v], 1)[None, :, None, :]
        ref = ref + Fn.grid_sample(img, g2, mode="bilinear", align_corners=True)[0, :, :, 0].T
    np.testing.assert_allclose(t, ref.numpy(), rtol=0, atol=1e-12)


def test_activations_textbook_values():
    t = torch.tensor([[math.log(2.0), 0.0, 100.0, -100.0, 0.0, math.log(3.0), 0.0, 0.0]], dtype=torch.float64)
    tau, cd, f = oracle.field.activations(t)
    assert tau.item() == pytest.approx(2.0, rel=1e-15)
    np.testing.assert_allclose(cd.numpy(), [[0.5, 1.0, 0.0]], atol=1e-15)
    np.testing.assert_allclose(f.numpy(), [[0.5, 0.75, 0.5, 0.5]], atol=1e-15)


# ---------------------------------------------------------------------------
# Compositing (Eq. 1, 4) and the deferred MLP
# ---------------------------------------------------------------------------

def _sigma32(sigma):
    """The density actually stored: exp of the binary32 value of ln(sigma)."""
    return math.exp(float(np.float32(math.log(sigma))))


def _constant_density_scene(sigma, colour_pre, mlp_b3):
    sc = micro_scene(zmin=0.0, zmax=0.25)
    sc["grid"][..., 0] = np.float32(math.log(sigma))
    sc["grid"][..., 1:] = np.float32(colour_pre)
    mlp = np.zeros(499, np.float32)
    mlp[-3:] = mlp_b3
    sc["mlp"] = mlp
    return sc


@pytest.mark.parametrize("sigma,n_max", [(50.0, 1024), (800.0, 1024), (30.0, 100)])
def test_constant_density_closed_form(sigma, n_max):
    """Constant tau = sigma over n samples: T = exp(-sigma n delta),
    sum w = 1 - T, Cd = (1 - T) sigmoid(c); zero MLP weights give
    G = sigmoid(b3)."""
    c = 0.4
    b3 = np.array([0.3, -0.7, 1.1], np.float32)
    sc = _constant_density_scene(sigma, c, b3)
    sigma = _sigma32(sigma)
    bg = (0.25, 0.5, 0.75)
    prm = oracle.RenderParams(n_max=n_max, c_bg=bg)
    o, d = _f32([[0.2, -0.4, 1.0]]), _f32([[0, 0, -1]])
    r = oracle.oracle_render(sc, o, d, prm)
    n = min(513, n_max)
    assert r["n_placed"][0] == n
    T = math.exp(-sigma * n * DELTA)
    s = 1 / (1 + math.exp(-float(np.float32(c))))
    assert r["T"][0] == pytest.approx(T, rel=1e-12)
    np.testing.assert_allclose(r["F"][0, :3], (1 - T) * s, rtol=1e-12)
    np.testing.assert_allclose(r["F"][0, 3:], (1 - T) * s, rtol=1e-12)
    g = 1 / (1 + np.exp(-b3.astype(np.float64)))
    np.testing.assert_allclose(r["C"][0], (1 - T) * s + g + T * np.array(bg), rtol=1e-12)


def test_single_sample_weight_is_alpha():
    """A one-point interval (z_min = z_max = 1 - k delta): w_1 = alpha_1."""
    sigma = 700.0
    sc = _constant_density_scene(sigma, 0.0, [0, 0, 0])
    sigma = _sigma32(sigma)
    z = np.float32(1 - 1700 * DELTA)
    sc["occ"][..., 0] = z
    sc["occ"][..., 1] = z
    r = oracle.oracle_render(sc, _f32([[0.1, 0.1, 1.0]]), _f32([[0, 0, -1]]), oracle.RenderParams(n_max=8))
    assert r["n_placed"][0] == 1
    alpha = 1 - math.exp(-sigma * DELTA)
    np.testing.assert_allclose(r["F"][0, :3], alpha * 0.5, rtol=1e-13)
    assert r["T"][0] == pytest.approx(1 - alpha, rel=1e-13)


def test_opaque_first_sample():
    """tau delta >> 1 at the first sample: C = c^d_1 + G, T = 0."""
    sc = _constant_density_scene(math.exp(30.0), 1.5, [0, 0, 0])
    r = oracle.oracle_render(sc, _f32([[0.1, 0.1, 1.0]]), _f32([[0, 0, -1]]),
                             oracle.RenderParams(n_max=64, c_bg=(1, 1, 1)))
    s = 1 / (1 + math.exp(-float(np.float32(1.5))))
    np.testing.assert_allclose(r["F"][0, :3], s, rtol=1e-14)
    assert r["T"][0] == 0.0
    np.testing.assert_allclose(r["C"][0], s + 0.5, rtol=1e-14)


def test_mlp_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "mlp_hand_example.json")))
    w1 = np.zeros((16, 10))
    w1[np.arange(10), np.arange(10)] = 1
    b1 = np.full(16, -0.5)
    w2 = np.zeros((16, 16))
    w2[:, :8] = 1
    b2 = np.zeros(16)
    w3 = np.full((3, 16), 0.1)
    b3 = np.array(g["b3"])
    mlp = torch.from_numpy(np.concatenate([w1.ravel(), b1, w2.ravel(), b2, w3.ravel(), b3]))
    out = oracle.render.mlp_forward(torch.tensor([g["x"]], dtype=torch.float64), mlp).numpy()[0]
    np.testing.assert_allclose(out, g["expected_g"], atol=1e-10)


def test_ert_stops_after_crossing_sample():
    """With t_term, the ray stops after the first sample whose T_{i+1}
    falls below t_term: n_eval = ceil(ln(1/t_term) / (sigma delta))."""
    sigma = 400.0
    sc = _constant_density_scene(sigma, 0.0, [0, 0, 0])
    sigma = _sigma32(sigma)
    t_term = 1e-3
    r = oracle.oracle_render(sc, _f32([[0.1, 0.1, 1.0]]), _f32([[0, 0, -1]]),
                             oracle.RenderParams(n_max=1024, t_term=t_term))
    want = math.ceil(math.log(1 / t_term) / (sigma * DELTA))
    assert r["n_placed"][0] == 513 and r["n_eval"][0] == want
    assert r["T"][0] == pytest.approx(math.exp(-sigma * DELTA * want), rel=1e-12)


# ---------------------------------------------------------------------------
# Gradients (O8): float64 FD, sum invariant, closed-form derivative
# ---------------------------------------------------------------------------

def _grad_problem(seed=0):
    import scenegen
    sc = micro_scene(grid=(5, 4, 3), planes=(7, 6, 5), m=4, zmin=0.02, zmax=0.2, seed=seed, std=0.7)
    sc["grid"][..., 0] += 3.0
    o, d = scenegen.oblique_rays(24, seed=seed + 10, origin_z=0.6)
    tgt = np.random.default_rng(seed).uniform(0, 1, (24, 3))
    return sc, o, d, tgt


def test_gradient_matches_fd_float64():
    sc, o, d, tgt = _grad_problem()
    prm = oracle.RenderParams(n_max=256, c_bg=(0.2, 0.4, 0.6))
    loss, _, grads = oracle.oracle_loss_and_grads(sc, o, d, prm, tgt)
    rng = np.random.default_rng(1)
    eps = 1e-6
    checked = 0
    for src in ("grid", "plane_xy", "plane_xz", "plane_yz", "mlp"):
        flat = sc[src].reshape(-1)
        if src == "mlp":
            cand = np.arange(499)
            gdense = grads["mlp"]
        else:
            u, g = grads[src]
            gdense = np.zeros(flat.size)
            gdense[(u[:, None] * 8 + np.arange(8)).ravel()] = g.ravel()
            cand = np.nonzero(gdense)[0]
        for e in rng.choice(cand, 6, replace=False):
            sp = {k: (v.astype(np.float64).copy() if k == src else v) for k, v in sc.items()}
            vals = []
            for s in (+1, -1):
                sp[src].reshape(-1)[e] = float(flat[e]) + s * eps
                r = oracle.oracle_render(sp, o, d, prm)
                vals.append(np.mean((r["C"] - tgt) ** 2))
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert abs(fd - gdense[e]) <= 1e-6 * max(abs(fd), 1e-3), (src, e, fd, gdense[e])
            checked += 1
    assert checked == 30


def test_gradient_sum_invariant_across_sources():
    """Each interpolation's weights sum to 1, so per channel the total
    gradient of every source equals sum_samples dL/dt_c."""
    sc, o, d, tgt = _grad_problem(seed=4)
    _, _, grads = oracle.oracle_loss_and_grads(sc, o, d, oracle.RenderParams(n_max=256), tgt)
    sums = [grads[s][1].sum(axis=0) for s in ("grid", "plane_xy", "plane_xz", "plane_yz")]
    for s in sums[1:]:
        np.testing.assert_allclose(s, sums[0], rtol=1e-10, atol=1e-14)


def test_gradient_constant_density_closed_form():
    """Shifting every grid ch0 value by e multiplies sigma by exp(e); with a
    zero-weight MLP, dL/de = sum_r sum_c 2 (C - C*)/(3R) * sigma n delta
    exp(-sigma n delta) s, which must equal the sum of the ch0 gradients."""
    sigma, c = 60.0, 0.3
    sc = _constant_density_scene(sigma, c, [0.1, 0.2, 0.3])
    sigma = _sigma32(sigma)
    o = _f32([[0.1, 0.1, 1.0], [-0.5, 0.6, 1.0], [0.7, -0.2, 1.0]])
    d = np.tile(_f32([0, 0, -1]), (3, 1))
    tgt = np.array([[0.2, 0.3, 0.4], [0.9, 0.1, 0.5], [0.5, 0.5, 0.5]])
    loss, C, grads = oracle.oracle_loss_and_grads(sc, o, d, oracle.RenderParams(n_max=1024), tgt)
    n = 513
    s = 1 / (1 + math.exp(-float(np.float32(c))))
    dcd = sigma * n * DELTA * math.exp(-sigma * n * DELTA) * s
    want = np.sum(2 * (C - tgt) / 9.0 * dcd)
    assert grads["grid"][1][:, 0].sum() == pytest.approx(want, rel=1e-10)


# ---------------------------------------------------------------------------
# Soft occupancy (Sec. 4.1 Eq. 5, 6, 8 with epsilon > 0)
# ---------------------------------------------------------------------------

def _eq6_cases(z, zmin, zmax, eps, q):
    """The four cases of Eq. 6 as printed (valid when zmax - zmin >= 2 eps)."""
    if zmin + eps <= z <= zmax - eps:
        return 1.0
    if z < zmin or z > zmax:
        return 0.0
    if zmin <= z <= zmin + eps:
        return (z - zmin) ** q / eps ** q
    return (zmax - z) ** q / eps ** q


@pytest.mark.parametrize("q", [2.0, 1.0])
def test_occupancy_value_matches_paper_cases(q):
    zmin, zmax, eps = 0.1, 0.2, 0.02
    z = np.linspace(0.05, 0.25, 401)
    got = oracle.occupancy_value(torch.from_numpy(z), torch.tensor(zmin, dtype=torch.float64),
                                 torch.tensor(zmax, dtype=torch.float64), eps, q).numpy()
    want = np.array([_eq6_cases(v, zmin, zmax, eps, q) for v in z])
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)


def test_soft_mask_single_sample_hand_value():
    """Vertical ray, n_max = 1: the one sample sits at the top lattice point
    z1 <= z_max, inside the upper buffer zone.  Eq. 8 scales its weight by
    M = ((z_max - z1) / eps)^2 and leaves T = exp(-sigma delta) unmasked."""
    sigma, c = 90.0, 0.25
    b3 = np.array([0.5, -0.25, 0.125], np.float32)
    sc = _constant_density_scene(sigma, c, b3)
    sigma = _sigma32(sigma)
    k1 = 1700
    z1 = 1.0 - k1 * DELTA                       # exact in binary32
    zmax = np.float32(z1 + 0.375 * DELTA)       # between z1 and the next lattice point up
    sc["occ"][..., 0] = np.float32(0.01)
    sc["occ"][..., 1] = zmax
    eps = 4 * DELTA
    bg = (0.25, 0.5, 0.75)
    r = oracle.oracle_render(sc, _f32([[0.3, -0.1, 1.0]]), _f32([[0, 0, -1]]),
                             oracle.RenderParams(n_max=1, c_bg=bg, occ_eps=eps))
    assert r["n_placed"][0] == 1 and r["k_list"][0, 0] == k1
    m = ((float(zmax) - z1) / eps) ** 2
    alpha = 1 - math.exp(-sigma * DELTA)
    s = 1 / (1 + math.exp(-float(np.float32(c))))
    T = math.exp(-sigma * DELTA)
    np.testing.assert_allclose(r["F"][0], m * alpha * s, rtol=1e-12)
    assert r["T"][0] == pytest.approx(T, rel=1e-13)
    g = 1 / (1 + np.exp(-b3.astype(np.float64)))
    np.testing.assert_allclose(r["C"][0], m * alpha * s + g + T * np.array(bg), rtol=1e-12)


def test_soft_mask_small_eps_is_the_hard_interval():
    """Interval ends half a lattice step from every sample of vertical rays
    and eps a quarter step: every placed sample has M = 1, so the soft and
    hard renders coincide."""
    sc = micro_scene(grid=(5, 4, 3), planes=(7, 6, 5), m=4, seed=3, std=0.6)
    rng = np.random.default_rng(4)
    lo = 1.0 - rng.integers(1600, 1900, (4, 4)) * DELTA + 0.5 * DELTA
    sc["occ"][..., 0] = lo.astype(np.float32)
    sc["occ"][..., 1] = (lo + rng.integers(5, 60, (4, 4)) * DELTA).astype(np.float32)
    o = np.column_stack([rng.uniform(-0.95, 0.95, (40, 2)), np.ones(40)]).astype(np.float32)
    d = np.tile(_f32([0, 0, -1]), (40, 1))
    hard = oracle.oracle_render(sc, o, d, oracle.RenderParams(n_max=128, c_bg=(0.1, 0.2, 0.3)))
    soft = oracle.oracle_render(sc, o, d, oracle.RenderParams(n_max=128, c_bg=(0.1, 0.2, 0.3),
                                                              occ_eps=0.25 * DELTA))
    assert (hard["n_placed"] > 0).all()
    for key in ("C", "F", "T"):
        np.testing.assert_array_equal(soft[key], hard[key])


def test_soft_mask_occupancy_gradient_matches_fd():
    """dL/dz_min and dL/dz_max (through M only: placement is piecewise
    constant in the bounds) against float64 central differences that keep
    every placement unchanged."""
    sc, o, d, tgt = _grad_problem(seed=2)
    rng = np.random.default_rng(7)
    sc["occ"][..., 0] = rng.uniform(0.02, 0.08, (4, 4)).astype(np.float32)
    sc["occ"][..., 1] = rng.uniform(0.12, 0.2, (4, 4)).astype(np.float32)
    prm = oracle.RenderParams(n_max=256, c_bg=(0.2, 0.4, 0.6), occ_eps=0.03)
    _, _, grads = oracle.oracle_loss_and_grads(sc, o, d, prm, tgt)
    cells, g = grads["occ"]
    assert np.abs(g).max() > 0
    h = 1e-8
    checked = 0
    for ci, cell in enumerate(cells):
        for b in (0, 1):
            vals, counts = [], []
            for s in (+1, -1):
                sp = dict(sc)
                occ = sc["occ"].astype(np.float64).copy()
                occ.reshape(-1, 2)[cell, b] += s * h
                sp["occ"] = occ
                r = oracle.oracle_render(sp, o, d, prm)
                vals.append(np.mean((r["C"] - tgt) ** 2))
                counts.append(r["n_placed"])
            if not np.array_equal(counts[0], counts[1]):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g[ci, b]) <= 1e-5 * max(abs(fd), 1e-4) + 1e-9, (cell, b, fd, g[ci, b])
            checked += 1
    assert checked >= 8


def test_occ_interval_loss_hand_example():
    """Eq. 5 on a 2 x 2 plane: spans 0.1, 0.2, 0, -0.05 (an empty cell)."""
    occ = np.array([[[0.0, 0.1], [0.1, 0.3]], [[0.2, 0.2], [0.15, 0.1]]])
    loss, grad = oracle.occ_interval_loss(occ)
    assert loss == pytest.approx(0.01 + 0.04 + 0.0 + 0.0025, rel=1e-12)
    np.testing.assert_allclose(grad[..., 1], [[0.2, 0.4], [0.0, -0.1]], atol=1e-15)
    np.testing.assert_allclose(grad[..., 0], [[-0.2, -0.4], [0.0, 0.1]], atol=1e-15)


# ---------------------------------------------------------------------------
# View-direction encoding and view-smoothness loss (Sec. 4.2, Eq. 9-10)
# ---------------------------------------------------------------------------

def test_direction_encoding_hand_values():
    """Four frequencies (the paper's deferred MLP, as in MERF): [d, sin(2^k d),
    cos(2^k d)] for k = 0..3, 27 values, at a hand-checked direction."""
    d = torch.tensor([[0.6, 0.0, -0.8]], dtype=torch.float64)
    e = oracle.encode_dir(d, 4).numpy()[0]
    assert e.shape == (27,)
    np.testing.assert_allclose(e[:3], [0.6, 0.0, -0.8], rtol=0, atol=0)
    np.testing.assert_allclose(e[3:6], [math.sin(0.6), 0.0, math.sin(-0.8)], rtol=1e-15)
    np.testing.assert_allclose(e[6:9], [math.cos(0.6), 1.0, math.cos(-0.8)], rtol=1e-15)
    np.testing.assert_allclose(e[21:24], [math.sin(4.8), 0.0, math.sin(-6.4)], rtol=1e-14)
    np.testing.assert_allclose(e[24:27], [math.cos(4.8), 1.0, math.cos(-6.4)], rtol=1e-14)


def _dir_mlp(n_in):
    """An MLP that reads only the view direction's x through one hidden path:
    h1_0 = relu(2 d_x + 0.5), h2_0 = relu(h1_0), G = sigmoid(h2_0 - 1) on all
    three outputs."""
    w1 = np.zeros((16, n_in))
    w1[0, 7] = 2.0
    b1 = np.zeros(16)
    b1[0] = 0.5
    w2 = np.zeros((16, 16))
    w2[0, 0] = 1.0
    w3 = np.zeros((3, 16))
    w3[:, 0] = 1.0
    b3 = np.full(3, -1.0)
    return np.concatenate([w1.ravel(), b1, w2.ravel(), np.zeros(16), w3.ravel(), b3])


def test_smooth_loss_hand_example():
    """One ray, two perturbations: L = sum_p cos(d, s_p) * 3 (G(s_p) - G(d))^2
    with G(v) = sigmoid(relu(2 v_x + 0.5) - 1), worked out by hand."""
    F = np.zeros((1, 7))
    d = np.array([[0.0, 0.0, -1.0]])
    pert = np.array([[[0.3, 0.0, 0.0], [-0.1, 0.2, 0.0]]])
    sig = lambda x: 1 / (1 + math.exp(-x))  # noqa: E731
    g = lambda vx: sig(max(2 * vx + 0.5, 0.0) - 1.0)  # noqa: E731
    want = 0.0
    for dx, dy, dz in pert[0]:
        s = np.array([dx, dy, -1.0 + dz])
        cos = -s[2] / np.linalg.norm(s)
        want += cos * 3 * (g(s[0]) - g(0.0)) ** 2
    loss, gF, gW = oracle.smooth_loss(F, d, pert, _dir_mlp(10), freqs=0, weight=1.0)
    assert loss == pytest.approx(want, rel=1e-13)
    np.testing.assert_allclose(gF, 0.0, atol=0)  # F enters only weights that are zero
    assert np.abs(gW).max() > 0


def test_smooth_loss_zero_cases():
    """No perturbation, or an MLP blind to the direction: L = 0 and no gradient."""
    rng = np.random.default_rng(3)
    F = rng.normal(size=(5, 7))
    d = rng.normal(size=(5, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mlp = rng.normal(0, 0.4, 16 * 34 + 339)
    loss, gF, gW = oracle.smooth_loss(F, d, np.zeros((5, 3, 3)), mlp, freqs=4)
    assert loss == 0.0 and not gF.any() and not gW.any()
    blind = mlp.copy()
    blind[:16 * 34].reshape(16, 34)[:, 7:] = 0.0
    loss, gF, gW = oracle.smooth_loss(F, d, rng.normal(0, 0.3, (5, 3, 3)), blind, freqs=4)
    assert loss == 0.0


@pytest.mark.parametrize("freqs", [0, 4])
def test_smooth_loss_gradient_matches_fd(freqs):
    rng = np.random.default_rng(8)
    n_in = 7 + 3 * (1 + 2 * freqs)
    F = rng.uniform(0, 1, (6, 7))
    d = rng.normal(size=(6, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pert = rng.normal(0, 0.3, (6, 4, 3))
    mlp = rng.normal(0, 0.5, 16 * n_in + 339)
    loss, gF, gW = oracle.smooth_loss(F, d, pert, mlp, freqs=freqs, weight=0.7)
    h = 1e-6
    for arr, g, picks in ((F, gF, [(0, 0), (3, 5), (5, 6)]), (mlp, gW, [(i,) for i in rng.choice(mlp.size, 8, replace=False)])):
        for idx in picks:
            vals = []
            for s in (+1, -1):
                a = arr.copy()
                a[idx] += s * h
                args = (a, d, pert, mlp) if arr is F else (F, d, pert, a)
                vals.append(oracle.smooth_loss(*args, freqs=freqs, weight=0.7)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(abs(fd), 1e-3), (idx, fd, g[idx])


def test_loss_with_smooth_term_is_l2_plus_smooth_of_rendered_features():
    """oracle_loss_and_grads(smooth=...) is the L2 loss plus smooth_loss on
    the rendered F (values), and its gradient in a feature row and in MLP
    entries matches central differences of that sum (the F path of the
    smoothness term reaches the features)."""
    sc, o, d, tgt = _grad_problem()
    prm = oracle.RenderParams(n_max=256, c_bg=(0.2, 0.4, 0.6))
    rng = np.random.default_rng(4)
    pert = rng.normal(0, 0.5, (o.shape[0], 3, 3))
    w = 0.3

    def total(s):
        r = oracle.oracle_render(s, o, d, prm, keep_k=False)
        return np.mean((r["C"] - tgt) ** 2) + oracle.smooth_loss(r["F"], d, pert, s["mlp"], 0, w)[0]

    loss, _, grads = oracle.oracle_loss_and_grads(sc, o, d, prm, tgt, smooth=dict(perturb=pert, weight=w))
    plain, _, plain_grads = oracle.oracle_loss_and_grads(sc, o, d, prm, tgt)
    assert abs(loss - total(sc)) <= 1e-12 * abs(loss) and loss > plain
    u, g = grads["grid"]
    gp = dict(zip(plain_grads["grid"][0].tolist(), plain_grads["grid"][1]))
    row = int(np.argmax(np.abs(g - np.stack([gp[int(k)] for k in u])).sum(1)))
    picks = [("grid", int(u[row]) * 8 + c) for c in range(8)] + [("mlp", int(i)) for i in rng.choice(499, 6, replace=False)]
    h = 1e-6
    for src, e in picks:
        gdense = grads["mlp"][e] if src == "mlp" else g[row, e % 8]
        vals = []
        for s in (+1, -1):
            sp = {k: (v.astype(np.float64).copy() if k == src else v) for k, v in sc.items()}
            sp[src].reshape(-1)[e] += s * h
            vals.append(total(sp))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gdense) <= 1e-6 * max(abs(fd), 1e-3), (src, e, fd, gdense)


# ---------------------------------------------------------------------------
# 8-bit feature storage (Sec. 4.4): code decision, parameters, round trip.
# ---------------------------------------------------------------------------
def test_quantize_u8_hand_values():
    """lo = -1, step = 0.5 (inv = 2): codes by hand, ties to even, clamping."""
    lo = np.full(8, -1.0, np.float32)
    step = np.full(8, 0.5, np.float32)
    x = np.array([-1.0, -0.75, -0.25, 0.0, 126.5, 126.25, 200.0, -5.0], np.float32)
    # (x + 1) * 2 = 0, 0.5, 1.5, 2, 255, 254.5, 402, -8
    want = np.array([0, 0, 2, 2, 255, 254, 255, 0], np.uint8)
    got = oracle.quantize_u8(np.tile(x[:, None], (1, 8)), lo, step)
    assert (got == want[:, None]).all()
    special = np.array([np.nan, np.inf, -np.inf, 0.0, 0, 0, 0, 0], np.float32)[None, :]
    assert oracle.quantize_u8(special, lo, step)[0, :3].tolist() == [0, 255, 0]


def test_quant_params_span_the_range():
    """lo = min and step = (max - min)/255: the channel's minimum encodes as 0
    and its maximum as 255; a constant channel has step 0 and decodes exactly."""
    rng = np.random.default_rng(0)
    x = (rng.standard_normal((500, 8)) * 0.5).astype(np.float32)
    x[:, 5] = 0.375
    mm = oracle.feature_range(x)
    assert np.array_equal(mm[:, 0], x.min(0)) and np.array_equal(mm[:, 1], x.max(0))
    lo, step = oracle.quant_params(mm)
    assert step[5] == 0.0 and np.allclose(step[:5], (x.max(0) - x.min(0))[:5] / 255.0, rtol=1e-6)
    q = oracle.quantize_u8(x, lo, step)
    for c in range(8):
        if c == 5:
            assert (q[:, c] == 0).all() and (oracle.dequantize(q[:, c], lo[c], step[c]) == 0.375).all()
            continue
        assert q[np.argmin(x[:, c]), c] == 0 and q[np.argmax(x[:, c]), c] == 255


def test_quantize_round_trip_within_half_step():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal((4000, 8)) * 0.7).astype(np.float32)
    lo, step = oracle.quant_params(oracle.feature_range(x))
    err = np.abs(oracle.dequantize(oracle.quantize_u8(x, lo, step), lo, step) - x)
    assert (err <= 0.5 * step.astype(np.float64) * (1 + 1e-5) + 1e-12).all()
    # codes are fixed points: decoding a code and encoding it again returns it
    q = rng.integers(0, 256, (300, 8)).astype(np.uint8)
    back = oracle.quantize_u8(oracle.dequantize(q, lo, step).astype(np.float32), lo, step)
    assert np.array_equal(back, q)


def test_u8_scene_render_is_render_of_decoded_scene():
    """Features that sit exactly on the codes of lo = -2, step = 2^-6 (each
    channel holding both end codes, so the ranges give back these
    parameters) survive the 8-bit scene round trip bit for bit, and the
    render of the 8-bit scene equals the float render exactly."""
    import scenegen
    sc = micro_scene(grid=(5, 4, 3), planes=(7, 6, 5), m=4, zmin=0.02, zmax=0.2)
    rng = np.random.default_rng(3)
    for src in oracle.quant.SOURCES:
        q = rng.integers(0, 256, sc[src].shape)
        q.reshape(-1, 8)[0], q.reshape(-1, 8)[1] = 0, 255
        sc[src] = (-2.0 + q * 2.0 ** -6).astype(np.float32)
    sc["grid"][..., 0] += np.float32(3.0)  # still on the codes of its own range (lo = 1)
    q8 = oracle.quantize_scene(sc)
    assert np.array_equal(q8["quant_step"], np.full((4, 8), 2.0 ** -6, np.float32))
    dec = oracle.dequantize_scene(q8)
    for src in oracle.quant.SOURCES:
        assert q8[src].dtype == np.uint8 and np.array_equal(dec[src], sc[src].astype(np.float64)), src
    o, d = scenegen.oblique_rays(24, seed=4, origin_z=0.6)
    prm = oracle.RenderParams(n_max=256, c_bg=(0.2, 0.4, 0.6))
    a = oracle.oracle_render(dec, o, d, prm, keep_k=False)
    b = oracle.oracle_render(sc, o, d, prm, keep_k=False)
    assert np.array_equal(a["C"], b["C"]) and (a["n_placed"] > 0).sum() > 10


# ---------------------------------------------------------------------------
# Upstream-gradient form and the float32 error scale of the gradient
# ---------------------------------------------------------------------------

def test_upstream_form_is_the_l2_gradient():
    """With upstream = dL/dC of the L2 loss, 2 (C - C*)/(3n), the linear
    functional sum(upstream * C) has the L2 loss's gradient."""
    sc, o, d, tgt = _grad_problem(seed=2)
    prm = oracle.RenderParams(n_max=256, c_bg=(0.2, 0.4, 0.6))
    _, C, g_l2 = oracle.oracle_loss_and_grads(sc, o, d, prm, tgt)
    up = 2.0 * (C - tgt) / (3.0 * o.shape[0])
    _, _, g_up = oracle.oracle_loss_and_grads(sc, o, d, prm, upstream=up)
    for src in ("grid", "plane_xy", "plane_xz", "plane_yz"):
        assert np.array_equal(g_l2[src][0], g_up[src][0])
        np.testing.assert_allclose(g_up[src][1], g_l2[src][1], rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(g_up["mlp"], g_l2["mlp"], rtol=1e-12, atol=1e-18)
    with pytest.raises(ValueError):
        oracle.oracle_loss_and_grads(sc, o, d, prm, tgt, upstream=up)


def _bound_problem(eps=0.0, freqs=0, t_term=0.0, seed=5):
    import scenegen
    sc = micro_scene(grid=(6, 5, 4), planes=(9, 8, 6), m=4, zmin=0.02, zmax=0.2, seed=seed, std=0.7)
    sc["grid"][..., 0] += 3.0
    if freqs:
        sc["mlp"] = (np.random.default_rng(seed).standard_normal(883) * 0.3).astype(np.float32)
        sc["dir_freqs"] = freqs
    o, d = scenegen.oblique_rays(32, seed=seed + 10, origin_z=0.6)
    up = np.random.default_rng(seed + 1).standard_normal((32, 3)) * 1e-2
    prm = oracle.RenderParams(n_max=256, c_bg=(0.25, -0.5, 0.75), occ_eps=eps, t_term=t_term)
    return sc, o, d, up, prm


@pytest.mark.parametrize("eps,freqs", [(0.0, 0), (0.02, 0), (0.0, 4)])
def test_error_scale_bounds_every_entry(eps, freqs):
    """Triangle inequality: the sum of absolute terms A_e is at least the
    magnitude of the entry, for every entry of every tensor (soft occupancy,
    smoothness term and a c_bg with a negative channel included); B >= 64 A
    (every term carries at least 64 roundings)."""
    from oracle.fp32_bound import gradient_error_scale
    sc, o, d, up, prm = _bound_problem(eps, freqs)
    smooth = None
    if freqs:
        import scenegen
        smooth = dict(perturb=scenegen.view_perturbations(o.shape[0], 3, seed=9), weight=0.1)
    _, _, g = oracle.oracle_loss_and_grads(sc, o, d, prm, upstream=up, smooth=smooth)
    es = gradient_error_scale(sc, o, d, prm, up, smooth=smooth)
    keys = ["grid", "plane_xy", "plane_xz", "plane_yz"] + (["occ"] if eps > 0 else [])
    for k in keys:
        u, rows = g[k]
        u2, A, B, N = es[k]
        assert np.array_equal(u, u2), k
        assert np.all(np.abs(rows) <= A * (1 + 1e-12) + 1e-300), k
        assert np.all(B >= 64 * A * (1 - 1e-12)), k
        assert np.all(N >= 1), k
    A, B, N = es["mlp"]
    assert np.all(np.abs(g["mlp"]) <= A * (1 + 1e-12) + 1e-300)
    assert N == (o.shape[0] + (2 * o.shape[0] * 3 if freqs else 0))


def test_error_scale_keeps_cancelled_terms():
    """Constant density and colour, zero-weight MLP and c_bg equal to the
    diffuse colour: dL/da_i = T_{i+1} gv - sum_{k>i} w_k gv - T_n gT
    = T_n (gv - gT) = 0, so the channel-0 gradient cancels exactly, while
    its terms (and A) do not vanish."""
    from oracle.fp32_bound import gradient_error_scale
    c = 0.3
    sc = _constant_density_scene(60.0, c, [0.1, 0.2, 0.3])
    s = 1 / (1 + math.exp(-float(np.float32(c))))
    prm = oracle.RenderParams(n_max=1024, c_bg=(s, s, s))
    o = _f32([[0.1, 0.1, 1.0], [-0.5, 0.6, 1.0]])
    d = np.tile(_f32([0, 0, -1]), (2, 1))
    up = np.array([[0.3, -0.2, 0.5], [0.1, 0.4, -0.7]])
    _, _, g = oracle.oracle_loss_and_grads(sc, o, d, prm, upstream=up)
    _, A, _, _ = gradient_error_scale(sc, o, d, prm, up)["grid"]
    g0 = g["grid"][1][:, 0]
    assert A[:, 0].min() > 0
    assert np.abs(g0).max() <= 1e-9 * A[:, 0].max()


def test_error_scale_counts_evaluated_incidences():
    """N_e sums to (evaluated samples) x (corners per sample) per source; with
    early termination the placed-but-unevaluated samples do not count."""
    from oracle.fp32_bound import gradient_error_scale
    sc, o, d, up, prm = _bound_problem(t_term=0.05)
    r = oracle.oracle_render(sc, o, d, prm, keep_k=False)
    assert r["n_eval"].sum() < r["n_placed"].sum()
    es = gradient_error_scale(sc, o, d, prm, up)
    for k, corners in (("grid", 8), ("plane_xy", 4), ("plane_xz", 4), ("plane_yz", 4)):
        assert es[k][3].sum() == corners * r["n_eval"].sum(), k


def test_error_scale_covers_float32_underflow():
    """Far behind a dense medium the transmittance falls below the binary32
    range: with a = 9 per sample (tau = 9 / delta) T_s = exp(-9 s) is below
    2^-100 from the 8th sample on.  A grid of 32 cells in z (16 samples per
    cell) has vertices that only such samples reach; their float64 gradient
    is nonzero but made of terms below 2^-80, which a float32 backward may
    flush to zero.  The floor u (B + N A) must cover those entries whole,
    and must not add the underflow allowance to entries of ordinary size."""
    import oracle.fp32_bound as fb
    from oracle.fp32_bound import U32, gradient_error_scale
    sc = micro_scene(grid=(4, 4, 33), planes=(6, 6, 5), zmin=0.0, zmax=0.25, seed=11, std=0.2)
    sc["grid"][..., 0] = np.float32(math.log(9.0 / DELTA))
    prm = oracle.RenderParams(n_max=1024, c_bg=(0.25, 0.5, 0.75))
    o, d = _f32([[0.13, -0.21, 1.0], [-0.4, 0.35, 1.0]]), np.tile(_f32([0, 0, -1]), (2, 1))
    up = np.array([[0.3, -0.2, 0.5], [0.1, 0.4, -0.7]])
    _, _, g = oracle.oracle_loss_and_grads(sc, o, d, prm, upstream=up)
    idx, A, B, N = gradient_error_scale(sc, o, d, prm, up)["grid"]
    rows = g["grid"][1]
    tiny = (A > 0) & (A < 2.0 ** -80)
    big = A > 2.0 ** -60
    assert tiny.sum() >= 8 and big.sum() >= 8
    fl = U32 * (B + N[:, None] * A)
    assert np.all(fl[tiny] >= np.abs(rows[tiny]))
    keep = fb.TINY_TERM
    try:
        fb.TINY_TERM = 0.0
        _, _, B0, _ = gradient_error_scale(sc, o, d, prm, up)["grid"]
    finally:
        fb.TINY_TERM = keep
    # the allowance adds at most 2^-80 / u per term, nothing of note to an ordinary entry
    Nc = np.broadcast_to(N[:, None], B.shape)
    assert np.all(B[big] - B0[big] <= Nc[big] * 2.0 ** -80 / U32)
    assert np.all(B[tiny] > B0[tiny])


def test_error_scale_input_errors_bound_a_perturbed_mlp():
    """The MLP-input error model against brute force in float64: (1) the
    encoded direction of s = fl32(d + delta) differs from that of the exact
    d + delta by at most the modelled input error less the sincos allowance;
    (2) moving every input by its modelled error, with random signs, moves
    z3 = W3 relu(W2 relu(W1 x + b1) + b2) + b3 by at most the propagated
    bound e_z3 (rows whose ReLU pattern does not change)."""
    from oracle.fp32_bound import SINCOS_ERR, U32, _input_abs_err, _input_err_coeffs, _mlp_abs
    from oracle.render import encode_dir, unpack_mlp
    rng = np.random.default_rng(21)
    n, freqs = 512, 4
    d = rng.standard_normal((n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    pert = (rng.standard_normal((n, 3)) * 0.3).astype(np.float32)
    s32 = (d + pert).astype(np.float64)  # float32 addition, as on the GPU
    s64 = d.astype(np.float64) + pert.astype(np.float64)
    raw = U32 * np.abs(s32)
    F = rng.uniform(0.0, 1.0, (n, 7))
    x64 = np.concatenate([F, encode_dir(torch.from_numpy(s64), freqs).numpy()], 1)
    x32 = np.concatenate([F, encode_dir(torch.from_numpy(s32), freqs).numpy()], 1)
    e_x = _input_abs_err(x32, raw, freqs)
    assert np.all(np.abs(x32 - x64)[:, 7:] <= (e_x - np.where(np.arange(34) >= 10, SINCOS_ERR, 0.0))[:, 7:] * (1 + 1e-9))
    mlp = (rng.standard_normal(883) * 0.4).astype(np.float64)
    fw = _mlp_abs(mlp, x32)
    _, ez3 = _input_err_coeffs(fw, e_x)
    w1, b1, w2, b2, w3, b3 = [t.numpy() for t in unpack_mlp(torch.from_numpy(mlp))]

    def fwd(x):
        z1 = x @ w1.T + b1
        z2 = np.maximum(z1, 0.0) @ w2.T + b2
        return np.maximum(z2, 0.0) @ w3.T + b3, np.concatenate([z1 > 0, z2 > 0], 1)

    z0, pat0 = fwd(x32)
    checked = 0
    for _ in range(32):
        sign = rng.choice([-1.0, 1.0], size=x32.shape)
        z, pat = fwd(x32 + sign * e_x)
        keep = np.all(pat == pat0, axis=1)
        checked += int(keep.sum())
        assert np.all(np.abs(z - z0)[keep] <= U32 * ez3[keep] * (1 + 1e-9) + 1e-300)
    assert checked >= 32 * n * 0.9


def test_error_scale_weight_error_bounds_perturbed_fractions():
    """The interpolation-weight term against brute force: moving every 1-D
    factor (f and 1 - f of each axis) by +-FRAC_ERR u with random signs
    changes each corner's weight (the product of its factors, Eq. 2) by at
    most FRAC_ERR u omega_c (first order; the products of two or three
    perturbations add at most 4 (FRAC_ERR u)^2), for the trilinear grid and
    the three planes."""
    from oracle.field import feature_terms
    from oracle.fp32_bound import FRAC_ERR, U32, _other_axis_weights
    rng = np.random.default_rng(31)
    sc = micro_scene(grid=(9, 7, 5), planes=(13, 11, 6))
    p = np.stack([rng.uniform(-1, 1, 4000), rng.uniform(-1, 1, 4000), rng.uniform(0, 0.25, 4000)], 1)
    p[:50, 0] = -1.0 + 2.0 * 3 / 12 + rng.uniform(-1e-7, 1e-7, 50)  # samples next to a vertex plane
    dims_g = (9, 7, 5)
    dims_p = (13, 11, 6)
    om = _other_axis_weights(p, sc)
    terms = feature_terms(p, BOX_LO, BOX_HI, dims_g, dims_p)
    e = FRAC_ERR * U32
    for _ in range(16):
        sg = rng.choice([-1.0, 1.0], size=(p.shape[0], 3, 2))  # axis, (1 - f, f)

        def fac(axis, n, side):
            u = (p[:, axis] - BOX_LO[axis]) / (BOX_HI[axis] - BOX_LO[axis]) * (n - 1)
            f = u - np.clip(np.floor(u), 0, n - 2)
            return (f if side else 1.0 - f) + sg[:, axis, side] * e

        for c in range(8):
            dx, dy, dz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            w = fac(0, 9, dx) * fac(1, 7, dy) * fac(2, 5, dz)
            assert np.all(np.abs(w - terms["grid"][1][:, c]) <= e * om["grid"][:, c] * (1 + 1e-9) + 4 * e * e)
        for src, (a0, n0), (a1, n1) in (("plane_xy", (0, 13), (1, 11)), ("plane_xz", (0, 13), (2, 6)),
                                         ("plane_yz", (1, 11), (2, 6))):
            for c in range(4):
                w = fac(a0, n0, c & 1) * fac(a1, n1, (c >> 1) & 1)
                assert np.all(np.abs(w - terms[src][1][:, c]) <= e * om[src][:, c] * (1 + 1e-9) + 4 * e * e)


def test_error_scale_fraction_slopes_bound_a_perturbed_field():
    """The interpolated t of Eq. 2 against brute force: moving every 1-D
    factor by +-FRAC_ERR u (random signs) moves t by at most FRAC_ERR u
    times the modelled slope sum_axes |dt/df_a| per channel (first order,
    plus the products of two perturbations)."""
    from oracle.field import feature_terms
    from oracle.fp32_bound import FRAC_ERR, U32, _fraction_slopes
    rng = np.random.default_rng(41)
    sc = micro_scene(grid=(9, 7, 5), planes=(13, 11, 6), seed=41, std=0.7)
    p = np.stack([rng.uniform(-1, 1, 3000), rng.uniform(-1, 1, 3000), rng.uniform(0, 0.25, 3000)], 1)
    dims = {"grid": (9, 7, 5), "plane_xy": (13, 11), "plane_xz": (13, 6), "plane_yz": (11, 6)}
    axes = {"grid": (0, 1, 2), "plane_xy": (0, 1), "plane_xz": (0, 2), "plane_yz": (1, 2)}
    terms = feature_terms(p, BOX_LO, BOX_HI, (9, 7, 5), (13, 11, 6))
    slopes = _fraction_slopes(p, sc, {k: terms[k][0] for k in terms})
    e = FRAC_ERR * U32

    def t_of(sign):
        t = np.zeros((p.shape[0], 8))
        for src, ax in axes.items():
            tab = np.asarray(sc[src], dtype=np.float64).reshape(-1, 8)
            idx = terms[src][0]
            fac = []
            for j, a in enumerate(ax):
                n = dims[src][j]
                u = (p[:, a] - BOX_LO[a]) / (BOX_HI[a] - BOX_LO[a]) * (n - 1)
                f = u - np.clip(np.floor(u), 0, n - 2)
                s_ = sign[:, a]
                fac.append((1.0 - f - s_ * e, f + s_ * e))
            for c in range(1 << len(ax)):
                w = np.ones(p.shape[0])
                for j in range(len(ax)):
                    w = w * fac[j][(c >> j) & 1]
                t += w[:, None] * tab[idx[:, c]]
        return t

    t0 = t_of(np.zeros((p.shape[0], 3)))
    tab_max = max(np.abs(np.asarray(sc[k])).max() for k in axes)
    for _ in range(16):
        dt = np.abs(t_of(rng.choice([-1.0, 1.0], size=(p.shape[0], 3))) - t0)
        assert np.all(dt <= e * slopes * (1 + 1e-9) + 64 * e * e * tab_max)
