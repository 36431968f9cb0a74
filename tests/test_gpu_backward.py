"""GPU backward: gradients into grid, planes and MLP against the float64
oracle gradient and against central finite differences of the GPU forward.

Oracle parity (tests/gradcheck.py): both sides take the same float32 dL/dC
(the oracle's L2 gradient), and every entry must satisfy
|g - g_oracle| <= 1e-3 |g_oracle| + u (B_e + N_e A_e), the 1e-3 relative bar
plus the float32 rounding floor of the entry's own terms.  Finite
differences (float64 loss reduction on the GPU) within
|g - g_fd| <= 1e-3 max(|g_fd|, 1e-2 RMS of the checked entries), on 64
entries stratified over the five tensors and over magnitude, plus 4 entries
with zero gradient.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2404_09531_amd as om
import scenegen
from tests._scenes import micro_scene
from tests.gpu_util import log, rays_to, upload_scene
from tests.gradcheck import check, oracle_reference, oracle_upstream

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)
SOURCES = ("grid", "plane_xy", "plane_xz", "plane_yz")


def _gpu_grads(scene, t, og, dg, target, n_max, t_term=0.0, batch_wv=False):
    res = om.render(scene, og, dg, n_max=n_max, c_bg=BG, t_term=t_term, batch_wv=batch_wv)
    dC, loss = om.l2_loss_grad(res["C"], target)
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}
    om.render_backward(scene, og, dg, res, dC, grads, n_max=n_max, c_bg=BG, t_term=t_term)
    torch.cuda.synchronize()
    return res, loss.item(), {k: v.double().cpu().numpy() for k, v in grads.items()}


def _gpu_vjp(scene, t, og, dg, up32, n_max, t_term=0.0, batch_wv=False, occ_eps=0.0, mlp_bf16=0, dL_dF=None):
    """GPU forward (saving F, T, n_eval) and backward for the given float32
    dL/dC (numpy [n, 3]); returns (forward outputs, numpy gradients)."""
    kw = dict(n_max=n_max, c_bg=BG, t_term=t_term, occ_eps=occ_eps)
    res = om.render(scene, og, dg, mlp_bf16=mlp_bf16, batch_wv=batch_wv, **kw)
    dC = torch.from_numpy(np.ascontiguousarray(up32, np.float32)).to(og.device)
    keys = (*SOURCES, "mlp") + (("occ",) if occ_eps > 0 else ())
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in keys}
    om.render_backward(scene, og, dg, res, dC, grads, dL_dF=dL_dF, **kw)
    torch.cuda.synchronize()
    return res, {k: v.double().cpu().numpy() for k, v in grads.items()}


def _loss_check(res, tg, ref_loss, tag):
    loss = om.l2_loss_fp64(res["C"], tg).item()
    log(f"  [{tag}] loss {loss:.9e}, oracle {ref_loss:.9e}, rel {abs(loss - ref_loss) / ref_loss:.2e}")
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss


@pytest.fixture(scope="module")
def tiny_train():
    sc = scenegen.make_scene(scenegen.TINY)
    pert = scenegen.perturb_scene(sc, 0.05, seed=2)
    o, d = scenegen.oblique_rays(256, seed=3)
    prm = oracle.RenderParams(n_max=64, c_bg=BG)
    target = oracle.oracle_render(pert, o, d, prm, keep_k=False)["C"]
    scene, t = upload_scene(sc)
    return sc, scene, t, o, d, target


def test_backward_tiny_vs_oracle(tiny_train):
    sc, scene, t, o, d, target = tiny_train
    log("test_backward_tiny_vs_oracle: 256 rays")
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target.astype(np.float32)).to(og.device)
    prm = oracle.RenderParams(n_max=64, c_bg=BG)
    up, ref_loss = oracle_upstream(sc, o, d, prm, target.astype(np.float32))
    ref, scale = oracle_reference(sc, o, d, prm, up)
    for bw in (False, True):  # batch totals from a replay / from the forward's per-batch sums
        res, grads = _gpu_vjp(scene, t, og, dg, up, 64, batch_wv=bw)
        _loss_check(res, tg, ref_loss, f"tiny batch_wv={bw}")
        check(grads, ref, scale, f"tiny batch_wv={bw}")


def _backward_plain_direct(scene, t, og, dg, res, up32, n_max):
    """om_render_backward (no dL/dF) called through the C ABI, with a
    workspace of exactly the queried size; the binding uses
    om_render_backward_ex."""
    from paper_2404_09531_amd import _lib
    L = _lib.lib()
    n = og.shape[0]
    dC = torch.from_numpy(np.ascontiguousarray(up32, np.float32)).to(og.device)
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}
    ws = torch.empty((L.om_render_backward_workspace_size(n),), dtype=torch.uint8, device=og.device)
    fo = _lib.OmFwdOut(res["C"].data_ptr(), res["T"].data_ptr(), res["F"].data_ptr(), res["n_placed"].data_ptr(),
                       res["n_eval"].data_ptr(), 0)
    p = om._params(n_max, om.DELTA, 0.0, BG, -1, 0.0)
    g = om._grads(scene, grads)
    rc = L.om_render_backward(scene.handle, og.data_ptr(), dg.data_ptr(), n, ctypes.byref(p), ctypes.byref(fo),
                              dC.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.byref(g), _lib.stream_of(og))
    assert rc == 0, L.om_last_error().decode()
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in grads.items()}


@pytest.mark.parametrize("n", [1, 3, 6, 1037])
def test_backward_ragged_counts_vs_oracle(tiny_train, n):
    """Ray counts that leave a partial quad of rays in the MLP backward's
    last step, with every fourth ray turned upwards out of the box
    (n_eval = 0: no sample and no MLP term): gradients against the oracle,
    through om_render_backward_ex (the binding) and om_render_backward."""
    sc, scene, t, _, _, _ = tiny_train
    log(f"test_backward_ragged_counts_vs_oracle: {n} rays")
    o, d = scenegen.oblique_rays(n, seed=11)
    away = np.arange(n) % 4 == 1
    d = d.copy()
    d[away, 2] = -d[away, 2]  # from z = 1 upwards: never enters the box
    g = np.random.Generator(np.random.PCG64(12))
    target = g.uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    prm = oracle.RenderParams(n_max=64, c_bg=BG)
    up, _ = oracle_upstream(sc, o, d, prm, target)
    ref, scale = oracle_reference(sc, o, d, prm, up)
    og, dg = rays_to(o, d)
    res, grads = _gpu_vjp(scene, t, og, dg, up, 64)
    ne = res["n_eval"].cpu().numpy()
    assert (ne[away] == 0).all() and (ne[~away] > 0).any()
    check(grads, ref, scale, f"ragged n={n}")
    check(_backward_plain_direct(scene, t, og, dg, res, up, 64), ref, scale, f"ragged n={n}, om_render_backward")


def test_backward_max_samples_vs_oracle():
    """Rays with up to n_max = 1024 samples (64 batches, every register
    slot of the batch totals): a box of height 0.5 that the occupancy
    fills, low density so that every sample keeps a share of the
    transmittance, near-vertical and oblique rays.  Gradients against the
    oracle, with the batch totals from a replay and from the forward."""
    sc = micro_scene(grid=(8, 8, 12), planes=(16, 16, 20), m=4, zmin=0.0, zmax=0.5, seed=31, std=0.5)
    sc["box_hi"][2] = 0.5
    g = np.random.Generator(np.random.PCG64(32))
    n = 37
    d = np.stack([g.uniform(-0.3, 0.3, n), g.uniform(-0.3, 0.3, n), -np.ones(n)], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.stack([g.uniform(-0.5, 0.5, n), g.uniform(-0.5, 0.5, n), np.ones(n)], axis=1)
    o, d = o.astype(np.float32), d.astype(np.float32)
    target = g.uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    prm = oracle.RenderParams(n_max=1024, c_bg=BG)
    up, _ = oracle_upstream(sc, o, d, prm, target)
    ref, scale = oracle_reference(sc, o, d, prm, up)
    scene, t = upload_scene(sc)
    og, dg = rays_to(o, d)
    for bw in (False, True):
        res, grads = _gpu_vjp(scene, t, og, dg, up, 1024, batch_wv=bw)
        ne = res["n_eval"].cpu().numpy()
        log(f"test_backward_max_samples_vs_oracle: batch_wv={bw}, samples per ray {ne.min()}..{ne.max()}")
        assert ne.max() > 768  # the last register slot of the batch totals is used
        check(grads, ref, scale, f"max samples batch_wv={bw}")


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_batch_wv_prefixes_match_truncated_oracle_renders(tiny_train, dtype):
    """The forward's per-batch sums of w v, accumulated over the first b + 1
    batches of 16 samples, equal F of the oracle render truncated to
    n_max = 16 (b + 1): truncation keeps exactly the first samples."""
    sc, _, _, o, d, _ = tiny_train
    log(f"test_batch_wv_prefixes_match_truncated_oracle_renders: {dtype}")
    scene, _ = upload_scene(sc, dtype=dtype)
    ref_sc = sc if dtype == torch.float32 else _rounded_scene(sc)
    og, dg = rays_to(o, d)
    res = om.render(scene, og, dg, n_max=64, c_bg=BG, mlp_bf16=0, batch_wv=True)
    bw = res["batch_wv"].double().cpu().numpy()
    ne = res["n_eval"].cpu().numpy()
    cum = np.cumsum(bw, axis=1)
    for b in range(om.batch_slots(64)):
        ref = oracle.oracle_render(ref_sc, o, d, oracle.RenderParams(n_max=16 * (b + 1), c_bg=BG), keep_k=False)
        live = ne > 16 * b  # rays whose slot b was written
        assert live.any()
        err = np.abs(cum[live, b] - ref["F"][live]).max()
        log(f"  batches 0..{b}: {live.sum()} rays, max |sum - F_oracle(n_max={16 * (b + 1)})| = {err:.2e}")
        assert err <= 1e-5
    assert np.abs(cum[np.arange(len(ne)), np.maximum((ne + 15) // 16 - 1, 0)][ne > 0]
                  - res["F"].double().cpu().numpy()[ne > 0]).max() <= 1e-5


def test_fused_training_step_matches_separate_calls(tiny_train):
    """om_render_fwd_bwd_l2 == om_render + om_l2_loss_grad + om_render_backward
    (both form dL/dC from the GPU's own C), and its loss matches the
    oracle's; the backward itself is held to the oracle in
    test_backward_tiny_vs_oracle."""
    sc, scene, t, o, d, target = tiny_train
    log("test_fused_training_step_matches_separate_calls")
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target.astype(np.float32)).to(og.device)
    res, loss_sep, g_sep = _gpu_grads(scene, t, og, dg, tg, 64, batch_wv=True)
    n = og.shape[0]
    out = dict(C=torch.empty((n, 3), device=og.device), T=torch.empty((n,), device=og.device),
               F=torch.empty((n, 7), device=og.device), n_placed=torch.empty((n,), dtype=torch.int32, device=og.device),
               n_eval=torch.empty((n,), dtype=torch.int32, device=og.device))
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}
    loss = torch.empty((1,), dtype=torch.float32, device=og.device)
    om.render_fwd_bwd_l2(scene, og, dg, tg, out, grads, n_max=64, c_bg=BG, loss=loss)
    torch.cuda.synchronize()
    for key in ("C", "T", "F", "n_placed", "n_eval"):
        assert torch.equal(out[key], res[key]), key
    assert loss.item() == loss_sep  # the same float32 sum in the same fixed order
    g = {k: v.double().cpu().numpy() for k, v in grads.items()}
    for k in g:
        scale = np.abs(g_sep[k]).max()
        assert np.abs(g[k] - g_sep[k]).max() <= 1e-5 * scale, k  # float32 atomics in another order
    _, ref_loss = oracle_upstream(sc, o, d, oracle.RenderParams(n_max=64, c_bg=BG), target.astype(np.float32))
    _loss_check(out, tg, ref_loss, "fused")


def test_backward_sum_invariant(tiny_train):
    """Per channel the four sources' gradient totals are equal."""
    sc, scene, t, o, d, target = tiny_train
    log("test_backward_sum_invariant")
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target.astype(np.float32)).to(og.device)
    _, _, grads = _gpu_grads(scene, t, og, dg, tg, 64)
    sums = [grads[s].reshape(-1, 8).sum(0) for s in SOURCES]
    for s in sums[1:]:
        np.testing.assert_allclose(s, sums[0], rtol=1e-4, atol=1e-7)


def test_backward_ert_matches_oracle(tiny_train):
    sc, scene, t, o, d, target = tiny_train
    log("test_backward_ert_matches_oracle: t_term=1e-2")
    og, dg = rays_to(o, d)
    prm = oracle.RenderParams(n_max=64, c_bg=BG, t_term=1e-2)
    up, _ = oracle_upstream(sc, o, d, prm, target.astype(np.float32))
    res, grads = _gpu_vjp(scene, t, og, dg, up, 64, t_term=1e-2)
    ref_f = oracle.oracle_render(sc, o, d, prm, keep_k=False)
    if not np.array_equal(res["n_eval"].cpu().numpy(), ref_f["n_eval"]):
        pytest.skip("a ray's transmittance sits at the threshold; gradients are compared with t_term=0")
    ref, scale = oracle_reference(sc, o, d, prm, up)
    check(grads, ref, scale, "ert")
    _, grads = _gpu_vjp(scene, t, og, dg, up, 64, t_term=1e-2, batch_wv=True)
    check(grads, ref, scale, "ert batch_wv")


def _pick_params(grads, per_source=12, mlp=16, seed=3, mlp_ok=None):
    """64 entries stratified over the five tensors and over magnitude, plus
    4 with zero gradient.  Per tensor, k targets log-uniform between
    1e-3 max|g| and max|g| (the centres of k equal bins of log |g|), each
    taking the unpicked entry nearest to it in log |g| (ties broken by a
    seeded draw); `mlp_ok` (bool per MLP parameter) restricts the MLP picks
    to the entries where the finite-difference step is valid.  The
    zero-gradient entries are neighbours in memory order (the next or
    previous vertex or texel) of touched rows that no sample reaches, one per
    feature source: the finite difference there is exactly 0."""
    rng = np.random.default_rng(seed)
    picks = []
    for src in (*SOURCES, "mlp"):
        k = mlp if src == "mlp" else per_source
        g = np.abs(grads[src].reshape(-1))
        m = g.max()
        ok = (g >= 1e-3 * m) & (mlp_ok if src == "mlp" and mlp_ok is not None else True)
        elig = np.nonzero(ok)[0]
        elig = elig[rng.permutation(elig.size)]
        lg = np.log10(g[elig] / m)
        used = np.zeros(elig.size, bool)
        for i in range(k):
            tgt = -3.0 * (i + 0.5) / k
            j = int(np.argmin(np.where(used, np.inf, np.abs(lg - tgt))))
            used[j] = True
            picks.append((src, int(elig[j])))
    for src in SOURCES:
        rows = grads[src].reshape(-1, 8)
        touched = np.nonzero(np.any(rows != 0, axis=1))[0]
        zero = np.setdiff1d(np.concatenate([touched + 1, touched - 1]), touched)
        zero = zero[(zero >= 0) & (zero < rows.shape[0])]
        r = int(rng.choice(zero))
        picks.append((src, r * 8 + int(rng.integers(8))))
    return picks


def _relu_signs_kept(mlp, x, gate, j, h):
    """True if no ReLU of the deferred MLP changes sign on any gated ray
    when parameter j moves by -h or +h (float64 on the host; x = [F, d]
    [n, 10]).  Between two such points G is smooth in the parameter, so a
    central difference there has only the O(h^2) truncation error."""
    nin = x.shape[1]
    pats = []
    for s_ in (-1.0, 0.0, 1.0):
        w = np.asarray(mlp, np.float64).copy()
        w[j] += s_ * h
        w1 = w[:16 * nin].reshape(16, nin)
        b1 = w[16 * nin:16 * nin + 16]
        w2 = w[16 * nin + 16:16 * nin + 272].reshape(16, 16)
        b2 = w[16 * nin + 272:16 * nin + 288]
        z1 = x @ w1.T + b1
        z2 = np.maximum(z1, 0.0) @ w2.T + b2
        pats.append(np.concatenate([z1 > 0, z2 > 0], axis=1)[gate])
    return bool(np.array_equal(pats[0], pats[1]) and np.array_equal(pats[1], pats[2]))


def _fd_check(scene, t, og, dg, tg, n_max, grads, eps=1e-3, picks=None, feature_eps=None, mlp_eps=None):
    """Central differences of the float64 loss of float32 renders; `eps` for
    the MLP weights, `feature_eps` (default `eps`) for grid and plane
    entries.  With `mlp_eps`, an MLP entry takes that step instead when no
    ReLU changes sign over it (_relu_signs_kept), else `eps`.  Error
    |g - g_fd| / max(|g_fd|, 1e-2 RMS of the checked nonzero g_fd).
    Returns (picks, g_fd, g, error, steps)."""
    picks = _pick_params(grads) if picks is None else picks
    if mlp_eps is not None:
        res0 = om.render(scene, og, dg, n_max=n_max, c_bg=BG)
        x = np.concatenate([res0["F"].double().cpu().numpy(), dg.double().cpu().numpy()], axis=1)
        gate = res0["n_placed"].cpu().numpy() > 0
        mlp0 = t["mlp"].double().cpu().numpy()
    fd, an, hs = [], [], []
    for src, e in picks:
        flat = t[src].view(-1)
        v0 = flat[e].item()
        if src == "mlp":
            h = mlp_eps if mlp_eps is not None and _relu_signs_kept(mlp0, x, gate, e, mlp_eps) else eps
        else:
            h = eps if feature_eps is None else feature_eps
        vals, steps = [], []
        for s in (+1.0, -1.0):
            flat[e] = v0 + s * h
            steps.append(flat[e].item())  # the binary32 value actually used
            res = om.render(scene, og, dg, n_max=n_max, c_bg=BG)
            vals.append(om.l2_loss_fp64(res["C"], tg).item())
        flat[e] = v0
        fd.append((vals[0] - vals[1]) / (steps[0] - steps[1]))
        an.append(grads[src].reshape(-1)[e])
        hs.append(h)
    fd, an, hs = np.array(fd), np.array(an), np.array(hs)
    rms = np.sqrt(np.mean(fd[an != 0] ** 2))
    err = np.abs(an - fd) / np.maximum(np.abs(fd), 1e-2 * rms)
    return picks, fd, an, err, hs


def _fd_log(tag, picks, fd, an, err, hs=None):
    for src in (*SOURCES, "mlp"):
        sel = [i for i, (s_, _) in enumerate(picks) if s_ == src]
        mags = np.abs(an[sel]) / np.abs(an[sel]).max()
        steps = "" if hs is None else f", steps {sorted(set(float(h) for h in hs[sel]))}"
        log(f"  FD {tag} {src:9s}: {len(sel)} entries, |g| from {mags.min():.1e} to 1 of the largest, "
            f"max err {err[sel].max():.2e}, median {np.median(err[sel]):.2e}{steps}")
    zero = an == 0
    log(f"  FD {tag}: {int(zero.sum())} zero-gradient entries, their |g_fd| = {np.abs(fd[zero]).tolist()}")


def test_backward_finite_differences_tiny(tiny_train):
    """Central FD on the tiny scene's 256 rays with a step of 1e-2 (reported
    at 1e-3 too).  With 256 rays one entry moves the float64 loss by ~1e-5
    of itself at a step of 1e-3, the size of the float32 rounding of the
    colours that the loss is formed from (measured: 1.6e-3 worst relative
    error on features and 4.4e-3 on the smallest MLP entries at 1e-3); the
    larger step divides that noise by ten while the truncation error (h^2
    times the third derivative) stays ~1e-4 relative.  The features enter
    the loss through exp and sigmoids only, so the loss is smooth in them;
    the MLP picks are drawn among the parameters over whose +-1e-2 no ReLU
    of any ray changes sign (checked in float64 on the host), where the
    central difference has only its O(h^2) error."""
    sc, scene, t, o, d, target = tiny_train
    log("test_backward_finite_differences_tiny")
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target.astype(np.float32)).to(og.device)
    res, _, grads = _gpu_grads(scene, t, og, dg, tg, 64)
    x = np.concatenate([res["F"].double().cpu().numpy(), dg.double().cpu().numpy()], axis=1)
    gate = res["n_placed"].cpu().numpy() > 0
    mlp0 = t["mlp"].double().cpu().numpy()
    mlp_ok = np.array([_relu_signs_kept(mlp0, x, gate, j, 1e-2) for j in range(mlp0.size)])
    log(f"  MLP entries without a ReLU sign change over +-1e-2: {int(mlp_ok.sum())} of {mlp0.size}")
    picks = _pick_params(grads, mlp_ok=mlp_ok)
    _, fd3, an3, err3, hs3 = _fd_check(scene, t, og, dg, tg, 64, grads, picks=picks)
    _fd_log("tiny step 1e-3 (reported)", picks, fd3, an3, err3, hs3)
    picks, fd, an, err, hs = _fd_check(scene, t, og, dg, tg, 64, grads, picks=picks, feature_eps=1e-2, mlp_eps=1e-2)
    _fd_log("tiny step 1e-2", picks, fd, an, err, hs)
    assert len(picks) == 68 and int((an == 0).sum()) == 4 and np.all(fd[an == 0] == 0)
    assert err.max() <= 1e-3, [(p, f, a, h) for p, f, a, e, h in zip(picks, fd, an, err, hs) if e > 1e-3]


@pytest.fixture(scope="module")
def towers():
    log("building towers scene (512^2 occupancy, 10% towers) and its perturbed copy")
    cfg, rec = scenegen.workload("towers-2^20")
    sc = scenegen.make_scene(cfg)
    pert = scenegen.perturb_scene(sc, 0.05, seed=2)
    o, d = scenegen.make_rays(rec)
    o, d = o[:256].copy(), d[:256].copy()
    prm = oracle.RenderParams(n_max=rec["n_max"], c_bg=BG)
    target = oracle.oracle_render(pert, o, d, prm, keep_k=False)["C"].astype(np.float32)
    del pert
    return sc, o, d, target, rec["n_max"]


def _rounded_scene(sc):
    from tests.gpu_util import bf16_round
    r = dict(sc)
    for k in SOURCES:
        r[k] = bf16_round(sc[k])
    return r


def test_towers_fp32_forward_parity(towers):
    """float32 render of the uneven towers rays (up to 512 samples per ray)."""
    sc, o, d, target, n_max = towers
    log("test_towers_fp32_forward_parity: 256 rays, n_max 512")
    scene, t = upload_scene(sc)
    og, dg = rays_to(o, d)
    res = om.render(scene, og, dg, n_max=n_max, c_bg=BG)
    ref = oracle.oracle_render(sc, o, d, oracle.RenderParams(n_max=n_max, c_bg=BG), keep_k=False)
    assert np.array_equal(res["n_placed"].cpu().numpy(), ref["n_placed"])
    assert np.array_equal(res["n_eval"].cpu().numpy(), ref["n_eval"])
    for key in ("C", "T", "F"):
        assert np.abs(res[key].double().cpu().numpy() - ref[key]).max() <= 1e-5, key
    log(f"  n_placed max {int(ref['n_placed'].max())}, mean {ref['n_placed'].mean():.1f}")
    del scene, t
    torch.cuda.empty_cache()


def test_towers_bf16_storage_gradient_vs_oracle(towers):
    """bfloat16 storage, float32 arithmetic and float32 master gradients:
    must match the float64 oracle on the bfloat16-rounded scene."""
    sc, o, d, target, n_max = towers
    log("test_towers_bf16_storage_gradient_vs_oracle: 256 rays, n_max 512")
    scene, t = upload_scene(sc, dtype=torch.bfloat16)
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target).to(og.device)
    rsc = _rounded_scene(sc)
    prm = oracle.RenderParams(n_max=n_max, c_bg=BG)
    up, ref_loss = oracle_upstream(rsc, o, d, prm, target)
    ref, scale = oracle_reference(rsc, o, d, prm, up)
    for bw in (False, True):
        res, g = _gpu_vjp(scene, t, og, dg, up, n_max, batch_wv=bw)
        npl = res["n_placed"].cpu().numpy()
        log(f"  samples/ray: min {npl.min()} mean {npl.mean():.1f} max {npl.max()}; "
            f"hist(32-wide bins) {np.histogram(npl, bins=np.arange(0, 545, 32))[0].tolist()}")
        _loss_check(res, tg, ref_loss, f"towers bf16 storage batch_wv={bw}")
        check(g, ref, scale, f"towers bf16 storage batch_wv={bw}")


def test_towers_full_bf16_gradient_error(towers):
    """Full BF16 form (bf16 storage + bf16 MFMA MLP forward) against the
    float64 oracle gradient of the float32 scene: the gradient's direction
    (cosine), its relative L2 error and the median per-entry relative error
    over the entries above 1e-2 max|g|, each within about 3x its measured
    value."""
    sc, o, d, target, n_max = towers
    log("test_towers_full_bf16_gradient_error")
    scene, t = upload_scene(sc, dtype=torch.bfloat16)
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target).to(og.device)
    res = om.render(scene, og, dg, n_max=n_max, c_bg=BG)
    dC, _ = om.l2_loss_grad(res["C"], tg)
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}
    om.render_backward(scene, og, dg, res, dC, grads, n_max=n_max, c_bg=BG)
    _, _, ref = oracle.oracle_loss_and_grads(sc, o, d, oracle.RenderParams(n_max=n_max, c_bg=BG),
                                             target.astype(np.float64))
    a, b = [], []
    for src in SOURCES:
        uniq, rows = ref[src]
        a.append(grads[src].double().cpu().numpy().reshape(-1, 8)[uniq].ravel())
        b.append(rows.ravel())
    a.append(grads["mlp"].double().cpu().numpy())
    b.append(ref["mlp"])
    a, b = np.concatenate(a), np.concatenate(b)
    cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
    big = np.abs(b) >= 1e-2 * np.abs(b).max()
    rel = np.abs(a - b)[big] / np.abs(b)[big]
    l2 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    log(f"  BF16 form vs FP64 oracle gradient: cosine {cos:.6f}, relative L2 error {l2:.3e}, "
        f"rel err on |g| >= 1e-2 max: median {np.median(rel):.3e}, 99th percentile {np.percentile(rel, 99):.3e}, "
        f"max {rel.max():.3e}")
    # about 3x the measured 1 - cos = 1.08e-4, 1.52e-2 and 1.8e-2: the bfloat16
    # rounding of the stored features and of the MLP's operands moves every
    # per-sample term by ~2^-9 relative, so individual entries that sum
    # cancelling terms can be off by far more (99th percentile 0.2)
    assert 1.0 - cos < 3.3e-4
    assert l2 < 4.5e-2 and np.median(rel) < 5.5e-2


@pytest.fixture(scope="module")
def oblique_train():
    log("building oblique scene, perturbed copy, 2^18 training rays and their oracle targets")
    cfg, rec = scenegen.workload("train-2^18")
    sc = scenegen.make_scene(cfg)
    pert = scenegen.perturb_scene(sc, 0.05, seed=2)
    o, d = scenegen.make_rays(rec)
    prm = oracle.RenderParams(n_max=rec["n_max"], c_bg=BG)
    target = oracle.oracle_render(pert, o, d, prm, keep_k=False, chunk=4096)["C"].astype(np.float32)
    del pert
    scene, t = upload_scene(sc)
    return sc, scene, t, o, d, target, rec["n_max"]


def test_oblique_backward_vs_oracle_256(oblique_train):
    sc, scene, t, o, d, target, n_max = oblique_train
    log("test_oblique_backward_vs_oracle_256: oblique scene, 256 rays, perturbed-scene targets")
    o256, d256, t256 = o[:256].copy(), d[:256].copy(), target[:256].copy()
    og, dg = rays_to(o256, d256)
    tg = torch.from_numpy(t256).to(og.device)
    prm = oracle.RenderParams(n_max=n_max, c_bg=BG)
    up, ref_loss = oracle_upstream(sc, o256, d256, prm, t256)
    ref, scale = oracle_reference(sc, o256, d256, prm, up)
    for bw in (False, True):
        res, grads = _gpu_vjp(scene, t, og, dg, up, n_max, batch_wv=bw)
        _loss_check(res, tg, ref_loss, f"oblique batch_wv={bw}")
        check(grads, ref, scale, f"oblique batch_wv={bw}")


def test_oblique_soft_occ_backward_vs_oracle_256(oblique_train):
    """The soft-occupancy training form (eps = 0.01) on the full oblique
    scene: loss and gradients into features, MLP and the occupancy bounds for
    256 of its rays against the oracle."""
    sc, scene, t, o, d, target, n_max = oblique_train
    eps = 0.01
    log("test_oblique_soft_occ_backward_vs_oracle_256: eps=0.01")
    o256, d256, t256 = o[:256].copy(), d[:256].copy(), target[:256].copy()
    og, dg = rays_to(o256, d256)
    tg = torch.from_numpy(t256).to(og.device)
    prm = oracle.RenderParams(n_max=n_max, c_bg=BG, occ_eps=eps)
    up, ref_loss = oracle_upstream(sc, o256, d256, prm, t256)
    ref, scale = oracle_reference(sc, o256, d256, prm, up)
    res, g = _gpu_vjp(scene, t, og, dg, up, n_max, occ_eps=eps, batch_wv=True)
    _loss_check(res, tg, ref_loss, "oblique soft occupancy")
    assert len(ref["occ"][0]) > 1000 and np.abs(ref["occ"][1]).max() > 0
    check(g, ref, scale, "oblique soft occupancy")


def test_oblique_enc_smooth_gradients_vs_oracle_256(oblique_train):
    """The encoded-direction training form on the full oblique scene: the
    34-input MLP, L2 + view-smoothness loss (4 perturbations per ray,
    weight 0.1) over 256 of its rays, loss and gradients against the
    oracle."""
    sc, scene, t, o, d, target, n_max = oblique_train
    log("test_oblique_enc_smooth_gradients_vs_oracle_256: dir_freqs=4, P=4")
    mlp = scenegen.mlp_params(4, seed=7)
    sc4 = dict(sc, mlp=mlp, dir_freqs=4)
    dev = t["grid"].device
    scene4 = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], torch.from_numpy(mlp).to(dev),
                      box_lo=tuple(float(v) for v in sc["box_lo"]), box_hi=tuple(float(v) for v in sc["box_hi"]))
    assert scene4.dir_freqs == 4
    o256, d256, t256 = o[:256].copy(), d[:256].copy(), target[:256].copy()
    pert = scenegen.view_perturbations(256, 4, seed=4)
    w = float(np.float32(0.1))
    smooth = dict(perturb=pert, weight=w)
    prm = oracle.RenderParams(n_max=n_max, c_bg=BG)
    up, _ = oracle_upstream(sc4, o256, d256, prm, t256)
    ref, scale = oracle_reference(sc4, o256, d256, prm, up, smooth=smooth)
    og, dg = rays_to(o256, d256)
    pg = torch.from_numpy(pert).to(dev)
    res = om.render(scene4, og, dg, n_max=n_max, c_bg=BG, mlp_bf16=0, batch_wv=True)
    grads = {k: torch.zeros(t[k].shape, dtype=torch.float32, device=dev) for k in SOURCES}
    grads["mlp"] = torch.zeros(mlp.shape, dtype=torch.float32, device=dev)
    dF = torch.zeros_like(res["F"])
    om.smooth_loss(scene4, res["F"], dg, pg, w, dL_dF=dF, grad_mlp=grads["mlp"], with_loss=False)
    om.render_backward(scene4, og, dg, res, torch.from_numpy(up).to(dev), grads, n_max=n_max, c_bg=BG, dL_dF=dF)
    torch.cuda.synchronize()
    check({k: v.double().cpu().numpy() for k, v in grads.items()}, ref, scale, "oblique encoded + smoothness")


def test_oblique_finite_differences_2e18(oblique_train):
    """Central FD (eps = 1e-3) of the float64 GPU loss over all 2^18 rays,
    L2 against oracle renders of the perturbed scene: 64 entries stratified
    over the five tensors and three decades of magnitude, and 4 entries
    with zero gradient."""
    sc, scene, t, o, d, target, n_max = oblique_train
    log("test_oblique_finite_differences_2e18: 64 + 4 params, 2^18 rays")
    og, dg = rays_to(o, d)
    tg = torch.from_numpy(target).to(og.device)
    res, _, grads = _gpu_grads(scene, t, og, dg, tg, n_max, batch_wv=True)  # the training path
    picks, fd, an, err, hs = _fd_check(scene, t, og, dg, tg, n_max, grads)
    _fd_log("2^18 eps=1e-3", picks, fd, an, err, hs)
    assert len(picks) == 68 and int((an == 0).sum()) == 4 and np.all(fd[an == 0] == 0)
    assert err.max() <= 1e-3, [(p, f, a) for p, f, a, e in zip(picks, fd, an, err) if e > 1e-3]


def test_backward_large_batch_equals_its_halves():
    """A batch of 4.26 M rays (the ray-order sort then runs as 1,024 blocks
    of ~4,160 rays, each reserving its own ranges of the order; the waves
    take rays from a counter that passes 2^22) against its two halves in
    two calls (the backward adds into the gradient buffers), with the same
    dL/dC: the same gradients."""
    n = 4096 * 1024 + 4096 * 16 + 5  # ragged against every block size involved
    log(f"test_backward_large_batch_equals_its_halves: {n} rays")
    sc = scenegen.make_scene(scenegen.TINY)
    scene, t = upload_scene(sc)
    o, d = scenegen.oblique_rays(n, seed=23)
    og, dg = rays_to(o, d)
    kw = dict(n_max=64, c_bg=BG)
    res = om.render(scene, og, dg, batch_wv=True, **kw)
    gen = torch.Generator(device=og.device)
    gen.manual_seed(3)
    dC = (torch.randn(res["C"].shape, device=og.device, generator=gen) * 1e-6).contiguous()
    zero = lambda: {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}  # noqa: E731
    whole = zero()
    om.render_backward(scene, og, dg, res, dC, whole, **kw)
    halves = zero()
    h = n // 2
    for sl in (slice(0, h), slice(h, n)):
        part = {k: v[sl].contiguous() for k, v in res.items()}
        om.render_backward(scene, og[sl].contiguous(), dg[sl].contiguous(), part, dC[sl].contiguous(), halves, **kw)
    torch.cuda.synchronize()
    # float32 atomics add millions of cancelling terms in a different order
    # in the two runs (up to 8.5e-6 of the largest entry measured), hence
    # the 5e-5 floor
    for k in (*SOURCES, "mlp"):
        scale = float(whole[k].abs().max())
        diff = (whole[k] - halves[k]).abs()
        log(f"  {k}: max |g| {scale:.3e}, max |whole - halves| / max |g| {float(diff.max()) / scale:.2e}")
        assert scale > 0
        assert float((diff - (1e-3 * halves[k].abs() + 5e-5 * scale)).max()) <= 0, k


def test_backward_does_not_depend_on_ray_order():
    """The march backward walks the rays longest first (by batch count) and
    hands them to its waves on demand, whatever order the caller gives.
    The same rays, saved outputs and dL/dC in a shuffled order must give the
    same gradients (lengths from 0 to ~450 samples, so the batch-count
    bins from 0 up are populated)."""
    sc = scenegen.make_scene(scenegen.TINY)
    scene, t = upload_scene(sc)
    n = 50_000
    o, d = scenegen.oblique_rays(n, seed=31)
    d = d.copy()
    d[::7, 2] = -d[::7, 2]  # every 7th ray points up, away from the box: no sample
    log(f"test_backward_does_not_depend_on_ray_order: {n} rays, n_max 512")
    og, dg = rays_to(o, d)
    kw = dict(n_max=512, c_bg=BG)
    res = om.render(scene, og, dg, batch_wv=True, **kw)
    gen = torch.Generator(device=og.device)
    gen.manual_seed(5)
    dC = (torch.randn(res["C"].shape, device=og.device, generator=gen) * 1e-5).contiguous()
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(7)).to(og.device)
    zero = lambda: {k: torch.zeros(t[k].shape, dtype=torch.float32, device=og.device) for k in (*SOURCES, "mlp")}  # noqa: E731
    a = zero()
    om.render_backward(scene, og, dg, res, dC, a, **kw)
    b = zero()
    shuffled = {k: v[perm].contiguous() for k, v in res.items()}
    om.render_backward(scene, og[perm].contiguous(), dg[perm].contiguous(), shuffled, dC[perm].contiguous(), b, **kw)
    torch.cuda.synchronize()
    ne = res["n_eval"].cpu().numpy()
    log(f"  n_eval from {ne.min()} to {ne.max()}, {len(np.unique((ne + 15) // 16))} batch counts")
    assert ne.max() > 256 and (ne == 0).any()
    for k in (*SOURCES, "mlp"):
        scale = float(a[k].abs().max())
        diff = (a[k] - b[k]).abs()
        log(f"  {k}: max |g| {scale:.3e}, max |a - b| / max |g| {float(diff.max()) / scale:.2e}")
        assert scale > 0
        assert float((diff - (1e-3 * b[k].abs() + 5e-5 * scale)).max()) <= 0, k
