/*
 * omerf.h -- C ABI of the MI355X (gfx950) occupancy-plane ray marcher.
 *
 * Implements the real-time hot path of Oblique-MERF (arXiv 2404.09531):
 * ray marching a MERF-style scene (low-resolution 3D feature grid plus three
 * high-resolution planes, Sec. 3 Eq. 2) that places samples only inside the
 * per-column [z_min, z_max] intervals of the occupancy plane (Sec. 4.1,
 * Eq. 6 with epsilon = 0 and Eq. 7; Sec. 4.4), applies the density and colour
 * activations (Eq. 3), alpha-composites (Eq. 1) and runs the deferred
 * view-dependent MLP once per ray (Eq. 4).  A backward pass scatter-adds
 * gradients of a per-ray colour loss into the grid, the planes and the MLP.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named "device" are HIP device pointers owned by the caller; the
 *   library never allocates, frees or keeps device memory, and never copies
 *   to or from the host inside render / backward calls.
 * - All work is enqueued asynchronously on the caller's stream `stream`
 *   (a hipStream_t passed as void*; NULL = the default stream).  A kernel
 *   fault surfaces at the caller's next synchronisation.
 * - Return value: OM_OK (0) or a negative status (OM_ERR_*).  On error,
 *   om_last_error() returns a message for the calling thread.  Nothing is
 *   enqueued when argument validation fails.  The library never aborts.
 * - Layout: rays are float32 [n][3] (origin o, unit direction d).  Feature
 *   sources are channels-last with 8 channels: grid [Lz][Ly][Lx][8],
 *   plane_xy [Ny][Nx][8], plane_xz [Nz][Nx][8], plane_yz [Nz][Ny][8];
 *   channel 0 = density pre-activation, 1..3 = diffuse colour,
 *   4..7 = specular features (Eq. 3).  Occupancy plane float32 [My][Mx][2]
 *   holding (z_min, z_max).  MLP float32[OM_MLP_NPARAMS(dir_freqs)] packed
 *   as W1[16][N], b1[16], W2[16][16], b2[16], W3[3][16], b3[3] (row-major
 *   (out, in)); input order [sum w c^d (3), sum w f (4), enc(d)] with
 *   enc(d) = d (N = 10) or d and its four sine/cosine frequencies (N = 34).
 * - Storage: float32, bfloat16 or 8-bit features (OM_U8, with per-source
 *   decoding); the grid dense or as sparse voxel blocks.  8-bit and sparse
 *   scenes are render only.
 *
 * Sample lattice and placement (Sec. 4.1 Eq. 6-7, Sec. 4.4)
 * ---------------------------------------------------------
 * Samples sit at t_k = k * delta (k = 0 .. 2^24 - 1) from the ray origin.
 * The point is p = fl32(o + fl32(t_k * d)) (binary32, no fused multiply-add).
 * Sample k is accepted iff p lies in the closed box and
 * z_min[j][i] <= p_z <= z_max[j][i], where (i, j) is the occupancy cell that
 * contains p's xy (half-open cells, far face in the last cell).  The first
 * n_max accepted samples in increasing k are used.
 *
 * Compositing and output (Eq. 1, Eq. 4)
 * -------------------------------------
 * a_i = exp(t0_i) * delta, alpha_i = 1 - exp(-a_i), T_i = exp(-sum_{j<i} a_j),
 * w_i = T_i alpha_i; F = [sum w c^d, sum w f]; T_n = transmittance after the
 * last evaluated sample; C = sum w c^d + [n_eval > 0] G(F, d) + T_n c_bg.
 * With t_term > 0 a ray stops after the first sample whose following
 * transmittance drops below t_term.
 */
#ifndef OMERF_H
#define OMERF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define OM_OK 0
#define OM_ERR_INVALID (-1)      /* bad pointer, size or parameter        */
#define OM_ERR_UNSUPPORTED (-2)  /* shape / dtype the kernels do not take */
#define OM_ERR_HIP (-3)          /* the HIP runtime reported an error     */

/* Storage types of the feature grid and planes. */
#define OM_F32 0
#define OM_BF16 1
#define OM_U8 2 /* 8-bit codes, decoded per source and channel (quant_lo, quant_step) */

#define OM_CHANNELS 8
#define OM_MAX_SAMPLES 1024       /* largest n_max the kernels accept   */

typedef struct om_scene om_scene; /* opaque handle, host metadata only */

/*
 * Scene description.  The device pointers are BORROWED: the handle keeps
 * them, the caller keeps ownership and must keep the memory alive (and
 * unchanged while a call using it runs).
 * Preconditions checked by om_scene_create / om_scene_update:
 *  - box_hi > box_lo on every axis; each extent (box_hi - box_lo) is a power
 *    of two, so that interpolation coordinates are exact scalings;
 *  - grid_dims >= 2 and plane_dims >= 2 per axis; occ_dims >= 1;
 *  - occ_dims[a] / (box_hi[a] - box_lo[a]) is a power of two and
 *    box_lo[a] * occ_dims[a] / (box_hi[a] - box_lo[a]) an integer (a = x, y),
 *    so the containing occupancy cell is an exact floor;
 *  - every feature source has fewer than 2^31 vertices;
 *  - dtype is OM_F32, OM_BF16 (bf16 = the upper 16 bits of a binary32) or
 *    OM_U8 (render only; quant_lo and quant_step finite, quant_step >= 0);
 *  - all pointers non-NULL and 16-byte aligned.
 */
typedef struct om_scene_desc {
    float box_lo[3];
    float box_hi[3];
    int32_t grid_dims[3];   /* Lx, Ly, Lz */
    int32_t plane_dims[3];  /* Nx, Ny, Nz */
    int32_t occ_dims[2];    /* Mx, My     */
    int32_t dtype;          /* OM_F32, OM_BF16 or OM_U8 */
    const void* grid;       /* device, [Lz][Ly][Lx][8] of dtype */
    const void* plane_xy;   /* device, [Ny][Nx][8] of dtype     */
    const void* plane_xz;   /* device, [Nz][Nx][8] of dtype     */
    const void* plane_yz;   /* device, [Nz][Ny][8] of dtype     */
    const float* occ;       /* device, [My][Mx][2] float32      */
    const float* mlp;       /* device, float32[OM_MLP_NPARAMS(dir_freqs)] */
    int32_t dir_freqs;      /* view-direction input of the deferred MLP:
                               0: x = [F (7), d (3)];  4: x = [F, d,
                               sin(2^k d), cos(2^k d) for k = 0..3] (34
                               inputs; Sec. 4.2).  Other values rejected. */
    /* OM_U8 only (ignored otherwise): channel c of source s (0 grid, 1 XY,
     * 2 XZ, 3 YZ) stores a byte q that stands for
     * quant_lo[s][c] + q * quant_step[s][c] (Sec. 4.4: baked features kept
     * as 8-bit images).  Copied when the handle is created or updated. */
    float quant_lo[4][8];
    float quant_step[4][8];
    /* Sparse voxel blocks of the grid (Sec. 4.4: the baked grid is kept as
     * sparse blocks).  block_shift = 0: grid is the dense array above.
     * block_shift = s in 1..5: B = 2^s cells per block edge; grid is an
     * atlas of n_blocks + 1 blocks of (B + 1)^3 vertices ([z][y][x][8] of
     * dtype each, one vertex of overlap with the next block), block 0 all
     * zero; grid_blocks (device int32 [ceil((Lz-1)/B)][ceil((Ly-1)/B)]
     * [ceil((Lx-1)/B)]) names the atlas block of each B^3 region of cells
     * (0 for regions no sample can reach).  Ids above n_blocks read block
     * n_blocks.  Built by om_sparse_grid_index / om_sparse_grid_fill.
     * Render only.  (n_blocks + 1) (B + 1)^3 must be below 2^31. */
    const int32_t* grid_blocks;
    int32_t block_shift;
    int32_t n_blocks;
} om_scene_desc;

/* Packed MLP parameters for an N -> 16 -> 16 -> 3 network: W1 [16][N], b1,
 * W2 [16][16], b2, W3 [3][16], b3, N = 10 + 6 dir_freqs (499 or 883). */
#define OM_MLP_NPARAMS(dir_freqs) (16 * (10 + 6 * (dir_freqs)) + 16 + 256 + 16 + 48 + 3)
#define OM_MLP_NPARAMS_RAW_DIR OM_MLP_NPARAMS(0) /* 499: input [F, d] */

/* Per-call render parameters. */
typedef struct om_params {
    float delta;      /* lattice step; must be a positive power of two      */
    int32_t n_max;    /* samples kept per ray, 1 .. OM_MAX_SAMPLES          */
    float t_term;     /* early-termination threshold, 0 = never stop        */
    float c_bg[3];    /* background colour                                  */
    int32_t mlp_bf16; /* 0: float32 MLP; 1: bfloat16 MLP on MFMA with
                         float32 accumulation; -1: bfloat16 for OM_BF16
                         scenes, float32 otherwise                          */
    float occ_eps;    /* soft occupancy (Sec. 4.1, Eq. 6 and 8), finite and
                         >= 0.  0: the hard interval.  > 0: each placed
                         sample's compositing weight is multiplied by
                         M = min(clamp((z - z_min)/eps, 0, 1)^2,
                         clamp((z_max - z)/eps, 0, 1)^2) of its cell (q = 2);
                         the transmittance is not masked.  Placement is the
                         same either way (M = 0 outside [z_min, z_max]).     */
} om_params;

/* Forward outputs, all device pointers, all REQUIRED (the backward pass
 * reads F, T and n_eval back).  C [n][3], T [n], F [n][7], n_placed [n],
 * n_eval [n].  With t_term > 0, n_placed counts the samples placed up to
 * termination; with t_term = 0 it is the full placed count. */
typedef struct om_fwd_out {
    float* C;
    float* T;
    float* F;
    int32_t* n_placed;
    int32_t* n_eval;
    /* Optional (NULL to skip), for the backward: float32
     * [n][OM_BATCH_SLOTS(n_max)][7].  Slot b of a ray holds, for its b-th
     * group of OM_BATCH consecutive evaluated samples (the last group may be
     * shorter), the sum over the group of w_i * v_i: the compositing weight
     * of Eq. 1 times the activated diffuse colour and feature channels of
     * Eq. 3 (the same 7 channels as F, which is the sum over all groups).
     * Slots from ceil(n_eval / OM_BATCH) on are not written.  The march
     * writes it when non-NULL; om_render_backward reads it when non-NULL
     * and otherwise recomputes these sums with an extra replay of the
     * samples.  Must be NULL for OM_U8 scenes (render only). */
    float* batch_wv;
} om_fwd_out;

#define OM_BATCH 16
#define OM_BATCH_SLOTS(n_max) (((n_max) + OM_BATCH - 1) / OM_BATCH)

/* Gradient buffers (device, float32, caller-zeroed or holding a running
 * sum: the backward pass ACCUMULATES into them).  Shapes match the scene:
 * grid [Lz][Ly][Lx][8] (sparse scenes are render only), planes as the
 * scene, mlp [OM_MLP_NPARAMS(dir_freqs)]. */
typedef struct om_grads {
    float* grid;
    float* plane_xy;
    float* plane_xz;
    float* plane_yz;
    float* mlp;
    /* Optional: gradient of (z_min, z_max), [My][Mx][2], accumulated when
     * occ_eps > 0 (the derivative of M; placement is piecewise constant in
     * the bounds).  NULL skips it. */
    float* occ;
} om_grads;

/* Create a scene handle from `desc` (validated as above).  On success
 * *out holds a new handle to be released with om_scene_destroy.  Cites:
 * representation of Sec. 3 (Eq. 2) and the occupancy plane of Sec. 4.1. */
int om_scene_create(const om_scene_desc* desc, om_scene** out);

/* Re-point an existing handle at new tensors (e.g. after an optimiser step
 * or a bf16 re-cast); same validation as om_scene_create.  The handle is
 * unchanged if validation fails.  Must not race with calls using it. */
int om_scene_update(om_scene* scene, const om_scene_desc* desc);

/*
 * Occupancy pyramid for hierarchical empty-space skipping (the jump through
 * blank columns of Sec. 4.4, extended from single columns to blocks of
 * 2^l x 2^l columns).  Level l = 1..levels holds (My >> l) x (Mx >> l)
 * float2 entries, row-major, levels stored one after the other from l = 1:
 * for each block, (min z_min, max z_max) over its cells with
 * z_min <= z_max, or (+inf, -inf) if it has none.
 *
 * om_occupancy_mips_size: bytes needed for `levels` levels, or -1 (with
 * om_last_error set) unless 0 <= levels <= 8 and both occupancy dims are
 * divisible by 2^levels.
 *
 * om_build_occupancy_mips: computes the pyramid of the scene's occupancy
 * plane into the caller-owned device buffer `mips` (8-byte aligned, at
 * least om_occupancy_mips_size bytes; it must outlive its use) on `stream`
 * and attaches it to the handle: every later placement, render and backward
 * call skips empty space level by level.  Sample placement is unchanged
 * (the pyramid only skips candidates that cannot be accepted).  levels = 0
 * detaches it; so does om_scene_update, after which it must be built again
 * for the new occupancy.  Must not race with calls using the handle.
 */
int64_t om_occupancy_mips_size(const om_scene* scene, int levels);
int om_build_occupancy_mips(om_scene* scene, void* mips, int64_t mips_bytes, int levels, void* stream);

/* Release a handle (never the tensors).  NULL is accepted. */
int om_scene_destroy(om_scene* scene);

/*
 * Sample placement only (Sec. 4.1 Eq. 6-7, Sec. 4.4), for inspection and
 * parity tests.  o, d: device float32 [n][3].  k_out: device int32
 * [n][n_max] receiving the accepted lattice indices in increasing order,
 * padded with -1.  n_placed: device int32 [n].  n = 0 is a no-op.
 * p->t_term and p->c_bg are ignored.
 */
int om_place_samples(const om_scene* scene, const float* o, const float* d, int64_t n,
                     const om_params* p, int32_t* k_out, int32_t* n_placed, void* stream);

/*
 * Feature rows a render reads (Eq. 2 over the samples of Sec. 4.1 / 4.4):
 * for every evaluated sample -- the first n_eval[r] placed samples of ray r
 * (n_eval: device int32 [n] from om_render with the same parameters), or
 * every placed sample when n_eval is NULL -- stores the byte 1 at its 8 grid
 * vertices and 12 plane texels.  grid_flags: device uint8 with one byte per
 * grid row ([Lz][Ly][Lx] for a dense grid, the atlas's
 * (n_blocks + 1) (B + 1)^3 vertices for sparse blocks); xy_flags [Ny][Nx],
 * xz_flags [Nz][Nx], yz_flags [Nz][Ny].  Flags are only set, never cleared:
 * the caller zeroes them (or accumulates several calls).  The marked rows are
 * the rows whose gradient a backward can touch, and their bytes the least
 * HBM traffic a render must move (each row read once).  p->t_term and
 * p->c_bg are ignored.
 */
int om_mark_rows(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                 const int32_t* n_eval, uint8_t* grid_flags, uint8_t* xy_flags, uint8_t* xz_flags,
                 uint8_t* yz_flags, void* stream);

/*
 * Forward render of n rays (Sec. 3 Eq. 1-4 with the occupancy-plane
 * sampling of Sec. 4.1 / 4.4).  o, d: device float32 [n][3]; out: see
 * om_fwd_out.  Deterministic: no atomics, identical results run to run.
 * Rays with non-finite o or d place no sample and return C = c_bg.
 */
int om_render(const om_scene* scene, const float* o, const float* d, int64_t n,
              const om_params* p, const om_fwd_out* out, void* stream);

/*
 * The two stages of om_render, callable separately (same arguments and
 * outputs; om_render == om_march followed by om_deferred_mlp):
 *  - om_march: placement, feature gather, activations and compositing
 *    (Sec. 4.1 / 4.4, Eq. 1-3); writes out->F, out->T, out->n_placed,
 *    out->n_eval (out->C is not touched and may be NULL);
 *  - om_deferred_mlp: the deferred MLP and final colour (Eq. 4); reads
 *    out->F, out->T, out->n_eval and d, writes out->C.
 */
int om_march(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
             const om_fwd_out* out, void* stream);
int om_deferred_mlp(const om_scene* scene, const float* d, int64_t n, const om_params* p,
                    const om_fwd_out* out, void* stream);

/*
 * Backward of om_render for a per-ray colour loss (derived from Eq. 1-4).
 * saved: the om_fwd_out written by om_render for the same scene, rays and
 * parameters (C is not read; batch_wv is used when non-NULL).  dL_dC:
 * device float32 [n][3].  Gradients are ADDED with float32 atomics into g
 * (grid, planes, MLP; no ray gradient); per-sample features are
 * recomputed, not stored.  Summation order of the atomics is not
 * deterministic.  The MLP part is differentiated in float32 regardless of
 * p->mlp_bf16.  OM_U8 and sparse-block scenes are render only: the
 * backward and the fused step return OM_ERR_UNSUPPORTED for them.
 *
 * The backward runs in two stages: the deferred MLP's backward (derivative
 * of Eq. 4) turns dL_dC (and dL_dF of om_render_backward_ex) into one total
 * dL/dF per ray and the MLP parameter gradients; the march backward
 * (derivative of Eq. 1-3) then distributes that dL/dF over the samples.
 * The march backward takes the rays longest first (by their number of
 * 16-sample batches), handed to its waves on demand.  The per-ray hand-over
 * between the stages (8 floats: dL/dF and dL/dC . c_bg), that ray order and
 * its scheduling counters live in `workspace`: caller-owned device memory
 * of at least om_render_backward_workspace_size(n) bytes, 256-byte aligned,
 * overwritten (OM_ERR_INVALID if it is smaller or misaligned).  The call
 * allocates nothing.
 */
int om_render_backward(const om_scene* scene, const float* o, const float* d, int64_t n,
                       const om_params* p, const om_fwd_out* saved, const float* dL_dC,
                       void* workspace, int64_t workspace_bytes, const om_grads* g, void* stream);

/* Workspace bytes om_render_backward(_ex) needs for n rays (0 for n = 0;
 * else 32 n and 4 n, each rounded up to a multiple of 256, plus 1024), or
 * -1 (with om_last_error set) if n < 0. */
int64_t om_render_backward_workspace_size(int64_t n);

/*
 * om_render_backward with an extra upstream gradient on the composited
 * features: dL_dF (device float32 [n][7], or NULL = zero) is the gradient
 * of a loss term that reads F directly (the view-smoothness loss of
 * om_smooth_loss), added to what flows back from dL_dC before the march
 * backward distributes it over the samples.  om_render_backward(...) is
 * om_render_backward_ex(..., dL_dC, NULL, workspace, workspace_bytes, g,
 * stream).
 */
int om_render_backward_ex(const om_scene* scene, const float* o, const float* d, int64_t n,
                          const om_params* p, const om_fwd_out* saved, const float* dL_dC,
                          const float* dL_dF, void* workspace, int64_t workspace_bytes,
                          const om_grads* g, void* stream);

/*
 * View-smoothness regulariser of Sec. 4.2 (Eq. 9-10) on the deferred MLP G
 * of the scene: L = weight * sum_r sum_p S(d_r, s_rp) ||G(F_r, s_rp) -
 * G(F_r, d_r)||^2 with s_rp = d_r + perturb[r][p] (used as it is, not
 * renormalised) and S the cosine similarity.  The Gaussian perturbations
 * of Eq. 9 are drawn by the caller.  F: device float32 [n][7] (the
 * composited features of om_render); d: [n][3]; perturb: [n][P][3],
 * 1 <= P <= 64; no direction or d + perturb may be the zero vector.
 * loss: optional device float[1] (overwritten; a float32 sum whose order
 * of float32 atomics is not deterministic); dL_dF: optional
 * device float32 [n][7] into which dL/dF is ADDED (pass it to
 * om_render_backward_ex); grad_mlp: optional device float32
 * [OM_MLP_NPARAMS(dir_freqs)] into which dL/dW is ADDED (float32 atomics, order not
 * deterministic).  Evaluated in float32 regardless of the scene dtype.
 */
int om_smooth_loss(const om_scene* scene, const float* F, const float* d, int64_t n,
                   const float* perturb, int32_t P, float weight, float* loss,
                   float* dL_dF, float* grad_mlp, void* stream);

/*
 * L2 loss in float64, for finite-difference gradient checks:
 * *out = sum over n rays and 3 channels of (C - target)^2 / (3 n).
 * C, target: device float32 [n][3]; out: device double[1] (overwritten).
 * Summed by one workgroup in a fixed order: the same colours always give
 * the same bits.  This is the library's only float64 arithmetic.
 */
int om_l2_loss_fp64(const float* C, const float* target, int64_t n, double* out, void* stream);

/*
 * Gradient of the same L2 loss with respect to C, for a training step that
 * stays inside the library: dL_dC[r][c] = 2 (C[r][c] - target[r][c]) / (3 n).
 * C, target, dL_dC: device float32 [n][3] (dL_dC may alias neither input).
 * loss_out: optional device float[1] that receives the loss as a float32
 * sum in a fixed order (overwritten), or NULL.
 */
int om_l2_loss_grad(const float* C, const float* target, int64_t n, float* dL_dC,
                    float* loss_out, void* stream);

/*
 * Fused training step for an L2 photometric loss, everything on `stream`:
 * the forward of om_render (writing out->C, T, F, n_placed, n_eval), the
 * gradient dL/dC = 2 (C - target) / (3 n) of the loss of om_l2_loss_fp64,
 * and om_render_backward, which ADDS the parameter gradients into g.  The
 * forward also records the per-batch sums of w v (see om_fwd_out.batch_wv)
 * so that the backward replays the samples once.  target: device float32
 * [n][3].  workspace: caller-owned device memory of at least
 * om_render_fwd_bwd_l2_workspace_size(n, p) bytes, 256-byte aligned; it
 * holds dL/dC, the backward's workspace (om_render_backward) and the
 * per-batch sums (out->batch_wv is ignored).
 * loss: optional device float[1] receiving the loss as om_l2_loss_grad
 * computes it (overwritten), or NULL.  Equivalent to om_render +
 * om_l2_loss_grad + om_render_backward.  Cites: Eq. 1-4 (forward) and
 * their derivative.
 */
int om_render_fwd_bwd_l2(const om_scene* scene, const float* o, const float* d, int64_t n,
                         const om_params* p, const float* target, const om_fwd_out* out,
                         void* workspace, int64_t workspace_bytes, float* loss,
                         const om_grads* g, void* stream);

/* Workspace bytes om_render_fwd_bwd_l2 needs for n rays and p->n_max, or
 * -1 (with om_last_error set) if n < 0 or p is invalid. */
int64_t om_render_fwd_bwd_l2_workspace_size(int64_t n, const om_params* p);

/*
 * om_render_fwd_bwd_l2 for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc.  Same arguments and results as om_render_fwd_bwd_l2
 * minus the workspace: the workspace (dL/dC, the backward's workspace and
 * the per-batch sums) lives
 * in a fixed array of om_render_fwd_bwd_l2_noalloc_max_bytes() bytes
 * (64 MiB) inside the library, one per GPU, held until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Limit: om_render_fwd_bwd_l2_workspace_size(n, p) must not
 * exceed that size (e.g. 135,296 rays at n_max 256, 419,421 at n_max 64),
 * else OM_ERR_UNSUPPORTED with om_last_error naming the sizes.  Every
 * call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call overwrites what it reads before reading it): calls
 * that overlap on one GPU (concurrent streams, threads) race and must be
 * serialised by the caller.
 */
int om_render_fwd_bwd_l2_noalloc(const om_scene* scene, const float* o, const float* d, int64_t n,
                                 const om_params* p, const float* target, const om_fwd_out* out,
                                 float* loss, const om_grads* g, void* stream);

/* Size in bytes of the fixed workspace of om_render_fwd_bwd_l2_noalloc. */
int64_t om_render_fwd_bwd_l2_noalloc_max_bytes(void);

/*
 * Interval-span regulariser of Sec. 4.1, Eq. 5, scaled by `weight` (the
 * schedule's lambda): L = weight * sum over the My x Mx grid points of
 * (z_max - z_min)^2.  occ: device float32 [cells][2].  loss: optional
 * device float[1] receiving L, a float32 sum in a fixed order
 * (overwritten); grad_occ: optional device float32 [cells][2] into which
 * dL/d(z_min, z_max) = 2 weight (z_max - z_min) (-1, +1) is ADDED.
 */
int om_occ_interval_loss(const float* occ, int64_t cells, float weight, float* loss, float* grad_occ,
                         void* stream);

/*
 * Baking to 8-bit storage (Sec. 4.4).  For one feature source, x: device
 * float32 [n][8] (no NaN), n >= 1.
 *  - om_feature_range: per-channel (min, max) into the device float32
 *    [8][2] buffer minmax (overwritten; it also serves as the reduction's
 *    scratch, so it must not alias x).
 *  - om_quant_params (host only): from a host copy of minmax, the
 *    per-channel lo = min and step = fl32((max - min) / 255) (host float[8]
 *    each), so that the codes 0..255 span the channel's range.
 *  - om_quantize_u8: out (device uint8 [n][8]) receives
 *    q = clamp(rint(fl32(fl32(x - lo) * inv)), 0, 255) per channel, with
 *    inv = fl32(1 / step) (0 when step = 0) and lo, step host float[8];
 *    the rounding is to nearest, ties to even; NaN encodes as 0.
 * The 8-bit scene is then created with dtype OM_U8 and these (lo, step)
 * per source.
 */
int om_feature_range(const float* x, int64_t n, float* minmax, void* stream);
int om_quant_params(const float* minmax_host, float* lo, float* step);
int om_quantize_u8(const float* x, int64_t n, const float* lo, const float* step, uint8_t* out, void* stream);

/*
 * Sparse voxel blocks for a dense scene handle (its grid, occupancy plane and
 * dtype), block edge B = 2^block_shift cells (1 <= block_shift <= 5):
 *  - om_sparse_grid_index: writes the block index grid_blocks (device int32
 *    [ceil((Lz-1)/B)][ceil((Ly-1)/B)][ceil((Lx-1)/B)], idx_len entries) and
 *    returns the number of kept blocks (>= 0), or -1 with om_last_error
 *    set.  A block is kept if an occupancy column overlapping its xy extent
 *    (one column of padding) has an interval meeting its z extent (one cell
 *    of padding), so every block holding a placeable sample is kept.  Ids
 *    are 1.. in index order.  Synchronous: it waits for `stream`.
 *  - om_sparse_grid_fill: copies the kept blocks into the caller's atlas
 *    (device, (n_blocks + 1) (B + 1)^3 vertices of the scene dtype, 16-byte
 *    aligned) and zeroes block 0.
 * The sparse scene is then created with the atlas as grid and grid_blocks,
 * block_shift and n_blocks set; it renders exactly like the dense one.
 */
int64_t om_sparse_grid_index(const om_scene* scene, int block_shift, int32_t* grid_blocks, int64_t idx_len,
                             void* stream);
int om_sparse_grid_fill(const om_scene* scene, int block_shift, const int32_t* grid_blocks, int64_t n_blocks,
                        void* atlas, void* stream);

/*
 * bfloat16 shadow of float32 parameters (the storage form of Sec. 4.4 kept
 * in 16 bits; the re-cast after each optimiser step of a bfloat16 scene
 * trained through float32 master copies): dst[i] = the upper 16 bits of
 * src[i] rounded to nearest, ties to even.  Finite values beyond the largest
 * bfloat16 become infinities of their sign; NaN stays NaN (quiet, same
 * sign); infinities and signed zeros are kept.  src: device float32 [n];
 * dst: device uint16 [n] (bfloat16 bit patterns), not overlapping src; both
 * 16-byte aligned.  n = 0 is a no-op.  Asynchronous on `stream`.
 */
int om_cast_bf16(const float* src, int64_t n, uint16_t* dst, void* stream);

/*
 * Locality order of a batch of rays (scheduling only; not part of the
 * method: each ray is rendered on its own, Eq. 1-3, so every result is the
 * same in any order).  Rays that cross the scene near one another read the
 * same grid and plane rows; rendered next to each other they share those
 * rows in the caches.  Callers whose rays come in no such order (row-major
 * pixels, random training rays) order them here, render the reordered
 * copies, and take results back with om_scatter_rows (or bring per-ray
 * inputs along, such as training targets, with om_gather_rows).
 *  - Key of a ray: the point where it meets the horizontal plane halfway up
 *    the scene box, on a 256 x 256 lattice over the box footprint (clamped
 *    to its edge), as a 16-bit Morton code; a ray parallel to that plane
 *    takes the cell of its origin, a non-finite point cell 0.
 *  - order: device int32 [n], written with a permutation of 0..n-1 that
 *    lists the rays by key; rays with equal keys keep their input order
 *    within runs of consecutive rays of one 64-ray wave, and such runs of
 *    one key follow one another in an unspecified order (it may differ
 *    between calls).
 *  - o_sorted, d_sorted: device float32 [n][3], written with o[order[i]]
 *    and d[order[i]]; they must not overlap o or d.
 *  - workspace: caller-owned device memory of at least
 *    om_order_rays_workspace_size(n) bytes, 256-byte aligned (the key
 *    histogram and one 16-bit key per ray).  n = 0 is a no-op and needs
 *    none.  n must not exceed 2^31 - 1.
 * Asynchronous on `stream`; calls that share a workspace must not overlap.
 * om_order_rays_workspace_size returns -1 (and sets the error) for n
 * outside [0, 2^31 - 1].
 */
int om_order_rays(const om_scene* scene, const float* o, const float* d, int64_t n, int32_t* order, float* o_sorted,
                  float* d_sorted, void* workspace, int64_t workspace_bytes, void* stream);
int64_t om_order_rays_workspace_size(int64_t n);

/*
 * Row gathers and scatters that apply a ray order to per-ray data (rows of
 * `cols` float32 values, 1 <= cols <= 64, row-major, device memory):
 *  - om_gather_rows: dst[i] = src[idx[i]] for i < n; src has src_rows rows,
 *    dst n rows.
 *  - om_scatter_rows: dst[idx[i]] = src[i] for i < n; src has n rows, dst
 *    dst_rows rows.  Rows of dst that no index names are left as they are;
 *    with repeated indices the surviving row is unspecified.
 * Index entries outside [0, src_rows) (gather) or [0, dst_rows) (scatter)
 * are skipped: the gather leaves that row of dst unwritten.  dst must not
 * overlap src.  n = 0 is a no-op.  Asynchronous on `stream`.
 */
int om_gather_rows(const float* src, int64_t src_rows, int cols, const int32_t* idx, int64_t n, float* dst,
                   void* stream);
int om_scatter_rows(const float* src, int cols, const int32_t* idx, int64_t n, float* dst, int64_t dst_rows,
                    void* stream);

/* Message for the last failing call on this thread ("" if none). */
const char* om_last_error(void);

/* Static description of a status code. */
const char* om_status_str(int status);

/* Library version: major * 10000 + minor * 100 + patch. */
int om_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OMERF_H */
