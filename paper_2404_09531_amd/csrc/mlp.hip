// mlp.hip -- deferred view-dependent MLP (Eq. 4) and the L2 loss kernels.
//
// C = F[0:3] + [n_eval > 0] G(F, d) + T c_bg,  G = sigmoid(W3 relu(W2 relu(W1 x + b1) + b2) + b3),
// x = [F (7), enc(d)] with enc(d) = d or d with four sine/cosine
// frequencies (NIN = 10 or 34, see mlp_input).
//
// k_mlp_f32      : one lane per ray, float32 FMA, weights read through the
//                  scalar path (uniform addresses).
// k_mlp_bf16     : bfloat16 operands on MFMA (v_mfma_f32_16x16x16_bf16) with
//                  float32 accumulation, 16 rays per MFMA tile.  Each layer
//                  is computed transposed, H^T = W X^T, with the weights as
//                  the A operand: the accumulator layout of one layer (lane l
//                  holds rows 4(l/16)..+3 of column l%16) is exactly the B
//                  operand layout of the next, so no data moves between
//                  layers.  Biases enter as the accumulator's initial value.
// k_mlp_bwd      : the backward of G ahead of the backward march: per ray
//                  dL/dF for the march, and the parameter gradients summed
//                  over each wave's four rays on MFMA (v_mfma_f32_16x16x4_f32).
// Also here: the L2 loss, the occupancy pyramid and interval loss, and the
// view-smoothness loss (Eq. 9-10).
#include "omerf_launch.h"

namespace omerf {

template <int NIN>
__global__ __launch_bounds__(kBlock) void k_mlp_f32(const float* __restrict__ W, RayParams rp,
                                                    const float* __restrict__ d_, int64_t n,
                                                    const float* __restrict__ F, const float* __restrict__ T,
                                                    const int32_t* __restrict__ n_eval, float* __restrict__ C) {
    using L = MlpLayout<NIN>;
    const int64_t r = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (r >= n) return;
    float f7[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) f7[c] = F[r * 7 + c];
    float x[NIN];
    mlp_input<NIN>(f7, make_float3(d_[r * 3 + 0], d_[r * 3 + 1], d_[r * 3 + 2]), x);
    float h1[16], h2[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        float z = W[L::B1 + j];
#pragma unroll
        for (int c = 0; c < NIN; ++c) z += W[L::W1 + j * NIN + c] * x[c];
        h1[j] = fmaxf(z, 0.0f);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        float z = W[L::B2 + j];
#pragma unroll
        for (int c = 0; c < 16; ++c) z += W[L::W2 + j * 16 + c] * h1[c];
        h2[j] = fmaxf(z, 0.0f);
    }
    const bool gate = n_eval[r] > 0;
    const float t = T[r];
    const float bg[3] = {rp.bg0, rp.bg1, rp.bg2};
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        float z = W[L::B3 + o];
#pragma unroll
        for (int c = 0; c < 16; ++c) z += W[L::W3 + o * 16 + c] * h2[c];
        const float g = gate ? sigmoidf_fast(z) : 0.0f;
        C[r * 3 + o] = x[o] + g + t * bg[o];
    }
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
    // round to nearest even
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 v;
    v[0] = to_bf16(a);
    v[1] = to_bf16(b);
    v[2] = to_bf16(c);
    v[3] = to_bf16(d);
    return v;
}

// Entry k of the MLP input x = [F (7), enc(d)] (see mlp_input).
template <int NIN>
__device__ __forceinline__ float mlp_x_at(const float* F7, const float* d3, int k) {
    if (k < 7) return F7[k];
    if (k < 10) return d3[k - 7];
    if (NIN == 10 || k >= NIN) return 0.0f;
    const int e = k - 10, f = e / 6, rr = e - 6 * f, comp = rr < 3 ? rr : rr - 3;
    const float v = (float)(1 << f) * d3[comp];
    float sn, cs;
    sincosf(v, &sn, &cs);
    return rr < 3 ? sn : cs;
}

template <int NIN>
__global__ __launch_bounds__(kBlock) void k_mlp_bf16(const float* __restrict__ W, RayParams rp,
                                                     const float* __restrict__ d_, int64_t n,
                                                     const float* __restrict__ F, const float* __restrict__ T,
                                                     const int32_t* __restrict__ n_eval, float* __restrict__ C) {
    using L = MlpLayout<NIN>;
    constexpr int KT = (NIN + 15) / 16;  // k-tiles of layer 1 (zero padded)
    const int lane = threadIdx.x & 63;
    const int col = lane & 15;  // ray within the tile / row of A
    const int q = lane >> 4;    // k-block (A, B) / row-block (C, D)
    // A operands: row `col`, k = 16 kt + 4q .. +3 (zero padded).
    bf16x4 A1[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
        float a1[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * kt + 4 * q + j;
            a1[j] = k < NIN ? W[L::W1 + col * NIN + k] : 0.0f;
        }
        A1[kt] = pack4(a1[0], a1[1], a1[2], a1[3]);
    }
    float a2[4], a3[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * q + j;
        a2[j] = W[L::W2 + col * 16 + k];
        a3[j] = col < 3 ? W[L::W3 + col * 16 + k] : 0.0f;
    }
    const bf16x4 A2 = pack4(a2[0], a2[1], a2[2], a2[3]);
    const bf16x4 A3 = pack4(a3[0], a3[1], a3[2], a3[3]);
    // Accumulator initial values: bias of output row 4q + i.
    f32x4 c1, c2, c3;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = 4 * q + i;
        c1[i] = W[L::B1 + m];
        c2[i] = W[L::B2 + m];
        c3[i] = m < 3 ? W[L::B3 + m] : 0.0f;
    }
    const int64_t tiles = (n + 15) / 16;
    const int64_t wave = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    // Every input of a tile (F, d, T, n_eval) is loaded before its MFMAs:
    // one memory round trip per tile.
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const int64_t r = tile * 16 + col;
        const bool valid = r < n;
        float f7[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, d3[3] = {0.f, 0.f, 0.f}, t = 0.0f;
        bool gate = false;
        if (valid) {
#pragma unroll
            for (int c = 0; c < 7; ++c) f7[c] = F[r * 7 + c];
#pragma unroll
            for (int c = 0; c < 3; ++c) d3[c] = d_[r * 3 + c];
            t = T[r];
            gate = n_eval[r] > 0;
        }
        // Layer 1 over the k-tiles: B operand x[k] of ray `col`, k = 16 kt + 4q .. +3.
        f32x4 h = c1;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            float xv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[j] = valid ? mlp_x_at<NIN>(f7, d3, 16 * kt + 4 * q + j) : 0.0f;
            h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A1[kt], pack4(xv[0], xv[1], xv[2], xv[3]), h, 0, 0, 0);
        }
        const bf16x4 B2 = pack4(fmaxf(h[0], 0.0f), fmaxf(h[1], 0.0f), fmaxf(h[2], 0.0f), fmaxf(h[3], 0.0f));
        h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A2, B2, c2, 0, 0, 0);
        const bf16x4 B3 = pack4(fmaxf(h[0], 0.0f), fmaxf(h[1], 0.0f), fmaxf(h[2], 0.0f), fmaxf(h[3], 0.0f));
        h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A3, B3, c3, 0, 0, 0);
        // Rows 0..2 of the output live in lanes with q == 0.
        if (q == 0 && valid) {
            C[r * 3 + 0] = f7[0] + (gate ? sigmoidf_fast(h[0]) : 0.0f) + t * rp.bg0;
            C[r * 3 + 1] = f7[1] + (gate ? sigmoidf_fast(h[1]) : 0.0f) + t * rp.bg1;
            C[r * 3 + 2] = f7[2] + (gate ? sigmoidf_fast(h[2]) : 0.0f) + t * rp.bg2;
        }
    }
}

// ---------------------------------------------------------------------------
// Group-cooperative MLP (one ray per 16-lane group, hidden unit h of both
// hidden layers in lane h) and its backward, used by the render's MLP
// backward and by the view-smoothness loss.
// ---------------------------------------------------------------------------
struct MlpAct {
    float z1, h1, z2, h2;  // this lane's hidden unit, both layers
    float g[3];            // G (after the sigmoid), the same on every lane
};

template <int NIN>
__device__ __forceinline__ MlpAct group_mlp_fwd(const float* W, const float* x, int h) {
    using L = MlpLayout<NIN>;
    MlpAct a;
    a.z1 = W[L::B1 + h];
#pragma unroll
    for (int c = 0; c < NIN; ++c) a.z1 += W[L::W1 + h * NIN + c] * x[c];
    a.h1 = fmaxf(a.z1, 0.0f);
    a.z2 = W[L::B2 + h];
#pragma unroll
    for (int j = 0; j < 16; ++j) a.z2 += W[L::W2 + h * 16 + j] * __shfl(a.h1, j, kGroup);
    a.h2 = fmaxf(a.z2, 0.0f);
#pragma unroll
    for (int r = 0; r < 3; ++r) a.g[r] = sigmoidf_fast(W[L::B3 + r] + g_sum(W[L::W3 + r * 16 + h] * a.h2));
    return a;
}

// MLP parameter gradients accumulated over the rays a wave visits.  The
// weight matrices are reduced on MFMA (v_mfma_f32_16x16x4_f32, A 16x4,
// B 4x16): with the wave's four rays in its four groups, a per-lane value
// of layer-2 pre-activation gradient dz2 is the A operand entry
// A[h][g] (lane 16 g + h) and a per-lane activation h1 the B operand entry
// B[g][j] (lane 16 g + j), so one instruction adds sum_g dz2_g h1_g^T over
// the four rays to a 16x16 accumulator, lane l holding rows
// 4 (l / 16) .. +3 of column l % 16.  W1 is reduced against the input
// extended by a constant 1, in column slices of 16 (its column NIN is the
// b1 gradient); b2 and b3 are per-lane sums.
template <int NIN>
struct MlpGradAcc {
    static constexpr int kSlices = (NIN + 1 + 15) / 16;
    f32x4 w1[kSlices];
    f32x4 w2, w3;
    float b2, b3;
    __device__ void zero() {
#pragma unroll
        for (int s = 0; s < kSlices; ++s) w1[s] = f32x4{0.f, 0.f, 0.f, 0.f};
        w2 = w3 = f32x4{0.f, 0.f, 0.f, 0.f};
        b2 = b3 = 0.0f;
    }
};

// Entry 16 s + h of [x, 1] (0 past it), the lane's B operand of W1 slice s.
template <int NIN>
__device__ __forceinline__ float mlp_x_slice(const float* F7, const float* d3, int s, int h) {
    const int k = 16 * s + h;
    return k < NIN ? mlp_x_at<NIN>(F7, d3, k) : (k == NIN ? 1.0f : 0.0f);
}

// Backward of group_mlp_fwd for dL/dG = dG (the same on every lane of the
// group; zero for a group without a ray, whose activations must be finite):
// adds dL/dx[0..6] to dx7 (the same on every lane) and the parameter
// gradients to acc.  xs[s] = mlp_x_slice(..., s, h).  All 64 lanes of the
// wave execute it (MFMA).
template <int NIN>
__device__ __forceinline__ void wave_mlp_bwd(const float* W, const float* xs, int h, const MlpAct& a,
                                             const float* dG, MlpGradAcc<NIN>& acc, float* dx7) {
    using L = MlpLayout<NIN>;
    float dz3[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) dz3[r] = dG[r] * a.g[r] * (1.0f - a.g[r]);
    const float dh2 = W[L::W3 + h] * dz3[0] + W[L::W3 + 16 + h] * dz3[1] + W[L::W3 + 32 + h] * dz3[2];
    const float dz2 = a.z2 > 0.0f ? dh2 : 0.0f;
    float dh1 = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) dh1 += W[L::W2 + j * 16 + h] * __shfl(dz2, j, kGroup);
    const float dz1 = a.z1 > 0.0f ? dh1 : 0.0f;
#pragma unroll
    for (int c = 0; c < 7; ++c) dx7[c] += g_sum(W[L::W1 + h * NIN + c] * dz1);
    const float d3 = h == 0 ? dz3[0] : h == 1 ? dz3[1] : h == 2 ? dz3[2] : 0.0f;
    acc.w2 = __builtin_amdgcn_mfma_f32_16x16x4f32(dz2, a.h1, acc.w2, 0, 0, 0);
    acc.w3 = __builtin_amdgcn_mfma_f32_16x16x4f32(d3, a.h2, acc.w3, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < MlpGradAcc<NIN>::kSlices; ++s)
        acc.w1[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(dz1, xs[s], acc.w1[s], 0, 0, 0);
    acc.b2 += dz2;
    acc.b3 += d3;
}

// Adds a wave's accumulators to the block's LDS copy of the gradient
// (SIZE floats, MlpLayout order).
template <int NIN>
__device__ __forceinline__ void mlp_grad_to_lds(const MlpGradAcc<NIN>& acc, int lane, float* sW) {
    using L = MlpLayout<NIN>;
    const int col = lane & 15, row0 = (lane >> 4) * 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = row0 + r;
        atomicAdd(&sW[L::W2 + row * 16 + col], acc.w2[r]);
        if (row < 3) atomicAdd(&sW[L::W3 + row * 16 + col], acc.w3[r]);
#pragma unroll
        for (int s = 0; s < MlpGradAcc<NIN>::kSlices; ++s) {
            const int c = 16 * s + col;
            if (c < NIN)
                atomicAdd(&sW[L::W1 + row * NIN + c], acc.w1[s][r]);
            else if (c == NIN)
                atomicAdd(&sW[L::B1 + row], acc.w1[s][r]);
        }
    }
    atomicAdd(&sW[L::B2 + col], acc.b2);
    if (col < 3) atomicAdd(&sW[L::B3 + col], acc.b3);
}

// Adds the block's LDS gradient to gmlp (one float atomic per nonzero entry).
template <int NIN>
__device__ __forceinline__ void mlp_grad_flush(const float* sW, float* gmlp) {
    for (int i = threadIdx.x; i < MlpLayout<NIN>::SIZE; i += blockDim.x) {
        const float v = sW[i];
        if (v != 0.0f) unsafeAtomicAdd(gmlp + i, v);
    }
}

// ---------------------------------------------------------------------------
// Backward of the deferred MLP of the render (Eq. 4), ahead of the backward
// march.  C = F[0:3] + [n_eval > 0] G(F, d) + T c_bg gives, per ray,
//
//   G8 = [dL/dF (7), dL/dC . c_bg],
//   dL/dF = dL/dC on the diffuse part + [n_eval > 0] dL/dx[0..6] of G
//           + dL/dF of losses on F itself (dF, optional),
//
// which is all the march needs of the MLP, and the MLP parameter gradients.
// One ray per 16-lane group; a wave walks quads of consecutive rays so that
// its four groups feed the MFMA reduction together.  Large blocks (1024
// threads; 512 for the 34-input MLP, whose encoded input needs more than 128
// registers), each over a contiguous range of quads, reduce in LDS before
// one set of global atomics per block.
// ---------------------------------------------------------------------------
template <int NIN>
constexpr int mlp_bwd_block() { return NIN == 10 ? 1024 : 512; }

template <int NIN>
__global__ __launch_bounds__(mlp_bwd_block<NIN>()) void k_mlp_bwd(const float* __restrict__ W, RayParams rp,
                                                          const float* __restrict__ F, const float* __restrict__ d_,
                                                          const int32_t* __restrict__ n_eval,
                                                          const float* __restrict__ dC, const float* __restrict__ dF,
                                                          int64_t n, int64_t quads_per_block, float* __restrict__ G8,
                                                          float* __restrict__ gmlp) {
    constexpr int kThreads = mlp_bwd_block<NIN>();
    __shared__ float sW[MlpLayout<NIN>::SIZE];
    for (int i = threadIdx.x; i < MlpLayout<NIN>::SIZE; i += kThreads) sW[i] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63, gl = lane & (kGroup - 1), g = lane >> 4;
    const int64_t nq = (n + 3) / 4;
    const int64_t q0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * quads_per_block;
    const int64_t q1 = min(nq, q0 + quads_per_block);
    MlpGradAcc<NIN> acc;
    acc.zero();
    for (int64_t q = q0 + (threadIdx.x >> 6); q < q1; q += kThreads / 64) {
        const int64_t ray = q * 4 + g;
        const bool in = ray < n;
        const bool live = in && n_eval[ray] > 0;  // G gated off without samples
        float f7[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, d3[3] = {0.f, 0.f, 0.f}, dc[3] = {0.f, 0.f, 0.f};
        if (in) {
#pragma unroll
            for (int c = 0; c < 3; ++c) dc[c] = dC[ray * 3 + c];
        }
        if (live) {
#pragma unroll
            for (int c = 0; c < 7; ++c) f7[c] = F[ray * 7 + c];
#pragma unroll
            for (int c = 0; c < 3; ++c) d3[c] = d_[ray * 3 + c];
        }
        // For the 34-input MLP the weights are re-read (L1 hits) in every
        // iteration instead of being hoisted into registers for the whole
        // loop, which would leave too few registers for the large blocks;
        // the 10-input MLP keeps them in registers.
        const float* Wq = W;
        if (NIN != 10) asm volatile("" : "+s"(Wq));
        float x[NIN];
        mlp_input<NIN>(f7, make_float3(d3[0], d3[1], d3[2]), x);
        const MlpAct a = group_mlp_fwd<NIN>(Wq, x, gl);
        float xs[MlpGradAcc<NIN>::kSlices];
#pragma unroll
        for (int s = 0; s < MlpGradAcc<NIN>::kSlices; ++s) xs[s] = mlp_x_slice<NIN>(f7, d3, s, gl);
        const float dG[3] = {live ? dc[0] : 0.0f, live ? dc[1] : 0.0f, live ? dc[2] : 0.0f};
        float g8[8] = {dc[0], dc[1], dc[2], 0.f, 0.f, 0.f, 0.f, dc[0] * rp.bg0 + dc[1] * rp.bg1 + dc[2] * rp.bg2};
        wave_mlp_bwd<NIN>(Wq, xs, gl, a, dG, acc, g8);
        if (in && gl < 8) {
            float v = g8[0];
#pragma unroll
            for (int c = 1; c < 8; ++c)
                if (gl == c) v = g8[c];
            if (dF && gl < 7) v += dF[ray * 7 + gl];
            G8[ray * 8 + gl] = v;
        }
    }
    mlp_grad_to_lds<NIN>(acc, lane, sW);
    __syncthreads();
    mlp_grad_flush<NIN>(sW, gmlp);
}

template <int NIN>
static void launch_mlp_bwd_nin(const float* W, const RayParams& rp, const float* F, const float* d,
                               const int32_t* n_eval, const float* dC, const float* dF, int64_t n, float* G8,
                               float* gmlp, hipStream_t s) {
    // At least 8 quads per wave; at most 512 blocks, whose LDS sums then
    // cost at most 512 global atomics per MLP parameter.
    const int64_t nq = (n + 3) / 4;
    const int64_t waves = mlp_bwd_block<NIN>() / 64;
    int64_t qpb = (nq + 511) / 512;
    if (qpb < 8 * waves) qpb = 8 * waves;
    qpb = (qpb + waves - 1) / waves * waves;
    const int64_t nb = (nq + qpb - 1) / qpb;
    hipLaunchKernelGGL(k_mlp_bwd<NIN>, dim3((unsigned)nb), dim3(mlp_bwd_block<NIN>()), 0, s, W, rp, F, d, n_eval, dC,
                       dF, n, qpb, G8, gmlp);
}

hipError_t launch_mlp_bwd(const float* W, int mlp_in, const RayParams& rp, const float* F, const float* d,
                          const int32_t* n_eval, const float* dC, const float* dF, int64_t n, float* G8, float* gmlp,
                          hipStream_t s) {
    if (n == 0) return hipGetLastError();
    if (mlp_in == 34)
        launch_mlp_bwd_nin<34>(W, rp, F, d, n_eval, dC, dF, n, G8, gmlp, s);
    else
        launch_mlp_bwd_nin<10>(W, rp, F, d, n_eval, dC, dF, n, G8, gmlp, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// L2 loss and its gradient.  dL/dC is elementwise float32 over the whole
// grid.  The loss value is summed by ONE workgroup in a fixed order -- each
// lane a fixed strided subset, then a fixed butterfly over the wave and a
// fixed sum over the waves -- so two calls on the same colours return the
// same bits (a cross-block atomic sum would not).  It is accumulated in
// float64 only for the finite-difference checks (om_l2_loss_fp64) and in
// float32 for the optional loss of a training step.
// ---------------------------------------------------------------------------
constexpr int kLossBlock = 1024;

__global__ __launch_bounds__(kBlock) void k_l2_grad(const float* __restrict__ C, const float* __restrict__ tgt,
                                                    int64_t n, float scale2, float* __restrict__ dC) {
    const int64_t m = n * 3;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
        dC[i] = scale2 * (C[i] - tgt[i]);
}

template <class Acc>
__global__ __launch_bounds__(kLossBlock) void k_l2_loss(const float* __restrict__ C, const float* __restrict__ tgt,
                                                       int64_t n, Acc* __restrict__ loss) {
    __shared__ Acc part[kLossBlock / 64];
    const int64_t m = n * 3;
    Acc s = 0;
    for (int64_t i = threadIdx.x; i < m; i += kLossBlock) {
        const Acc e = (Acc)C[i] - (Acc)tgt[i];
        s += e * e;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t = 0;
        for (int w = 0; w < kLossBlock / 64; ++w) t += part[w];
        *loss = t / (Acc)3 / (Acc)n;
    }
}

template <int NIN>
static void launch_mlp_nin(const float* W, bool bf16, const RayParams& rp, const float* d, int64_t n, const float* F,
                           const float* T, const int32_t* n_eval, float* C, hipStream_t s) {
    if (bf16) {
        const int64_t tiles = (n + 15) / 16;
        int64_t blocks = (tiles + 3) / 4;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_mlp_bf16<NIN>, dim3((unsigned)blocks), dim3(kBlock), 0, s, W, rp, d, n, F, T, n_eval, C);
    } else {
        const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_mlp_f32<NIN>, dim3(blocks), dim3(kBlock), 0, s, W, rp, d, n, F, T, n_eval, C);
    }
}

hipError_t launch_mlp(const float* W, int mlp_in, bool bf16, const RayParams& rp, const float* d, int64_t n,
                      const float* F, const float* T, const int32_t* n_eval, float* C, hipStream_t s) {
    if (mlp_in == 34)
        launch_mlp_nin<34>(W, bf16, rp, d, n, F, T, n_eval, C, s);
    else
        launch_mlp_nin<10>(W, bf16, rp, d, n, F, T, n_eval, C, s);
    return hipGetLastError();
}

hipError_t launch_l2(const float* C, const float* tgt, int64_t n, float* dC, float* loss, hipStream_t s) {
    if (dC) {
        int64_t blocks = (n * 3 + kBlock - 1) / kBlock;
        if (blocks > 2048) blocks = 2048;
        const float scale2 = (float)(2.0 / (3.0 * (double)n));  // 2 / (3 n), rounded once on the host
        hipLaunchKernelGGL(k_l2_grad, dim3((unsigned)blocks), dim3(kBlock), 0, s, C, tgt, n, scale2, dC);
    }
    if (loss) hipLaunchKernelGGL(k_l2_loss<float>, dim3(1), dim3(kLossBlock), 0, s, C, tgt, n, loss);
    return hipGetLastError();
}

hipError_t launch_l2_fp64(const float* C, const float* tgt, int64_t n, double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_l2_loss<double>, dim3(1), dim3(kLossBlock), 0, s, C, tgt, n, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Occupancy pyramid: one level from the one below.  Each output block holds
// (min z_min, max z_max) over the non-empty entries of its 2 x 2 children
// (an entry is empty when not z_min <= z_max, NaN included); a block with
// no non-empty child gets (+inf, -inf), which no segment meets.
// ---------------------------------------------------------------------------
__global__ void k_occ_pool(const float2* __restrict__ src, int sw, float2* __restrict__ dst, int dw, int dh) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)dw * dh) return;
    const int i = (int)(idx % dw), j = (int)(idx / dw);
    float lo = INFINITY, hi = -INFINITY;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float2 z = src[(2 * j + (c >> 1)) * sw + 2 * i + (c & 1)];
        if (z.x <= z.y) {
            lo = fminf(lo, z.x);
            hi = fmaxf(hi, z.y);
        }
    }
    dst[idx] = make_float2(lo, hi);
}

hipError_t launch_occ_pyramid(const float2* occ, int Mx, int My, float2* mips, int levels, hipStream_t s) {
    const float2* src = occ;
    int sw = Mx, sh = My;
    float2* dst = mips;
    for (int l = 1; l <= levels; ++l) {
        const int dw = sw / 2, dh = sh / 2;
        const int64_t cells = (int64_t)dw * dh;
        hipLaunchKernelGGL(k_occ_pool, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, src, sw, dst, dw, dh);
        src = dst;
        dst += cells;
        sw = dw;
        sh = dh;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interval-span regulariser (Eq. 5): weight * sum (z_max - z_min)^2 and its
// gradient 2 weight (z_max - z_min) (-1, +1) added to grad_occ, in float32.
// The loss is summed by one workgroup in a fixed order (see k_l2_loss).
// ---------------------------------------------------------------------------
__global__ void k_occ_grad(const float2* __restrict__ occ, int64_t cells, float weight, float2* __restrict__ grad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += (int64_t)gridDim.x * blockDim.x) {
        const float2 z = occ[i];
        const float g = 2.0f * weight * (z.y - z.x);
        float2 cur = grad[i];
        cur.x -= g;
        cur.y += g;
        grad[i] = cur;
    }
}

__global__ __launch_bounds__(kLossBlock) void k_occ_loss(const float2* __restrict__ occ, int64_t cells, float weight,
                                                        float* __restrict__ loss) {
    __shared__ float part[kLossBlock / 64];
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < cells; i += kLossBlock) {
        const float2 z = occ[i];
        const float span = z.y - z.x;
        s += span * span;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < kLossBlock / 64; ++w) t += part[w];
        *loss = weight * t;
    }
}

hipError_t launch_occ_loss(const float* occ, int64_t cells, float weight, float* loss, float* grad, hipStream_t s) {
    if (grad) {
        int64_t blocks = (cells + 255) / 256;
        if (blocks > 1024) blocks = 1024;
        hipLaunchKernelGGL(k_occ_grad, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const float2*>(occ),
                           cells, weight, reinterpret_cast<float2*>(grad));
    }
    if (loss)
        hipLaunchKernelGGL(k_occ_loss, dim3(1), dim3(kLossBlock), 0, s, reinterpret_cast<const float2*>(occ), cells,
                           weight, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// View-smoothness loss (Sec. 4.2, Eq. 9-10):
// L = weight sum_r sum_p S(d_r, s_rp) ||G(F_r, s_rp) - G(F_r, d_r)||^2,
// s_rp = d_r + delta_rp (the caller draws delta ~ N(0, Sigma)), S the
// cosine similarity.  One (ray, perturbation) pair per 16-lane group, one
// hidden unit per lane: G at d and at s, and the backward of both
// evaluations (dL/dG = +g at s, -g at d; the MLP backward is linear in
// dL/dG), whose parameter gradients are reduced on MFMA per wave and in LDS
// per block (MlpGradAcc); dL/dF is added to dF with float32 atomics (the P
// pairs of a ray land in different groups).  The loss value is a float32
// sum (per group, then one float32 atomic per group).
// ---------------------------------------------------------------------------
__global__ void k_zero_f32(float* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0.0f;
}

template <int NIN>
__global__ __launch_bounds__(kBlock) void k_smooth(const float* __restrict__ W, const float* __restrict__ F,
                                                   const float* __restrict__ d_, int64_t items, int64_t chunk,
                                                   const float* __restrict__ perturb, int P, float weight,
                                                   float* __restrict__ loss, float* __restrict__ dF,
                                                   float* __restrict__ gmlp) {
    __shared__ float sW[MlpLayout<NIN>::SIZE];
    for (int i = threadIdx.x; i < MlpLayout<NIN>::SIZE; i += kBlock) sW[i] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int g = lane >> 4;
    // chunk is a multiple of 16 items, so a block's range is whole quads;
    // each wave walks quads (4 items, one per group) in step.
    const int64_t start = (int64_t)xcd_block(blockIdx.x, gridDim.x) * chunk;
    const int64_t stop = min(items, start + chunk);
    MlpGradAcc<NIN> macc;
    macc.zero();
    float acc = 0.0f;
    for (int64_t it0 = start + 4 * (threadIdx.x >> 6); it0 < stop; it0 += kBlock / kGroup) {
        const int64_t it = it0 + g;
        const bool live = it < stop;
        const int64_t ray = live ? it / P : 0;
        float f7[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, d3[3] = {0.f, 0.f, 0.f}, s3[3] = {0.f, 0.f, 0.f};
        if (live) {
#pragma unroll
            for (int c = 0; c < 7; ++c) f7[c] = F[ray * 7 + c];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                d3[c] = d_[ray * 3 + c];
                s3[c] = d3[c] + perturb[it * 3 + c];
            }
        }
        const float dn = sqrtf(d3[0] * d3[0] + d3[1] * d3[1] + d3[2] * d3[2]);
        const float sn = sqrtf(s3[0] * s3[0] + s3[1] * s3[1] + s3[2] * s3[2]);
        const float cosv = live ? (d3[0] * s3[0] + d3[1] * s3[1] + d3[2] * s3[2]) / (dn * sn) : 0.0f;
        float g7[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        MlpAct ad, as;
        {
            float x[NIN];
            mlp_input<NIN>(f7, make_float3(d3[0], d3[1], d3[2]), x);
            ad = group_mlp_fwd<NIN>(W, x, gl);
        }
        {
            float x[NIN];
            mlp_input<NIN>(f7, make_float3(s3[0], s3[1], s3[2]), x);
            as = group_mlp_fwd<NIN>(W, x, gl);
        }
        float gs[3], gd[3], e2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float diff = as.g[c] - ad.g[c];
            e2 += diff * diff;
            gs[c] = 2.0f * weight * cosv * diff;
            gd[c] = -gs[c];
        }
        acc += weight * cosv * e2;
        float xs[MlpGradAcc<NIN>::kSlices];
#pragma unroll
        for (int s = 0; s < MlpGradAcc<NIN>::kSlices; ++s) xs[s] = mlp_x_slice<NIN>(f7, s3, s, gl);
        wave_mlp_bwd<NIN>(W, xs, gl, as, gs, macc, g7);
#pragma unroll
        for (int s = 0; s < MlpGradAcc<NIN>::kSlices; ++s) xs[s] = mlp_x_slice<NIN>(f7, d3, s, gl);
        wave_mlp_bwd<NIN>(W, xs, gl, ad, gd, macc, g7);
        if (dF && live && gl < 7) {
            float v = g7[0];
#pragma unroll
            for (int c = 1; c < 7; ++c)
                if (gl == c) v = g7[c];
            unsafeAtomicAdd(dF + ray * 7 + gl, v);
        }
    }
    if (loss && gl == 0 && acc != 0.0f) unsafeAtomicAdd(loss, acc);
    if (gmlp) {
        mlp_grad_to_lds<NIN>(macc, lane, sW);
        __syncthreads();
        mlp_grad_flush<NIN>(sW, gmlp);
    }
}

hipError_t launch_smooth(const float* W, int mlp_in, const float* F, const float* d, int64_t n, const float* perturb,
                         int P, float weight, float* loss, float* dF, float* gmlp, hipStream_t s) {
    if (loss) hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, loss);
    if (n == 0) return hipGetLastError();
    const int64_t items = n * P;
    const int64_t max_blocks = 4096;
    int64_t nb = (items + kGroupsPerBlock - 1) / kGroupsPerBlock;
    if (nb > max_blocks) nb = max_blocks;
    int64_t chunk = (items + nb - 1) / nb;
    chunk = (chunk + kGroupsPerBlock - 1) / kGroupsPerBlock * kGroupsPerBlock;
    nb = (items + chunk - 1) / chunk;
    if (mlp_in == 34)
        hipLaunchKernelGGL(k_smooth<34>, dim3((unsigned)nb), dim3(kBlock), 0, s, W, F, d, items, chunk, perturb, P,
                           weight, loss, dF, gmlp);
    else
        hipLaunchKernelGGL(k_smooth<10>, dim3((unsigned)nb), dim3(kBlock), 0, s, W, F, d, items, chunk, perturb, P,
                           weight, loss, dF, gmlp);
    return hipGetLastError();
}

}  // namespace omerf
