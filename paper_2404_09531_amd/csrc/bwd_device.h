// bwd_device.h -- device-side building blocks of the backward pass and of the
// group-cooperative deferred MLP (one hidden unit per lane of a 16-lane
// group): run detection and segmented sums over the lanes of a group, and
// the MLP forward/backward shared by the backward march and the
// view-smoothness loss.
#pragma once

#include "omerf_device.h"

namespace omerf {

// Runs of equal keys among the active lanes of a group, in lane order:
// `len` = lanes of the run before this one (this lane is the run's head when
// 0), `tail` = last active lane of its run.  Inactive lanes end runs.
struct Runs {
    int len;
    bool tail;
};
__device__ __forceinline__ Runs g_runs(uint32_t key, bool act, int gl) {
    const int a = act ? 1 : 0;
    const int prev_act = dpp_row_i<kRowShr | 1>(a), next_act = dpp_row_i<kRowShl | 1>(a);
    const uint32_t prev_key = (uint32_t)dpp_row_i<kRowShr | 1>((int)key);
    const uint32_t next_key = (uint32_t)dpp_row_i<kRowShl | 1>((int)key);
    int st = (!prev_act || prev_key != key) ? gl : 0;
    st = max(st, dpp_row_i<kRowShr | 1>(st));
    st = max(st, dpp_row_i<kRowShr | 2>(st));
    st = max(st, dpp_row_i<kRowShr | 4>(st));
    st = max(st, dpp_row_i<kRowShr | 8>(st));
    return Runs{gl - st, act && (!next_act || next_key != key)};
}

// Inclusive sums over the lane's run (see g_runs) of 8 values: the run's
// tail lane gets the run totals.  `lmax` is the group's largest `len`; only
// the scan steps that some run needs are executed.
__device__ __forceinline__ void g_seg_sum8(float* x, int len, int lmax) {
    if (lmax >= 1) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float y = dpp_row<kRowShr | 1>(x[c]);
            x[c] = len >= 1 ? x[c] + y : x[c];
        }
    }
    if (lmax >= 2) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float y = dpp_row<kRowShr | 2>(x[c]);
            x[c] = len >= 2 ? x[c] + y : x[c];
        }
    }
    if (lmax >= 4) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float y = dpp_row<kRowShr | 4>(x[c]);
            x[c] = len >= 4 ? x[c] + y : x[c];
        }
    }
    if (lmax >= 8) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float y = dpp_row<kRowShr | 8>(x[c]);
            x[c] = len >= 8 ? x[c] + y : x[c];
        }
    }
}

// g_seg_sum8 for the first 2 of the values.
__device__ __forceinline__ void g_seg_sum2(float* x, int len, int lmax) {
#pragma unroll
    for (int st = 1; st < kGroup; st <<= 1) {
        if (lmax >= st) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float y = st == 1 ? dpp_row<kRowShr | 1>(x[c])
                                : st == 2 ? dpp_row<kRowShr | 2>(x[c])
                                : st == 4 ? dpp_row<kRowShr | 4>(x[c]) : dpp_row<kRowShr | 8>(x[c]);
                x[c] = len >= st ? x[c] + y : x[c];
            }
        }
    }
}

// Inclusive scan towards lower lanes: lane i gets x_i + ... + x_15.
__device__ __forceinline__ float g_rscan_incl(float x, int /*gl*/) {
    x += dpp_row<kRowShl | 1>(x);
    x += dpp_row<kRowShl | 2>(x);
    x += dpp_row<kRowShl | 4>(x);
    x += dpp_row<kRowShl | 8>(x);
    return x;
}

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

// Backward of group_mlp_fwd for dL/dG = dG (the same on every lane): adds
// the parameter gradients into the LDS array sW (distinct addresses per
// lane) and dL/dx[0..6] into dx7 (the same on every lane).
template <int NIN>
__device__ __forceinline__ void group_mlp_bwd(const float* W, const float* x, int h, const MlpAct& a,
                                              const float* dG, float* sW, float* dx7) {
    using L = MlpLayout<NIN>;
    float dz3[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) dz3[r] = dG[r] * a.g[r] * (1.0f - a.g[r]);
    const float dh2 = W[L::W3 + h] * dz3[0] + W[L::W3 + 16 + h] * dz3[1] + W[L::W3 + 32 + h] * dz3[2];
    const float dz2 = a.z2 > 0.0f ? dh2 : 0.0f;
    float dh1 = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        dh1 += W[L::W2 + j * 16 + h] * __shfl(dz2, j, kGroup);
        atomicAdd(&sW[L::W2 + h * 16 + j], dz2 * __shfl(a.h1, j, kGroup));
    }
    const float dz1 = a.z1 > 0.0f ? dh1 : 0.0f;
#pragma unroll
    for (int c = 0; c < 7; ++c) dx7[c] += g_sum(W[L::W1 + h * NIN + c] * dz1);
#pragma unroll
    for (int c = 0; c < NIN; ++c) atomicAdd(&sW[L::W1 + h * NIN + c], dz1 * x[c]);
    atomicAdd(&sW[L::B1 + h], dz1);
    atomicAdd(&sW[L::B2 + h], dz2);
#pragma unroll
    for (int r = 0; r < 3; ++r) atomicAdd(&sW[L::W3 + r * 16 + h], dz3[r] * a.h2);
    if (h < 3) atomicAdd(&sW[L::B3 + h], h == 0 ? dz3[0] : h == 1 ? dz3[1] : dz3[2]);
}

}  // namespace omerf
