// bwd_device.h -- device-side building blocks of the backward march: run
// detection, segmented sums and reverse scans over the lanes of a 16-lane
// group.
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

}  // namespace omerf
