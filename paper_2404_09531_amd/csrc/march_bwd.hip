// march_bwd.hip -- backward of the occupancy-plane ray march for gfx950:
// replay of the samples with recomputed features + scatter-add of the
// feature gradients (derivative of Eq. 1-3), given dL/dF from the deferred
// MLP's backward (k_mlp_bwd, Eq. 4).
//
// One ray per 16-lane group; see omerf_device.h for the decomposition.
#include "../../include/omerf.h"
#include "bwd_device.h"
#include "omerf_launch.h"

namespace omerf {

// ---------------------------------------------------------------------------
// Backward.  Per ray, g7 = dL/dF (dL/dC on the diffuse part + the deferred
// MLP's backward + losses on F) and dL/dC . c_bg come precomputed from
// k_mlp_bwd, so the march holds no MLP state.  The samples are replayed
// twice in the forward's order with recomputed features:
//
//   pass 1 records, per 16-sample batch, B_b = sum_{i in b} w_i (g7 . v_i);
//   pass 2 forms for each sample the suffix S_i = sum_{k > i} w_k (g7 . v_k)
//   from an in-batch reverse scan plus the totals of the later batches, and
//
//   dL/da_i = T_{i+1} (g7 . v_i) - S_i - T_n (dL/dC . c_bg),
//
// derived from Eq. 1 with w_k = T_k - T_{k+1}; then dL/dt0 = dL/da delta tau
// and dL/dt_c = w g7_c v_c (1 - v_c) through the sigmoids of Eq. 3.  The
// suffix is summed from its own terms (never as a total minus a prefix), so
// samples behind opaque surfaces keep their relative accuracy.
//
// Scatter: per batch and per feature source, the contributions of the
// batch's samples to each vertex are summed with DPP over the run of
// samples that share it, and the group adds them to global memory one
// 64-byte segment (two row-adjacent vertices) per atomic instruction, each
// segment once per batch (see scatter_row_class).  Device-memory float
// atomics are performed beyond L2, one request per 64-byte segment an
// instruction touches, so the request count is what the scatter minimises.
// ---------------------------------------------------------------------------
constexpr int kBatchSlots = 1024 / kGroup / kGroup;  // registers holding batch totals (n_max <= 1024)

// Segment scatter.  Device-memory float atomics cost one request per
// 64-byte segment an instruction touches, and a float32 vertex is 32 bytes,
// so the unit of work is the segment {2s, 2s+1} of a row: one instruction
// whose 16 lanes add both vertices' 8 channels.  Per batch and feature
// source, the rows a sample touches are split into classes by the parities
// of their row coordinates (4 classes for the grid, 2 for a plane): each
// sample has exactly one row in each class, and a vertex stays in the same
// class, as the even-x (E) or odd-x (O) vertex of the sample's corner pair,
// for every sample whose cell it bounds.  The samples bounding a vertex are
// consecutive along the ray (the union of the cells around a vertex is
// convex), so per class the samples with equal E (or O) vertex form one run
// of lanes; its tail gets the vertex total from a segmented sum.  A lane
// whose cell has even x holds the E and O vertices of one segment, which
// pairs its E run with its O run: each paired segment is flushed once with
// both halves, an unpaired vertex with one half.
struct Stage {
    float v[kGroup][16];    // one segment per record: E vertex (0..7), O vertex (8..15)
    uint32_t base[kGroup];  // flat index of the segment's first vertex
};

// Lanes [t - len, t] of a group as a bit mask.
__device__ __forceinline__ uint32_t run_mask(int t, int len) {
    return ((2u << t) - 1u) & ~((1u << (t - len)) - 1u);
}

// Stages a segment whose lower vertex has no contribution.
__device__ __forceinline__ void stage_upper(Stage& st, int rank, uint32_t base, const float* v) {
    float4* q4 = reinterpret_cast<float4*>(st.v[rank]);
    q4[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    q4[1] = q4[0];
    q4[2] = make_float4(v[0], v[1], v[2], v[3]);
    q4[3] = make_float4(v[4], v[5], v[6], v[7]);
    st.base[rank] = base;
}

// Adds the first n staged segments to G, one 64-byte atomic instruction each.
__device__ __forceinline__ void flush_segments(float* G, const Stage& st, int n, int gl) {
    for (int i = 0; i < n; ++i) {
        const float val = st.v[i][gl];
        const uint32_t base = st.base[i];
        if (val != 0.0f) unsafeAtomicAdd(G + (size_t)base * 8 + gl, val);
    }
}

// One row class of one source.  Per lane: the flat index of the first
// vertex of its row in this class, the cell's index x along the row (the
// corners are x and x + 1), the row's weight wr and the fraction fx along
// the row; gt = dL/dt of the sample.  The E runs are staged at their rank,
// each with its paired O run's totals (or zeros) in the upper half, and
// followed by the unpaired O runs (lower half zero), and flushed together
// (in two rounds if they exceed the 16 records).
__device__ __forceinline__ void scatter_row_class(float* G, Stage& st, bool act, uint32_t rowbase, int x, float wr,
                                                  float fx, const float* gt, int gl, int lane) {
    const bool xodd = (x & 1) != 0;
    const uint32_t ve = rowbase + (uint32_t)(xodd ? x + 1 : x);
    const uint32_t vo = rowbase + (uint32_t)(xodd ? x : x + 1);
    const float we = wr * (xodd ? fx : 1.0f - fx);
    const float wo = wr * (xodd ? 1.0f - fx : fx);
    const Runs re = g_runs(ve, act, gl), ro = g_runs(vo, act, gl);
    const uint32_t tme = g_ballot(re.tail, lane);
    const uint32_t evm = g_ballot(act && !xodd, lane);  // lanes holding both vertices of one segment
    float4* q4 = nullptr;
    {
        float v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = we * gt[c];
        g_seg_sum8(v, re.len, g_max(act ? re.len : 0));
        if (re.tail) {
            const int rank = __popc(tme & ((1u << gl) - 1u));
            q4 = reinterpret_cast<float4*>(st.v[rank]);
            q4[0] = make_float4(v[0], v[1], v[2], v[3]);
            q4[1] = make_float4(v[4], v[5], v[6], v[7]);
            if (!(evm & run_mask(gl, re.len))) {  // no O run to pair with
                q4[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                q4[3] = q4[2];
            }
            st.base[rank] = ve;
        }
    }
    const int lmo = g_max(act ? ro.len : 0);
    bool unpaired = false;
    {
        float v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = wo * gt[c];
        g_seg_sum8(v, ro.len, lmo);
        if (ro.tail) {
            const uint32_t ev = evm & run_mask(gl, ro.len);
            if (ev) {  // paired with the E run through its first even-x lane f
                const int f = __ffs(ev) - 1;
                const int et = f + __ffs(tme >> f) - 1;
                q4 = reinterpret_cast<float4*>(st.v[__popc(tme & ((1u << et) - 1u))]);
                q4[2] = make_float4(v[0], v[1], v[2], v[3]);
                q4[3] = make_float4(v[4], v[5], v[6], v[7]);
            } else {
                unpaired = true;
            }
        }
        const uint32_t um = g_ballot(unpaired, lane);
        const int ne = __popc(tme), nu = __popc(um);
        const int urank = __popc(um & ((1u << gl) - 1u));
        if (ne + nu <= kGroup) {  // usual case: one flush for both kinds
            if (unpaired) stage_upper(st, ne + urank, vo - 1u, v);
            wave_order();
            flush_segments(G, st, ne + nu, gl);
            wave_order();
            return;
        }
        wave_order();
        flush_segments(G, st, ne, gl);
        wave_order();
        if (unpaired) stage_upper(st, urank, vo - 1u, v);
        wave_order();
        flush_segments(G, st, nu, gl);
        wave_order();
    }
}

// The row of class q (parity bit q) among rows i and i + 1, and its weight
// (1 - f for row i, f for row i + 1).
__device__ __forceinline__ int class_row(int i, int q, float f, float& w) {
    const int d = (i ^ q) & 1;
    w = d ? f : 1.0f - f;
    return i + d;
}

__device__ __forceinline__ void scatter_batch_runs(const SceneDev& sc, float* gV, float* gxy, float* gxz, float* gyz,
                                                   Stage& st, bool act, const Corners& cn, const float* gt, int gl,
                                                   int lane) {
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        float wy, wz;
        const int y = class_row(cn.iy, q & 1, cn.fy, wy), z = class_row(cn.iz, q >> 1, cn.fz, wz);
        const uint32_t rowbase = ((uint32_t)z * (uint32_t)sc.Ly + (uint32_t)y) * (uint32_t)sc.Lx;
        scatter_row_class(gV, st, act, rowbase, cn.ix, wy * wz, cn.fx, gt, gl, lane);
    }
#pragma unroll 1
    for (int q = 0; q < 2; ++q) {
        float w;
        int r = class_row(cn.jy, q, cn.uy, w);
        scatter_row_class(gxy, st, act, (uint32_t)r * (uint32_t)sc.Nx, cn.jx, w, cn.ux, gt, gl, lane);
        r = class_row(cn.jz, q, cn.uz, w);
        scatter_row_class(gxz, st, act, (uint32_t)r * (uint32_t)sc.Nx, cn.jx, w, cn.ux, gt, gl, lane);
        scatter_row_class(gyz, st, act, (uint32_t)r * (uint32_t)sc.Ny, cn.jy, w, cn.uy, gt, gl, lane);
    }
}

// One replayed sample: optical depth, density, activated colours/features
// and, for the soft occupancy, its value and derivatives.
template <class S, bool kSoft>
__device__ __forceinline__ void replay_sample(const SceneDev& sc, const RayParams& rp, float3 o, float3 d, int kq,
                                              bool act, float& a, float& tau, float* v, Corners& cn, OccValue& oc) {
    a = 0.0f;
    tau = 0.0f;
    cn = Corners{};  // defined keys and weights on inactive lanes, which the group scans read
    oc = OccValue{1.0f, 0.0f, 0.0f, -1};
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = 0.0f;
    if (act) {
        const float3 p = lattice_point(kq, o, d, rp.delta);
        cn = corners_of(sc, p);
        if (kSoft) oc = occ_value(sc, p, rp.occ_inv_eps);
        float t[8];
        gather_features_split<S>(sc, cn, t);
        tau = __expf(t[0]);
        a = tau * rp.delta;
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = sigmoidf_fast(t[c + 1]);
    }
}

// z_min / z_max gradient of the soft occupancy: run sums over the samples
// that share an occupancy cell, one pair of atomics per run.
__device__ __forceinline__ void scatter_occ(float* gocc, bool act, const OccValue& oc, float gm, int gl, int lane) {
    float g[8] = {gm * oc.dzmin, gm * oc.dzmax, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const Runs rn = g_runs((uint32_t)oc.cell, act, gl);
    const int lmax = g_max(act ? rn.len : 0);
    g_seg_sum2(g, rn.len, lmax);
    if (rn.tail) {
        if (g[0] != 0.0f) unsafeAtomicAdd(gocc + (size_t)oc.cell * 2, g[0]);
        if (g[1] != 0.0f) unsafeAtomicAdd(gocc + (size_t)oc.cell * 2 + 1, g[1]);
    }
}

// ---------------------------------------------------------------------------
// Ray order of the backward: longest first, handed out on demand.
//
// A wave's four groups walk their rays in step, so a wave waits for its
// longest ray, and the kernel waits for its slowest wave.  The rays are
// therefore counting-sorted by their number of 16-sample batches,
// descending (k_order_*), and each wave takes the next four rays of that
// order from a counter whenever it is free: a wave's rays have the same
// batch count, and the short rays at the end even out the finish.
//
// Scheduling words in the workspace (int32): bins [0, 65), cursors
// [65, 130), the hand-out counter at kOrderCounter.
// ---------------------------------------------------------------------------
constexpr int kOrderBins = OM_MAX_SAMPLES / kGroup + 1;  // batch counts 0 .. n_max / 16
constexpr int kOrderCursor = kOrderBins;
constexpr int kOrderCounter = 2 * kOrderBins;
static_assert(kOrderCounter < kBwdSchedWords, "scheduling words");

__device__ __forceinline__ int batch_bin(int ne, int nbins) {
    return ne <= 0 ? 0 : min((ne + kGroup - 1) / kGroup, nbins - 1);
}

__global__ __launch_bounds__(64) void k_order_clear(int* __restrict__ hdr) {
    for (int i = threadIdx.x; i < kBwdSchedWords; i += 64) hdr[i] = 0;
}

// Rays per batch count: a histogram per block in LDS, added to the bins.
__global__ __launch_bounds__(256) void k_order_hist(const int32_t* __restrict__ n_eval, int64_t n, int64_t chunk,
                                                    int nbins, int* __restrict__ hdr) {
    __shared__ int cnt[kOrderBins];
    for (int i = threadIdx.x; i < nbins; i += 256) cnt[i] = 0;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * chunk, e = min(n, s + chunk);
    for (int64_t r = s + threadIdx.x; r < e; r += 256) atomicAdd(&cnt[batch_bin(n_eval[r], nbins)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += 256)
        if (cnt[i]) atomicAdd(&hdr[i], cnt[i]);
}

// Start of each batch count's range in the order, longest first.
__global__ __launch_bounds__(64) void k_order_scan(int nbins, int* __restrict__ hdr) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = nbins - 1; b >= 0; --b) {
            hdr[kOrderCursor + b] = acc;
            acc += hdr[b];
        }
    }
}

// Each block reserves a range per batch count for its rays (one global
// atomic per count), then places them there (order within a count is
// arbitrary).
__global__ __launch_bounds__(256) void k_order_scatter(const int32_t* __restrict__ n_eval, int64_t n, int64_t chunk,
                                                       int nbins, int* __restrict__ hdr, int32_t* __restrict__ order) {
    __shared__ int cnt[kOrderBins], base[kOrderBins];
    for (int i = threadIdx.x; i < nbins; i += 256) cnt[i] = 0;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * chunk, e = min(n, s + chunk);
    for (int64_t r = s + threadIdx.x; r < e; r += 256) atomicAdd(&cnt[batch_bin(n_eval[r], nbins)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += 256) {
        base[i] = cnt[i] ? atomicAdd(&hdr[kOrderCursor + i], cnt[i]) : 0;
        cnt[i] = 0;
    }
    __syncthreads();
    for (int64_t r = s + threadIdx.x; r < e; r += 256) {
        const int bb = batch_bin(n_eval[r], nbins);
        order[base[bb] + atomicAdd(&cnt[bb], 1)] = (int32_t)r;
    }
}

template <class S, bool kSoft>
__global__ __launch_bounds__(kBlock, 4) void k_march_bwd(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                       const float* __restrict__ d_, int64_t n,
                                                       const int32_t* __restrict__ order, unsigned int* __restrict__ next_ray,
                                                       const float* __restrict__ Ts,
                                                       const int32_t* __restrict__ n_eval,
                                                       const float* __restrict__ BW, const float* __restrict__ G8,
                                                       float* __restrict__ gV, float* __restrict__ gxy,
                                                       float* __restrict__ gxz, float* __restrict__ gyz,
                                                       float* __restrict__ gocc) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    __shared__ __attribute__((aligned(16))) Stage stages[kGroupsPerBlock];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    Stage& stage = stages[gid];
    auto ray_body = [&](int64_t ray) {
        const float3 o = load3(o_, ray), d = load3(d_, ray);
        const int ne = n_eval[ray];
        const float Tn = Ts[ray];
        if (ne <= 0) return;  // no sample: C = c_bg, no parameter gradient
        const float4 ga = *reinterpret_cast<const float4*>(G8 + ray * 8);
        const float4 gb = *reinterpret_cast<const float4*>(G8 + ray * 8 + 4);
        const float g7[7] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z};
        const float gT = gb.w;

        // Pass 1: per-batch totals of w (g7 . v); batch b lives in lane b % 16
        // of register slot b / 16.
        float btot[kBatchSlots];
#pragma unroll
        for (int s = 0; s < kBatchSlots; ++s) btot[s] = 0.0f;
        if (BW) {
            // The forward's per-batch sums of w v: B_b = g7 . sum_{i in b} w_i v_i.
            const int slots = (rp.n_max + kGroup - 1) / kGroup, nbat = (ne + kGroup - 1) / kGroup;
#pragma unroll 1
            for (int s = 0; s < (nbat + kGroup - 1) / kGroup; ++s) {
                const int b = s * kGroup + gl;
                float t = 0.0f;
                if (b < nbat) {
                    const float* src = BW + ((size_t)ray * slots + b) * 7;
#pragma unroll
                    for (int c = 0; c < 7; ++c) t += g7[c] * src[c];
                }
#pragma unroll
                for (int k = 0; k < kBatchSlots; ++k)
                    if (s == k) btot[k] = t;
            }
        } else {
            float carry = 0.0f;
            int done = 0, b = 0;
            march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
                const int nb_eff = min(nb, ne - done);
                const bool act = gl < nb_eff;
                float a, tau, v[7];
                Corners cn;
                OccValue oc;
                replay_sample<S, kSoft>(sc, rp, o, d, kq, act, a, tau, v, cn, oc);
                const float incl = g_scan_incl(a, gl);
                const float excl = g_shift_up1(incl);
                const float w = act ? __expf(-(carry + excl)) * (-expm1f(-a)) * (kSoft ? oc.m : 1.0f) : 0.0f;
                float gv = 0.0f;
#pragma unroll
                for (int c = 0; c < 7; ++c) gv += g7[c] * v[c];
                const float tot = g_sum(w * gv);
#pragma unroll
                for (int s = 0; s < kBatchSlots; ++s)
                    if ((b >> 4) == s && gl == (b & 15)) btot[s] = tot;
                carry += __shfl(incl, kGroup - 1, kGroup);
                done += nb_eff;
                ++b;
                return done >= ne;
            });
        }
        // R[s] at lane l = sum of the totals of batches >= 16 s + l.
        float R[kBatchSlots];
        {
            float above = 0.0f;
#pragma unroll
            for (int s = kBatchSlots - 1; s >= 0; --s) {
                const float r = g_rscan_incl(btot[s], gl);
                R[s] = r + above;
                above += __shfl(r, 0, kGroup);
            }
        }

        // Pass 2: gradients and scatter.
        float carry = 0.0f;
        int done = 0, b = 0;
        march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
            const int nb_eff = min(nb, ne - done);
            const bool act = gl < nb_eff;
            float a, tau, v[7];
            Corners cn;
            OccValue oc;
            replay_sample<S, kSoft>(sc, rp, o, d, kq, act, a, tau, v, cn, oc);
            const float incl = g_scan_incl(a, gl);
            const float excl = g_shift_up1(incl);
            const float Ti = __expf(-(carry + excl));
            const float Tnext = __expf(-(carry + incl));
            const float w0 = act ? Ti * (-expm1f(-a)) : 0.0f;  // Eq. 1 weight
            const float msoft = kSoft ? oc.m : 1.0f;             // Eq. 8 scales the weight, not T
            const float w = w0 * msoft;
            float gv = 0.0f;
#pragma unroll
            for (int c = 0; c < 7; ++c) gv += g7[c] * v[c];
            const float cterm = w * gv;
            const float rin = g_shift_down1(g_rscan_incl(cterm, gl));  // terms of later lanes
            const int nxt = b + 1;
            float after = 0.0f;
#pragma unroll
            for (int s = 0; s < kBatchSlots; ++s)
                if ((nxt >> 4) == s) after = __shfl(R[s], nxt & 15, kGroup);
            const float suffix = rin + after;
            float gt[8];
            gt[0] = (Tnext * msoft * gv - suffix - Tn * gT) * rp.delta * tau;
#pragma unroll
            for (int c = 0; c < 7; ++c) gt[c + 1] = w * g7[c] * v[c] * (1.0f - v[c]);
            scatter_batch_runs(sc, gV, gxy, gxz, gyz, stage, act, cn, gt, gl, lane);
            if (kSoft && gocc) scatter_occ(gocc, act, oc, w0 * gv, gl, lane);  // dL/dM = w0 (g7 . v)
            carry += __shfl(incl, kGroup - 1, kGroup);
            done += nb_eff;
            ++b;
            return done >= ne;
        });
    };
    // Four rays per wave and turn, the next turn's requested ahead.  The
    // counter is unsigned: it ends below n + 8 x 4 per wave < 2^32.
    unsigned int first = 0u;
    if (lane == 0) first = atomicAdd(next_ray, 4u);
    int64_t base = (int64_t)(unsigned int)__shfl((int)first, 0);
    while (base < n) {
        unsigned int ahead = 0u;
        if (lane == 0) ahead = atomicAdd(next_ray, 4u);
        const int64_t idx = base + (gid & 3);
        if (idx < n) ray_body(order[idx]);
        base = (int64_t)(unsigned int)__shfl((int)ahead, 0);
    }
}

hipError_t launch_march_bwd(const SceneDev& sc, bool bf16, const RayParams& rp, const float* o, const float* d,
                            int64_t n, const float* T, const int32_t* n_eval, const float* batch_wv, const float* G8,
                            int32_t* order, int* sched, float* gV, float* gxy, float* gxz, float* gyz, float* gocc,
                            hipStream_t s) {
    // Longest-first order (counting sort by batch count), then persistent
    // blocks whose waves take rays from it on demand.  2048 blocks of 4 waves
    // cover every wave slot of the device (4 per SIMD); blocks beyond the
    // slots start when the order is handed out and leave at once.
    const int nbins = (rp.n_max + kGroup - 1) / kGroup + 1;
    const int64_t sort_blocks = min((n + 4095) / 4096, (int64_t)1024);
    const int64_t sort_chunk = (n + sort_blocks - 1) / sort_blocks;
    hipLaunchKernelGGL(k_order_clear, dim3(1), dim3(64), 0, s, sched);
    hipLaunchKernelGGL(k_order_hist, dim3((unsigned)sort_blocks), dim3(256), 0, s, n_eval, n, sort_chunk, nbins, sched);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, nbins, sched);
    hipLaunchKernelGGL(k_order_scatter, dim3((unsigned)sort_blocks), dim3(256), 0, s, n_eval, n, sort_chunk, nbins,
                       sched, order);
    unsigned int* next_ray = reinterpret_cast<unsigned int*>(sched + kOrderCounter);
    const dim3 grid((unsigned)min((n + kGroupsPerBlock - 1) / kGroupsPerBlock, (int64_t)2048)), block(kBlock);
    const bool soft = rp.occ_inv_eps > 0.0f;
    if (bf16) {
        if (soft)
            hipLaunchKernelGGL((k_march_bwd<BF16Store, true>), grid, block, 0, s, sc, rp, o, d, n, order, next_ray, T,
                               n_eval, batch_wv, G8, gV, gxy, gxz, gyz, gocc);
        else
            hipLaunchKernelGGL((k_march_bwd<BF16Store, false>), grid, block, 0, s, sc, rp, o, d, n, order, next_ray, T,
                               n_eval, batch_wv, G8, gV, gxy, gxz, gyz, gocc);
    } else {
        if (soft)
            hipLaunchKernelGGL((k_march_bwd<F32Store, true>), grid, block, 0, s, sc, rp, o, d, n, order, next_ray, T,
                               n_eval, batch_wv, G8, gV, gxy, gxz, gyz, gocc);
        else
            hipLaunchKernelGGL((k_march_bwd<F32Store, false>), grid, block, 0, s, sc, rp, o, d, n, order, next_ray, T,
                               n_eval, batch_wv, G8, gV, gxy, gxz, gyz, gocc);
    }
    return hipGetLastError();
}

}  // namespace omerf
