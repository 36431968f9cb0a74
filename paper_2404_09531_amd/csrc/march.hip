// march.hip -- occupancy-plane ray marching kernels for gfx950.
//
// k_place      : sample placement only (k-lists), Sec. 4.1 Eq. 6-7 / Sec. 4.4
// k_march_fwd_f32q / k_march_fwd_lane : placement + feature gather (Eq. 2)
//                + activations (Eq. 3) + compositing (Eq. 1) -> F, T, counts
//                per ray (float32 lane quads; bfloat16 and 8-bit one lane
//                per sample)
// k_march_bwd  : deferred-MLP backward (Eq. 4) + replay of the samples with
//                recomputed features + scatter-add of feature gradients
//
// One ray per 16-lane group; see omerf_device.h for the decomposition.
#include "../../include/omerf.h"
#include "omerf_device.h"
#include "omerf_launch.h"

namespace omerf {

// Candidate driver shared by the three kernels.  Walks the conservative
// lattice range of one ray 16 candidates at a time, appends accepted k to
// the group's LDS queue in increasing order and hands full batches (or the
// final partial batch) to `shade(k, nb)`, which returns true to stop.
template <class Shade>
__device__ __forceinline__ int march_candidates(const SceneDev& sc, const RayParams& rp, float3 o,
                                                float3 d, int* q, int gl, int lane, Shade&& shade) {
    const KRange kr = candidate_range(sc, o, d, rp.delta);
    int k = kr.lo;
    int n_acc = 0;
    int qn = 0;
    bool more = (k <= kr.hi) && rp.n_max > 0;
    while (true) {
        if (more) {
            const int kk = k + gl;
            bool ok = false;
            if (kk <= kr.hi) ok = accept_point(sc, lattice_point(kk, o, d, rp.delta));
            const uint32_t m = g_ballot(ok, lane);
            const int room = rp.n_max - n_acc;
            const int rank = __popc(m & ((1u << gl) - 1u));
            if (ok && rank < room) q[qn + rank] = kk;
            const int cnt = min(__popc(m), room);
            qn += cnt;
            n_acc += cnt;
            k += kGroup;
            more = (k <= kr.hi) && (n_acc < rp.n_max);
            wave_order();
            // An empty window: jump over the segments whose columns cannot
            // hold a sample.  16 lanes test 16 consecutive segments of
            // 16 << lv candidates against pyramid level lv; after two sweeps
            // in a row with no possible sample the level coarsens (when a
            // pyramid is attached), the first possible segment is refined
            // one level at a time, and candidate testing resumes at level 0.
            int lv = 0, empty_sweeps = 0;
            while (more && m == 0u) {
                const int seg = kGroup << lv;
                const bool maybe = column_maybe(sc, o, d, rp.delta, k + gl * seg, seg, lv);
                const uint32_t mm = g_ballot(maybe, lane);
                if (mm) {
                    k += seg * (__ffs(mm) - 1);
                    more = k <= kr.hi;
                    if (lv == 0) break;
                    --lv;
                    empty_sweeps = 0;
                } else {
                    k += kGroup * seg;
                    more = k <= kr.hi;
                    if (++empty_sweeps >= 2 && lv < sc.mip_levels) {
                        ++lv;
                        empty_sweeps = 0;
                    }
                }
            }
        }
        if (qn >= kGroup || (!more && qn > 0)) {
            const int nb = min(qn, kGroup);
            const int kq = gl < nb ? q[gl] : 0;
            const int rest = qn - nb;
            const int tail = gl < rest ? q[kGroup + gl] : 0;
            wave_order();
            if (gl < rest) q[gl] = tail;
            wave_order();
            qn = rest;
            if (shade(kq, nb)) break;
        }
        if (!more && qn == 0) break;
    }
    return n_acc;
}

__device__ __forceinline__ float3 load3(const float* p, int64_t r) {
    return make_float3(p[r * 3 + 0], p[r * 3 + 1], p[r * 3 + 2]);
}

// ---------------------------------------------------------------------------
// Placement only.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_place(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                  const float* __restrict__ d_, int64_t n,
                                                  int32_t* __restrict__ k_out, int32_t* __restrict__ n_placed) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int64_t ray = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kGroupsPerBlock + gid;
    if (ray >= n) return;
    const float3 o = load3(o_, ray), d = load3(d_, ray);
    int32_t* kr = k_out + ray * rp.n_max;
    int written = 0;
    const int cnt = march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
        if (gl < nb) kr[written + gl] = kq;
        written += nb;
        return false;
    });
    for (int i = cnt + gl; i < rp.n_max; i += kGroup) kr[i] = -1;
    if (gl == 0) n_placed[ray] = cnt;
}

// ---------------------------------------------------------------------------
// Forward marches: write F [n][7], T [n], n_placed [n], n_eval [n] (and, with
// kBW, the per-batch sums of w v).
// ---------------------------------------------------------------------------
// Group total of x (inclusive DPP scan; the row's last lane holds it) stored
// by that lane at dst, for the optional per-batch sums of w v.
__device__ __forceinline__ void store_group_total(float x, int gl, float* dst) {
    x = g_scan_incl(x, gl);
    if (gl == kGroup - 1) *dst = x;
}

// ---------------------------------------------------------------------------
// Forward march with one lane per sample, for 8-bit and bfloat16 features.
// A corner pair is 16 (8-bit) or 32 (bfloat16) contiguous bytes, so lane s
// of the group shades sample s of the batch on its own (10 or 20 loads),
// and the batch of 16 samples is composited with one 16-lane scan.
// ---------------------------------------------------------------------------
struct GatherU8 {
    static __device__ __forceinline__ void run(const SceneDev& sc, const Corners& c, float* t) { gather_u8(sc, c, t); }
};
struct GatherBF16 {
    static __device__ __forceinline__ void run(const SceneDev& sc, const Corners& c, float* t) {
        gather_features_split<BF16Store>(sc, c, t);
    }
};

template <class Gather, bool kBW, bool kSoft, bool kSparse>
__global__ __launch_bounds__(kBlock) void k_march_fwd_lane(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                           const float* __restrict__ d_, int64_t n,
                                                           float* __restrict__ F, float* __restrict__ T,
                                                           int32_t* __restrict__ n_placed,
                                                           int32_t* __restrict__ n_eval, float* __restrict__ BW) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int64_t ray = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kGroupsPerBlock + gid;
    if (ray >= n) return;
    const float3 o = load3(o_, ray), d = load3(d_, ray);
    float acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = 0.0f;
    float carry = 0.0f;
    int evals = 0, batch = 0;
    const int slots = (rp.n_max + kGroup - 1) / kGroup;
    const int placed = march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
        const bool act = gl < nb;
        float t[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) t[c] = 0.0f;
        float msoft = 0.0f;
        if (act) {
            const float3 p = lattice_point(kq, o, d, rp.delta);
            Gather::run(sc, corners_of<kSparse>(sc, p), t);
            if (kSoft) msoft = occ_value(sc, p, rp.occ_inv_eps).m;
        }
        float a = 0.0f;
        float v[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = 0.0f;
        if (act) {
            a = __expf(t[0]) * rp.delta;
#pragma unroll
            for (int c = 0; c < 7; ++c) v[c] = sigmoidf_fast(t[c + 1]);
        }
        const float incl = g_scan_incl(a, gl);
        const float excl = g_shift_up1(incl);
        float w = __expf(-(carry + excl)) * (-expm1f(-a));
        int nb_eff = nb;
        bool stop = false;
        if (rp.t_term > 0.0f) {
            const float Tnext = __expf(-(carry + incl));
            const uint32_t m = g_ballot(act && Tnext < rp.t_term, lane);
            if (m) {
                nb_eff = __ffs(m);
                stop = true;
            }
        }
        if (kSoft) w *= msoft;  // Eq. 8: the weight, not T
        if (gl >= nb_eff) w = 0.0f;
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[c] += w * v[c];
        if (kBW) {
            float* dst = BW + ((size_t)ray * slots + batch) * 7;
#pragma unroll
            for (int c = 0; c < 7; ++c) store_group_total(w * v[c], gl, dst + c);
        }
        carry += __shfl(incl, nb_eff - 1, kGroup);
        evals += nb_eff;
        ++batch;
        return stop;
    });
    float f[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) f[c] = g_sum(acc[c]);
    if (gl == 0) {
#pragma unroll
        for (int c = 0; c < 7; ++c) F[ray * 7 + c] = f[c];
        T[ray] = __expf(-carry);
        n_placed[ray] = placed;
        n_eval[ray] = evals;
    }
}

// ---------------------------------------------------------------------------
// Forward march for float32 features, lane-quad shading.  A queued batch of
// up to 16 samples is shaded in four quarters; in quarter j, lanes
// 4s..4s+3 of the group shade sample 4j + s, lane 4s+q taking x-offset
// (q & 1) and channel half (q >> 1).  A float32 corner pair is 64
// contiguous bytes, so each gather instruction reads one 64-byte span for
// each of 4 consecutive samples of the ray; consecutive samples often share
// a grid cell or plane texel, and lanes of one instruction that hit the same
// cache line cost one lookup.  After the x-offset sum, lanes with c = 0 hold
// channels 0..3 (density, diffuse colour) and lanes with c = 1 channels
// 4..7, so the activations split evenly over the quad.  The four quarters
// are gathered before the batch is composited, so their loads overlap.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void quad_gather(const SceneDev& sc, const Corners& c, int h, int ch, float* t) {
    const uint32_t sy = sc.gsy, sz = sc.gsz;
    const uint32_t nx = (uint32_t)sc.Nx, ny = (uint32_t)sc.Ny;
    const uint32_t hh = (uint32_t)h;
    const float4* G = reinterpret_cast<const float4*>(sc.grid) + ch;
    const float4* XY = reinterpret_cast<const float4*>(sc.pxy) + ch;
    const float4* XZ = reinterpret_cast<const float4*>(sc.pxz) + ch;
    const float4* YZ = reinterpret_cast<const float4*>(sc.pyz) + ch;
    float4 r[10];
    r[0] = G[(size_t)(c.g + hh) * 2];
    r[1] = G[(size_t)(c.g + sy + hh) * 2];
    r[2] = G[(size_t)(c.g + sz + hh) * 2];
    r[3] = G[(size_t)(c.g + sz + sy + hh) * 2];
    r[4] = XY[(size_t)(c.xy + hh) * 2];
    r[5] = XY[(size_t)(c.xy + nx + hh) * 2];
    r[6] = XZ[(size_t)(c.xz + hh) * 2];
    r[7] = XZ[(size_t)(c.xz + nx + hh) * 2];
    r[8] = YZ[(size_t)(c.yz + hh) * 2];
    r[9] = YZ[(size_t)(c.yz + ny + hh) * 2];
    const float wx = h ? c.fx : 1.0f - c.fx;
    const float y0 = 1.0f - c.fy, y1 = c.fy, z0 = 1.0f - c.fz, z1 = c.fz;
    const float wa = h ? c.ux : 1.0f - c.ux;  // x for XY / XZ
    const float wb = h ? c.uy : 1.0f - c.uy;  // y for YZ
    const float b0 = 1.0f - c.uy, b1 = c.uy, e0 = 1.0f - c.uz, e1 = c.uz;
    const float w[10] = {wx * y0 * z0, wx * y1 * z0, wx * y0 * z1, wx * y1 * z1, wa * b0,
                         wa * b1,      wa * e0,      wa * e1,      wb * e0,      wb * e1};
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        t[0] += w[j] * r[j].x;
        t[1] += w[j] * r[j].y;
        t[2] += w[j] * r[j].z;
        t[3] += w[j] * r[j].w;
    }
}

template <bool kBW, bool kSoft, bool kSparse>
__global__ __launch_bounds__(kBlock) void k_march_fwd_f32q(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                           const float* __restrict__ d_, int64_t n,
                                                           float* __restrict__ F, float* __restrict__ T,
                                                           int32_t* __restrict__ n_placed,
                                                           int32_t* __restrict__ n_eval,
                                                           float* __restrict__ BW) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int h = gl & 1, ch = (gl >> 1) & 1;
    const int s = gl >> 2;            // sample of the quad within a quarter
    const bool lead = (gl & 3) == 0;  // lane 4s: the quad's depth owner
    const int64_t ray = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kGroupsPerBlock + gid;
    if (ray >= n) return;
    const float3 o = load3(o_, ray), d = load3(d_, ray);
    float acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = 0.0f;
    float carry = 0.0f;
    int evals = 0, batch = 0;
    const int slots = (rp.n_max + kGroup - 1) / kGroup;
    const int placed = march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
        float a[4], v[4][4], msoft[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * j + s;
            const int ks = __shfl(kq, i, kGroup);
            float t[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            msoft[j] = 0.0f;
            if (i < nb) {
                const float3 p = lattice_point(ks, o, d, rp.delta);
                quad_gather(sc, corners_of<kSparse>(sc, p), h, ch, t);
                if (kSoft) msoft[j] = occ_value(sc, p, rp.occ_inv_eps).m;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) t[c] += pair_swap(t[c]);
            a[j] = 0.0f;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[j][c] = 0.0f;
            if (i < nb) {
                if (ch == 0) {
                    a[j] = __expf(t[0]) * rp.delta;
#pragma unroll
                    for (int c = 0; c < 3; ++c) v[j][c] = sigmoidf_fast(t[c + 1]);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) v[j][c] = sigmoidf_fast(t[c]);
                }
            }
            a[j] = quad_bcast0(a[j]);
        }
        // Optical depth in front of sample 4j + s: carry + all samples of
        // quarters < j + samples of quads < s in quarter j.
        float incl[4], pre[4];
        float run = carry;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            incl[j] = g_scan_incl(lead ? a[j] : 0.0f, gl);
            pre[j] = run + quad_bcast0(g_shift_up1(incl[j]));
            run += __shfl(incl[j], kGroup - 1, kGroup);
        }
        int nb_eff = nb;
        bool stop = false;
        if (rp.t_term > 0.0f) {
            int first = kGroup;
#pragma unroll
            for (int j = 3; j >= 0; --j)
                if (4 * j + s < nb && __expf(-(pre[j] + a[j])) < rp.t_term) first = 4 * j + s;
            first = g_min(first);
            if (first < nb) {
                nb_eff = first + 1;
                stop = true;
            }
        }
        float bacc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float w = __expf(-pre[j]) * (-expm1f(-a[j]));
            if (kSoft) w *= msoft[j];                // Eq. 8: the weight, not T
            if (4 * j + s >= nb_eff || h) w = 0.0f;  // once per sample and channel half
#pragma unroll
            for (int c = 0; c < 4; ++c) bacc[c] += w * v[j][c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += bacc[c];
        if (kBW) {
            float* dst = BW + ((size_t)ray * slots + batch) * 7;
#pragma unroll
            for (int c = 0; c < 3; ++c) store_group_total(ch == 0 ? bacc[c] : 0.0f, gl, dst + c);
#pragma unroll
            for (int c = 0; c < 4; ++c) store_group_total(ch == 1 ? bacc[c] : 0.0f, gl, dst + 3 + c);
        }
        ++batch;
        // depth through the last evaluated sample, from the quad that owns it
        const int jl = (nb_eff - 1) >> 2;
        const float mine = (jl == 0 ? pre[0] + a[0] : jl == 1 ? pre[1] + a[1] : jl == 2 ? pre[2] + a[2] : pre[3] + a[3]);
        carry = __shfl(mine, 4 * ((nb_eff - 1) & 3), kGroup);
        evals += nb_eff;
        return stop;
    });
    float f[7];
#pragma unroll
    for (int c = 0; c < 3; ++c) f[c] = g_sum(ch == 0 ? acc[c] : 0.0f);
#pragma unroll
    for (int c = 0; c < 4; ++c) f[3 + c] = g_sum(ch == 1 ? acc[c] : 0.0f);
    if (gl == 0) {
#pragma unroll
        for (int c = 0; c < 7; ++c) F[ray * 7 + c] = f[c];
        T[ray] = __expf(-carry);
        n_placed[ray] = placed;
        n_eval[ray] = evals;
    }
}

// ---------------------------------------------------------------------------
// Backward.  Per ray: the deferred MLP backward runs across the 16 lanes of
// the group (lane h owns hidden unit h of both hidden layers), giving
// g7 = dL/dF (+ dL/dC on the diffuse part).  The samples are then replayed
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

// Longest chunk of rays a backward block sorts by length (LDS: 6 KB).
constexpr int kSortMax = 1024;

template <class S, bool kSoft, int NIN>
__global__ __launch_bounds__(kBlock, NIN == 10 ? 4 : 1) void k_march_bwd(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                      const float* __restrict__ d_, int64_t n, int64_t chunk,
                                                      const float* __restrict__ Fs, const float* __restrict__ Ts,
                                                      const int32_t* __restrict__ n_eval,
                                                      const float* __restrict__ BW,
                                                      const float* __restrict__ dC,
                                                      const float* __restrict__ dF, float* __restrict__ gV,
                                                      float* __restrict__ gxy, float* __restrict__ gxz,
                                                      float* __restrict__ gyz, float* __restrict__ gmlp,
                                                      float* __restrict__ gocc) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    __shared__ float sW[kMlpMaxSize];
    __shared__ __attribute__((aligned(16))) Stage stages[kGroupsPerBlock];
    __shared__ int s_key[kSortMax];
    __shared__ uint16_t s_ord[kSortMax];
    for (int i = threadIdx.x; i < kMlpMaxSize; i += kBlock) sW[i] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int h = gl;
    Stage& stage = stages[gid];
    const float* W = sc.mlp;
    const int64_t start = (int64_t)xcd_block(blockIdx.x, gridDim.x) * chunk;
    const int cnt = (int)(min(n, start + chunk) - start);
    // A wave's four groups walk their rays in step, so a wave waits for its
    // longest ray.  The chunk is therefore walked longest-first (a stable
    // rank sort of n_eval in LDS), which hands each wave rays of similar
    // length; chunks longer than kSortMax keep their order.
    const bool by_len = cnt <= kSortMax;
    if (by_len) {
        for (int i = threadIdx.x; i < cnt; i += kBlock) s_key[i] = n_eval[start + i];
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += kBlock) {
            const int ki = s_key[i];
            int r = 0;
            for (int j = 0; j < cnt; ++j) {
                const int kj = s_key[j];
                r += (kj > ki) || (kj == ki && j < i);
            }
            s_ord[r] = (uint16_t)i;
        }
        __syncthreads();
    }
    for (int it = gid; it < cnt; it += kGroupsPerBlock) {
        const int64_t ray = start + (by_len ? (int)s_ord[it] : it);
        const float3 o = load3(o_, ray), d = load3(d_, ray);
        const int ne = n_eval[ray];
        const float Tn = Ts[ray];
        const float dc0 = dC[ray * 3 + 0], dc1 = dC[ray * 3 + 1], dc2 = dC[ray * 3 + 2];
        if (ne <= 0) continue;  // no sample: C = c_bg, no parameter gradient
        // g7 = dL/dF: the diffuse part of dL/dC, the deferred MLP G (Eq. 4)
        // backward (hidden unit h per lane) and an optional dL/dF from
        // losses on F itself.
        float g7[7];
        {
            float x[NIN];
            mlp_input<NIN>(Fs + ray * 7, d, x);
            const MlpAct act = group_mlp_fwd<NIN>(W, x, h);
            const float dG[3] = {dc0, dc1, dc2};
            g7[0] = dc0;
            g7[1] = dc1;
            g7[2] = dc2;
            g7[3] = g7[4] = g7[5] = g7[6] = 0.0f;
            group_mlp_bwd<NIN>(W, x, h, act, dG, sW, g7);
            if (dF) {
#pragma unroll
                for (int c = 0; c < 7; ++c) g7[c] += dF[ray * 7 + c];
            }
        }
        const float gT = dc0 * rp.bg0 + dc1 * rp.bg1 + dc2 * rp.bg2;

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
    }
    __syncthreads();
    for (int i = threadIdx.x; i < MlpLayout<NIN>::SIZE; i += kBlock) {
        const float v = sW[i];
        if (v != 0.0f) unsafeAtomicAdd(gmlp + i, v);
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kGroupsPerBlock - 1) / kGroupsPerBlock); }

hipError_t launch_place(const SceneDev& sc, const RayParams& rp, const float* o, const float* d, int64_t n,
                        int32_t* k_out, int32_t* n_placed, hipStream_t s) {
    hipLaunchKernelGGL(k_place, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, rp, o, d, n, k_out, n_placed);
    return hipGetLastError();
}

template <bool kSoft, bool kSparse>
static void launch_fwd_soft(const SceneDev& sc, int dtype, const RayParams& rp, const float* o, const float* d,
                            int64_t n, float* F, float* T, int32_t* n_placed, int32_t* n_eval, float* batch_wv,
                            hipStream_t s) {
    const dim3 grid(blocks_for(n)), block(kBlock);
    if (dtype == OM_U8) {  // render only: no per-batch sums
        hipLaunchKernelGGL((k_march_fwd_lane<GatherU8, false, kSoft, kSparse>), grid, block, 0, s, sc, rp, o, d, n, F,
                           T, n_placed, n_eval, nullptr);
    } else if (dtype == OM_BF16) {
        if (batch_wv)
            hipLaunchKernelGGL((k_march_fwd_lane<GatherBF16, true, kSoft, kSparse>), grid, block, 0, s, sc, rp, o, d,
                               n, F, T, n_placed, n_eval, batch_wv);
        else
            hipLaunchKernelGGL((k_march_fwd_lane<GatherBF16, false, kSoft, kSparse>), grid, block, 0, s, sc, rp, o, d,
                               n, F, T, n_placed, n_eval, batch_wv);
    } else {
        if (batch_wv)
            hipLaunchKernelGGL((k_march_fwd_f32q<true, kSoft, kSparse>), grid, block, 0, s, sc, rp, o, d, n, F, T,
                               n_placed, n_eval, batch_wv);
        else
            hipLaunchKernelGGL((k_march_fwd_f32q<false, kSoft, kSparse>), grid, block, 0, s, sc, rp, o, d, n, F, T,
                               n_placed, n_eval, batch_wv);
    }
}

hipError_t launch_march_fwd(const SceneDev& sc, int dtype, const RayParams& rp, const float* o, const float* d,
                            int64_t n, float* F, float* T, int32_t* n_placed, int32_t* n_eval, float* batch_wv,
                            hipStream_t s) {
    // The per-batch sums and the soft occupancy are separate
    // specialisations, so the plain render path carries neither.
    // Sparse blocks are render only (the API refuses per-batch sums for them).
    const bool soft = rp.occ_inv_eps > 0.0f;
    if (sc.blk_shift > 0) {
        if (soft)
            launch_fwd_soft<true, true>(sc, dtype, rp, o, d, n, F, T, n_placed, n_eval, nullptr, s);
        else
            launch_fwd_soft<false, true>(sc, dtype, rp, o, d, n, F, T, n_placed, n_eval, nullptr, s);
    } else if (soft) {
        launch_fwd_soft<true, false>(sc, dtype, rp, o, d, n, F, T, n_placed, n_eval, batch_wv, s);
    } else {
        launch_fwd_soft<false, false>(sc, dtype, rp, o, d, n, F, T, n_placed, n_eval, batch_wv, s);
    }
    return hipGetLastError();
}

template <class S, bool kSoft>
static void launch_bwd_nin(const SceneDev& sc, const RayParams& rp, const float* o, const float* d, int64_t n,
                           int64_t chunk, dim3 grid, const float* F, const float* T, const int32_t* n_eval,
                           const float* batch_wv, const float* dC, const float* dF, float* gV, float* gxy, float* gxz,
                           float* gyz, float* gmlp, float* gocc, hipStream_t s) {
    if (sc.mlp_in == 34)
        hipLaunchKernelGGL((k_march_bwd<S, kSoft, 34>), grid, dim3(kBlock), 0, s, sc, rp, o, d, n, chunk, F, T, n_eval,
                           batch_wv, dC, dF, gV, gxy, gxz, gyz, gmlp, gocc);
    else
        hipLaunchKernelGGL((k_march_bwd<S, kSoft, 10>), grid, dim3(kBlock), 0, s, sc, rp, o, d, n, chunk, F, T, n_eval,
                           batch_wv, dC, dF, gV, gxy, gxz, gyz, gmlp, gocc);
}

hipError_t launch_march_bwd(const SceneDev& sc, bool bf16, const RayParams& rp, const float* o, const float* d,
                            int64_t n, const float* F, const float* T, const int32_t* n_eval, const float* batch_wv,
                            const float* dC, const float* dF, float* gV, float* gxy, float* gxz, float* gyz,
                            float* gmlp, float* gocc, hipStream_t s) {
    // Persistent blocks, each owning a contiguous chunk of rays, so the MLP
    // weight gradients are reduced in LDS over many rays before one set of
    // global atomics per block.
    const int64_t max_blocks = 4096;
    int64_t nb = (n + kGroupsPerBlock - 1) / kGroupsPerBlock;
    if (nb > max_blocks) nb = max_blocks;
    int64_t chunk = (n + nb - 1) / nb;
    chunk = (chunk + kGroupsPerBlock - 1) / kGroupsPerBlock * kGroupsPerBlock;
    nb = (n + chunk - 1) / chunk;
    const dim3 grid((unsigned)nb);
    const bool soft = rp.occ_inv_eps > 0.0f;
    if (bf16) {
        if (soft)
            launch_bwd_nin<BF16Store, true>(sc, rp, o, d, n, chunk, grid, F, T, n_eval, batch_wv, dC, dF, gV, gxy, gxz,
                                            gyz, gmlp, gocc, s);
        else
            launch_bwd_nin<BF16Store, false>(sc, rp, o, d, n, chunk, grid, F, T, n_eval, batch_wv, dC, dF, gV, gxy, gxz,
                                             gyz, gmlp, gocc, s);
    } else {
        if (soft)
            launch_bwd_nin<F32Store, true>(sc, rp, o, d, n, chunk, grid, F, T, n_eval, batch_wv, dC, dF, gV, gxy, gxz,
                                           gyz, gmlp, gocc, s);
        else
            launch_bwd_nin<F32Store, false>(sc, rp, o, d, n, chunk, grid, F, T, n_eval, batch_wv, dC, dF, gV, gxy, gxz,
                                            gyz, gmlp, gocc, s);
    }
    return hipGetLastError();
}

}  // namespace omerf
