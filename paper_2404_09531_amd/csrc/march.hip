// march.hip -- occupancy-plane ray marching kernels for gfx950.
//
// k_place      : sample placement only (k-lists), Sec. 4.1 Eq. 6-7 / Sec. 4.4
// k_march_fwd  : placement + feature gather (Eq. 2) + activations (Eq. 3) +
//                compositing (Eq. 1) -> F, T, counts per ray
// k_march_bwd  : deferred-MLP backward (Eq. 4) + replay of the samples with
//                recomputed features + scatter-add of feature gradients
//
// One ray per 16-lane group; see omerf_device.h for the decomposition.
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
// Forward march: writes F [n][7], T [n], n_placed [n], n_eval [n].
// Lane-pair shading: each queued batch of up to 16 samples is
// shaded as two halves of 8 samples; sample s of a half is owned by lanes
// 2s and 2s+1, which fetch the x-offset-0 and x-offset-1 corners (the two
// 32-byte halves of one contiguous 64-byte pair) and add their partial sums
// with a lane swap.  Each gather instruction then covers 32 samples with two
// adjacent corners per sample.  Transmittance comes from a 16-lane scan with
// the optical depth on the even lanes only.
// ---------------------------------------------------------------------------
// Group total of x (inclusive DPP scan; the row's last lane holds it) stored
// by that lane at dst, for the optional per-batch sums of w v.
__device__ __forceinline__ void store_group_total(float x, int gl, float* dst) {
    x = g_scan_incl(x, gl);
    if (gl == kGroup - 1) *dst = x;
}

template <class S, bool kBW, bool kSoft>
__global__ __launch_bounds__(kBlock) void k_march_fwd(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                           const float* __restrict__ d_, int64_t n,
                                                           float* __restrict__ F, float* __restrict__ T,
                                                           int32_t* __restrict__ n_placed,
                                                           int32_t* __restrict__ n_eval,
                                                           float* __restrict__ BW) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int half = gl & 1;
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
        bool stop = false;
        float bacc[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) bacc[c] = 0.0f;
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const int nsub = min(max(nb - sub * 8, 0), 8);  // samples in this half (group-uniform)
            if (nsub > 0 && !stop) {
                const int s = gl >> 1;
                const bool act = s < nsub;
                const int ks = __shfl(kq, sub * 8 + s, kGroup);
                float t[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) t[c] = 0.0f;
                float msoft = 0.0f;
                if (act) {
                    const float3 p = lattice_point(ks, o, d, rp.delta);
                    gather_half<S>(sc, corners_of(sc, p), half, t);
                    if (kSoft) msoft = occ_value(sc, p, rp.occ_inv_eps).m;
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) t[c] += pair_swap(t[c]);
                float a = 0.0f;
                float v[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) v[c] = 0.0f;
                if (act) {
                    a = __expf(t[0]) * rp.delta;
#pragma unroll
                    for (int c = 0; c < 7; ++c) v[c] = sigmoidf_fast(t[c + 1]);
                }
                const float ae = half ? 0.0f : a;             // depth on the even lane of each pair
                const float incl = g_scan_incl(ae, gl);         // lane 2s: sum_{j<=s} a_j
                const float excl_e = g_shift_up1(incl);         // even lanes: sum_{j<s} a_j (from lane 2s-1)
                const float excl = half ? pair_swap(excl_e) : excl_e;
                const float Ti = __expf(-(carry + excl));
                float w = Ti * (-expm1f(-a));
                int nb_eff = nsub;
                if (rp.t_term > 0.0f) {
                    const float Tnext = __expf(-(carry + incl));
                    const uint32_t m = g_ballot(act && !half && Tnext < rp.t_term, lane);
                    if (m) {
                        nb_eff = ((__ffs(m) - 1) >> 1) + 1;
                        stop = true;
                    }
                }
                if (kSoft) w *= msoft;              // Eq. 8: the weight, not T
                if (s >= nb_eff || half) w = 0.0f;  // accumulate once per sample (even lane)
#pragma unroll
                for (int c = 0; c < 7; ++c) bacc[c] += w * v[c];
                carry += __shfl(incl, 2 * (nb_eff - 1), kGroup);
                evals += nb_eff;
            }
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[c] += bacc[c];
        if (kBW) {
            float* dst = BW + ((size_t)ray * slots + batch) * 7;
#pragma unroll
            for (int c = 0; c < 7; ++c) store_group_total(bacc[c], gl, dst + c);
        }
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
    const uint32_t sy = (uint32_t)sc.Lx, sz = (uint32_t)sc.Lx * (uint32_t)sc.Ly;
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

template <bool kBW, bool kSoft>
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
                quad_gather(sc, corners_of(sc, p), h, ch, t);
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
// Scatter: per batch and per feature source, consecutive samples of a ray
// that share a cell (or texel) are summed onto the last lane of their run
// with DPP, so each corner gets one contribution per run; the run tails
// stage two row-adjacent corners (64 contiguous bytes) in LDS, and the group
// adds each staged pair to global memory with one atomic instruction whose
// 16 lanes cover those 64 bytes.  Device-memory float atomics are performed
// beyond L2, one request per 64-byte segment of an instruction, so
// contiguous lanes are ~16x cheaper than scattered ones.
// ---------------------------------------------------------------------------
constexpr int kBatchSlots = 1024 / kGroup / kGroup;  // registers holding batch totals (n_max <= 1024)

// Row-list scatter.  Per source, the samples sharing a cell form runs (see
// g_runs); for every pair of corners adjacent along the row axis (two
// contiguous 32-byte rows) each run's totals are summed onto its tail lane,
// the tails stage their 16 floats in LDS at their rank, and the group flushes
// one staged pair per instruction: 16 lanes x 4 B = 64 contiguous bytes.
struct Stage {
    float v[kGroup][16];
    int row[kGroup];
};

__device__ __forceinline__ void flush_pair(float* G, Stage& st, const Runs& rn, int rank, int nt, uint32_t row0,
                                           float w0, float w1, const float* gt, int lmax, int gl) {
    float4* q = reinterpret_cast<float4*>(st.v[rank]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // the two rows one after the other: fewer live registers
        const float w = h ? w1 : w0;
        float v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = w * gt[c];
        g_seg_sum8(v, rn.len, lmax);
        if (rn.tail) {
            q[2 * h] = make_float4(v[0], v[1], v[2], v[3]);
            q[2 * h + 1] = make_float4(v[4], v[5], v[6], v[7]);
        }
    }
    if (rn.tail) st.row[rank] = (int)row0;
    wave_order();
    for (int e = 0; e < nt; ++e) {
        const float val = st.v[e][gl];
        const uint32_t r = (uint32_t)st.row[e];
        if (val != 0.0f) unsafeAtomicAdd(G + (size_t)r * 8 + gl, val);
    }
    wave_order();
}

struct RunSet {
    Runs rn;
    int lmax, rank, nt;
};

__device__ __forceinline__ RunSet run_set(uint32_t key, bool act, int gl, int lane) {
    RunSet r;
    r.rn = g_runs(key, act, gl);
    r.lmax = g_max(act ? r.rn.len : 0);
    const uint32_t tm = g_ballot(r.rn.tail, lane);
    r.nt = __popc(tm);
    r.rank = __popc(tm & ((1u << gl) - 1u));
    return r;
}

__device__ __forceinline__ void scatter_plane_runs(float* gP, int na, Stage& st, bool act, uint32_t key, float fa,
                                                   float fb, const float* gt, int gl, int lane) {
    const RunSet rs = run_set(key, act, gl, lane);
    const float a0 = 1.0f - fa, a1 = fa;
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
        const float wb = p ? fb : 1.0f - fb;
        flush_pair(gP, st, rs.rn, rs.rank, rs.nt, key + (p ? (uint32_t)na : 0u), a0 * wb, a1 * wb, gt, rs.lmax, gl);
    }
}

__device__ __forceinline__ void scatter_batch_runs(const SceneDev& sc, float* gV, float* gxy, float* gxz, float* gyz,
                                                   Stage& st, bool act, const Corners& cn, const float* gt, int gl,
                                                   int lane) {
    {
        const RunSet rs = run_set(cn.g, act, gl, lane);
        const float x0w = 1.0f - cn.fx, x1w = cn.fx, y0w = 1.0f - cn.fy, y1w = cn.fy;
        const float z0w = 1.0f - cn.fz, z1w = cn.fz;
        const uint32_t sy = (uint32_t)sc.Lx, sz = (uint32_t)sc.Lx * (uint32_t)sc.Ly;
#pragma unroll 1
        for (int p = 0; p < 4; ++p) {
            const float yw = (p & 1) ? y1w : y0w, zw = (p >> 1) ? z1w : z0w;
            flush_pair(gV, st, rs.rn, rs.rank, rs.nt, cn.g + ((p & 1) ? sy : 0u) + ((p >> 1) ? sz : 0u),
                       x0w * yw * zw, x1w * yw * zw, gt, rs.lmax, gl);
        }
    }
    scatter_plane_runs(gxy, sc.Nx, st, act, cn.xy, cn.ux, cn.uy, gt, gl, lane);
    scatter_plane_runs(gxz, sc.Nx, st, act, cn.xz, cn.ux, cn.uz, gt, gl, lane);
    scatter_plane_runs(gyz, sc.Ny, st, act, cn.yz, cn.uy, cn.uz, gt, gl, lane);
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

template <class S, bool kSoft, int NIN>
__global__ __launch_bounds__(kBlock) void k_march_bwd(SceneDev sc, RayParams rp, const float* __restrict__ o_,
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
    for (int i = threadIdx.x; i < kMlpMaxSize; i += kBlock) sW[i] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int h = gl;
    Stage& stage = stages[gid];
    const float* W = sc.mlp;
    const int64_t start = (int64_t)xcd_block(blockIdx.x, gridDim.x) * chunk;
    const int64_t stop_r = min(n, start + chunk);
    for (int64_t ray = start + gid; ray < stop_r; ray += kGroupsPerBlock) {
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

template <bool kSoft>
static void launch_fwd_soft(const SceneDev& sc, bool bf16, const RayParams& rp, const float* o, const float* d,
                            int64_t n, float* F, float* T, int32_t* n_placed, int32_t* n_eval, float* batch_wv,
                            hipStream_t s) {
    const dim3 grid(blocks_for(n)), block(kBlock);
    if (bf16) {
        if (batch_wv)
            hipLaunchKernelGGL((k_march_fwd<BF16Store, true, kSoft>), grid, block, 0, s, sc, rp, o, d, n, F, T,
                               n_placed, n_eval, batch_wv);
        else
            hipLaunchKernelGGL((k_march_fwd<BF16Store, false, kSoft>), grid, block, 0, s, sc, rp, o, d, n, F, T,
                               n_placed, n_eval, batch_wv);
    } else {
        if (batch_wv)
            hipLaunchKernelGGL((k_march_fwd_f32q<true, kSoft>), grid, block, 0, s, sc, rp, o, d, n, F, T, n_placed,
                               n_eval, batch_wv);
        else
            hipLaunchKernelGGL((k_march_fwd_f32q<false, kSoft>), grid, block, 0, s, sc, rp, o, d, n, F, T, n_placed,
                               n_eval, batch_wv);
    }
}

hipError_t launch_march_fwd(const SceneDev& sc, bool bf16, const RayParams& rp, const float* o, const float* d,
                            int64_t n, float* F, float* T, int32_t* n_placed, int32_t* n_eval, float* batch_wv,
                            hipStream_t s) {
    // The per-batch sums and the soft occupancy are separate
    // specialisations, so the plain render path carries neither.
    if (rp.occ_inv_eps > 0.0f)
        launch_fwd_soft<true>(sc, bf16, rp, o, d, n, F, T, n_placed, n_eval, batch_wv, s);
    else
        launch_fwd_soft<false>(sc, bf16, rp, o, d, n, F, T, n_placed, n_eval, batch_wv, s);
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
