// march_fwd.hip -- occupancy-plane ray marching kernels for gfx950 (forward).
//
// k_place      : sample placement only (k-lists), Sec. 4.1 Eq. 6-7 / Sec. 4.4
// k_march_fwd_f32q / k_march_fwd_lane : placement + feature gather (Eq. 2)
//                + activations (Eq. 3) + compositing (Eq. 1) -> F, T, counts
//                per ray (float32 lane quads; bfloat16 and 8-bit one lane
//                per sample)
//
// One ray per 16-lane group; see omerf_device.h for the decomposition.
#include "../../include/omerf.h"
#include "omerf_device.h"
#include "omerf_launch.h"

#include <type_traits>

namespace omerf {

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
// Rows read by a render: for every evaluated sample (the first n_eval placed
// samples of the ray, or all placed samples without n_eval), a byte 1 is
// stored at each of its 8 grid vertices and 12 plane texels (Eq. 2).
// Plain byte stores: marking is idempotent, so no atomics are needed.
// ---------------------------------------------------------------------------
template <bool kSparse>
__global__ __launch_bounds__(kBlock) void k_mark(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                 const float* __restrict__ d_, int64_t n,
                                                 const int32_t* __restrict__ n_eval, uint8_t* __restrict__ fg,
                                                 uint8_t* __restrict__ fxy, uint8_t* __restrict__ fxz,
                                                 uint8_t* __restrict__ fyz) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int64_t ray = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kGroupsPerBlock + gid;
    if (ray >= n) return;
    const float3 o = load3(o_, ray), d = load3(d_, ray);
    const int ne = n_eval ? n_eval[ray] : rp.n_max;
    if (ne <= 0) return;
    int done = 0;
    march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
        const int nbe = min(nb, ne - done);
        if (gl < nbe) {
            const Corners c = corners_of<kSparse>(sc, lattice_point(kq, o, d, rp.delta));
            const uint32_t nx = (uint32_t)sc.Nx, ny = (uint32_t)sc.Ny;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t b = c.g + ((q & 1) ? sc.gsy : 0u) + ((q >> 1) ? sc.gsz : 0u);
                fg[b] = 1;
                fg[b + 1] = 1;
            }
            fxy[c.xy] = 1;
            fxy[c.xy + 1] = 1;
            fxy[c.xy + nx] = 1;
            fxy[c.xy + nx + 1] = 1;
            fxz[c.xz] = 1;
            fxz[c.xz + 1] = 1;
            fxz[c.xz + nx] = 1;
            fxz[c.xz + nx + 1] = 1;
            fyz[c.yz] = 1;
            fyz[c.yz + 1] = 1;
            fyz[c.yz + ny] = 1;
            fyz[c.yz + ny + 1] = 1;
        }
        done += nbe;
        return done >= ne;
    });
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

// Waves per SIMD the one-lane-per-sample forwards are compiled for: the
// bfloat16 gather without the soft occupancy fits 6 (<= 80 VGPRs) without
// spilling; the other forms keep the compiler's choice.
template <class Gather, bool kSoft>
constexpr int lane_min_waves() { return std::is_same<Gather, GatherBF16>::value && !kSoft ? 6 : 1; }

template <class Gather, bool kBW, bool kSoft, bool kSparse>
__global__ __launch_bounds__(kBlock, (lane_min_waves<Gather, kSoft>())) void k_march_fwd_lane(
    SceneDev sc, RayParams rp, const float* __restrict__ o_, const float* __restrict__ d_, int64_t n,
    float* __restrict__ F, float* __restrict__ T, int32_t* __restrict__ n_placed, int32_t* __restrict__ n_eval,
    float* __restrict__ BW) {
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

// Sparse voxel blocks, in two steps (corners_of<true> does both): the
// atlas block of a sample's grid cell, clamped as there, and the flat
// index of the cell's base vertex inside that block.
__device__ __forceinline__ uint32_t sparse_block(const SceneDev& sc, const Corners& c) {
    const int32_t id = sc.blk_idx[((c.iz >> sc.blk_shift) * sc.bny + (c.iy >> sc.blk_shift)) * sc.bnx +
                                  (c.ix >> sc.blk_shift)];
    return min((uint32_t)id, sc.n_blocks);
}
__device__ __forceinline__ uint32_t sparse_vertex(const SceneDev& sc, const Corners& c, uint32_t b) {
    const int m = (1 << sc.blk_shift) - 1;
    return b * sc.blk_verts + ((uint32_t)(c.iz & m) * sc.gsy + (uint32_t)(c.iy & m)) * sc.gsy + (uint32_t)(c.ix & m);
}

// Waves per SIMD the float32 forward is compiled for: the soft-occupancy
// and sparse forms at 4 (<= 128 VGPRs, no spill); the others keep the
// compiler's choice, which is 4 already.
template <bool kSoft, bool kSparse>
constexpr int f32q_min_waves() { return kSoft || kSparse ? 4 : 1; }

template <bool kBW, bool kSoft, bool kSparse>
__global__ __launch_bounds__(kBlock, (f32q_min_waves<kSoft, kSparse>())) void k_march_fwd_f32q(SceneDev sc, RayParams rp, const float* __restrict__ o_,
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
        // Sparse blocks: lane gl looks up the block of sample gl, so the
        // batch's 16 index loads are in flight together, not one per
        // quarter ahead of that quarter's corner loads.
        uint32_t blk = 0u;
        if (kSparse && gl < nb) blk = sparse_block(sc, corners_of<false>(sc, lattice_point(kq, o, d, rp.delta)));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * j + s;
            const int ks = __shfl(kq, i, kGroup);
            const uint32_t bj = kSparse ? (uint32_t)__shfl((int)blk, i, kGroup) : 0u;
            float t[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            msoft[j] = 0.0f;
            if (i < nb) {
                const float3 p = lattice_point(ks, o, d, rp.delta);
                Corners c = corners_of<false>(sc, p);
                if (kSparse) c.g = sparse_vertex(sc, c, bj);
                quad_gather(sc, c, h, ch, t);
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
        if (kSoft) {
            // The soft mask (Eq. 6, 8) once the quarters are gathered: its
            // occupancy loads and arithmetic then do not add to the
            // gather's registers, which keeps the kernel at 4 waves.
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * j + s;
                const int ks = __shfl(kq, i, kGroup);
                if (i < nb) msoft[j] = occ_value(sc, lattice_point(ks, o, d, rp.delta), rp.occ_inv_eps).m;
            }
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
// Launchers.
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kGroupsPerBlock - 1) / kGroupsPerBlock); }

hipError_t launch_place(const SceneDev& sc, const RayParams& rp, const float* o, const float* d, int64_t n,
                        int32_t* k_out, int32_t* n_placed, hipStream_t s) {
    hipLaunchKernelGGL(k_place, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, rp, o, d, n, k_out, n_placed);
    return hipGetLastError();
}

hipError_t launch_mark(const SceneDev& sc, const RayParams& rp, const float* o, const float* d, int64_t n,
                       const int32_t* n_eval, uint8_t* fg, uint8_t* fxy, uint8_t* fxz, uint8_t* fyz, hipStream_t s) {
    if (sc.blk_shift > 0)
        hipLaunchKernelGGL(k_mark<true>, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, rp, o, d, n, n_eval, fg, fxy,
                           fxz, fyz);
    else
        hipLaunchKernelGGL(k_mark<false>, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, rp, o, d, n, n_eval, fg, fxy,
                           fxz, fyz);
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

}  // namespace omerf
