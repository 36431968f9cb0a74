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
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(kBlock) void k_march_fwd(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                      const float* __restrict__ d_, int64_t n,
                                                      float* __restrict__ F, float* __restrict__ T,
                                                      int32_t* __restrict__ n_placed, int32_t* __restrict__ n_eval) {
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
    float carry = 0.0f;  // optical depth of all samples before the batch
    int evals = 0;
    const int placed = march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
        float a = 0.0f;
        float v[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = 0.0f;
        if (gl < nb) {
            const float3 p = lattice_point(kq, o, d, rp.delta);
            const Corners cn = corners_of(sc, p);
            float t[8];
            gather_features<S>(sc, cn, t);
            a = __expf(t[0]) * rp.delta;
#pragma unroll
            for (int c = 0; c < 7; ++c) v[c] = sigmoidf_fast(t[c + 1]);
        }
        const float incl = g_scan_incl(a, gl);
        float excl = __shfl_up(incl, 1, kGroup);
        if (gl == 0) excl = 0.0f;
        const float Ti = __expf(-(carry + excl));
        float w = Ti * (-expm1f(-a));
        int nb_eff = nb;
        bool stop = false;
        if (rp.t_term > 0.0f) {
            const float Tnext = __expf(-(carry + incl));
            const uint32_t m = g_ballot(gl < nb && Tnext < rp.t_term, lane);
            if (m) {
                nb_eff = __ffs(m);  // index of first terminating lane + 1
                stop = true;
            }
        }
        if (gl >= nb_eff) w = 0.0f;
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[c] += w * v[c];
        carry += __shfl(incl, nb_eff - 1, kGroup);
        evals += nb_eff;
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
// Backward.  Per ray: the deferred MLP backward runs across the 16 lanes of
// the group (lane h owns hidden unit h of both hidden layers), giving
// g7 = dL/dF (+ dL/dC on the diffuse part); then the samples are replayed in
// the forward's order and each lane scatters the gradient of its sample's
// 8 feature channels into the 8 grid and 12 plane corners.
//
// dL/da_i = T_{i+1} (g7 . v_i) - (g7 . F - S_i) - T_n (dL/dC . c_bg),
// S_i = sum_{k<=i} w_k (g7 . v_k), derived from Eq. 1 with
// w_k = T_k - T_{k+1}; then dL/dt0 = dL/da * delta * tau and
// dL/dt_c = w g7_c v_c (1 - v_c) through the sigmoids of Eq. 3.
// ---------------------------------------------------------------------------
struct F32Scatter {
    static __device__ __forceinline__ void add(float* base, uint32_t idx, float w, const float* g) {
        float* q = base + (size_t)idx * 8;
#pragma unroll
        for (int c = 0; c < 8; ++c) unsafeAtomicAdd(q + c, w * g[c]);
    }
};

template <class S>
__global__ __launch_bounds__(kBlock) void k_march_bwd(SceneDev sc, RayParams rp, const float* __restrict__ o_,
                                                      const float* __restrict__ d_, int64_t n, int64_t chunk,
                                                      const float* __restrict__ Fs, const float* __restrict__ Ts,
                                                      const int32_t* __restrict__ n_eval,
                                                      const float* __restrict__ dC, float* __restrict__ gV,
                                                      float* __restrict__ gxy, float* __restrict__ gxz,
                                                      float* __restrict__ gyz, float* __restrict__ gmlp) {
    __shared__ int qs[kGroupsPerBlock][kQueue];
    __shared__ float sW[512];
    for (int i = threadIdx.x; i < 512; i += kBlock) sW[i] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kGroup - 1);
    const int gid = threadIdx.x / kGroup;
    const int h = gl;
    const float* W = sc.mlp;
    const int64_t start = (int64_t)xcd_block(blockIdx.x, gridDim.x) * chunk;
    const int64_t stop_r = min(n, start + chunk);
    for (int64_t ray = start + gid; ray < stop_r; ray += kGroupsPerBlock) {
        const float3 o = load3(o_, ray), d = load3(d_, ray);
        const int ne = n_eval[ray];
        float x[10];
#pragma unroll
        for (int c = 0; c < 7; ++c) x[c] = Fs[ray * 7 + c];
        x[7] = d.x;
        x[8] = d.y;
        x[9] = d.z;
        const float Tn = Ts[ray];
        const float dc0 = dC[ray * 3 + 0], dc1 = dC[ray * 3 + 1], dc2 = dC[ray * 3 + 2];
        float g7[7];
        g7[0] = dc0;
        g7[1] = dc1;
        g7[2] = dc2;
        g7[3] = g7[4] = g7[5] = g7[6] = 0.0f;
        if (ne > 0) {
            // Forward of G for hidden unit h (Eq. 4).
            float z1 = W[kB1 + h];
#pragma unroll
            for (int c = 0; c < 10; ++c) z1 += W[kW1 + h * 10 + c] * x[c];
            const float h1 = fmaxf(z1, 0.0f);
            float z2 = W[kB2 + h];
#pragma unroll
            for (int j = 0; j < 16; ++j) z2 += W[kW2 + h * 16 + j] * __shfl(h1, j, kGroup);
            const float h2 = fmaxf(z2, 0.0f);
            float dz3[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const float z3 = W[kB3 + r] + g_sum(W[kW3 + r * 16 + h] * h2);
                const float g = sigmoidf_fast(z3);
                dz3[r] = (r == 0 ? dc0 : r == 1 ? dc1 : dc2) * g * (1.0f - g);
            }
            const float dh2 = W[kW3 + h] * dz3[0] + W[kW3 + 16 + h] * dz3[1] + W[kW3 + 32 + h] * dz3[2];
            const float dz2 = z2 > 0.0f ? dh2 : 0.0f;
            float dh1 = 0.0f;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const float dz2j = __shfl(dz2, j, kGroup);
                dh1 += W[kW2 + j * 16 + h] * dz2j;
                atomicAdd(&sW[kW2 + h * 16 + j], dz2 * __shfl(h1, j, kGroup));
            }
            const float dz1 = z1 > 0.0f ? dh1 : 0.0f;
#pragma unroll
            for (int c = 0; c < 7; ++c) g7[c] += g_sum(W[kW1 + h * 10 + c] * dz1);
#pragma unroll
            for (int c = 0; c < 10; ++c) atomicAdd(&sW[kW1 + h * 10 + c], dz1 * x[c]);
            atomicAdd(&sW[kB1 + h], dz1);
            atomicAdd(&sW[kB2 + h], dz2);
#pragma unroll
            for (int r = 0; r < 3; ++r) atomicAdd(&sW[kW3 + r * 16 + h], dz3[r] * h2);
            if (h < 3) atomicAdd(&sW[kB3 + h], h == 0 ? dz3[0] : h == 1 ? dz3[1] : dz3[2]);
        }
        const float gT = dc0 * rp.bg0 + dc1 * rp.bg1 + dc2 * rp.bg2;
        float gF = 0.0f;
#pragma unroll
        for (int c = 0; c < 7; ++c) gF += g7[c] * x[c];
        float carry = 0.0f, carryS = 0.0f;
        int done = 0;
        if (ne > 0) {
            march_candidates(sc, rp, o, d, qs[gid], gl, lane, [&](int kq, int nb) {
                const int nb_eff = min(nb, ne - done);
                const bool act = gl < nb_eff;
                float a = 0.0f, tau = 0.0f, v[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) v[c] = 0.0f;
                Corners cn;
                if (act) {
                    const float3 p = lattice_point(kq, o, d, rp.delta);
                    cn = corners_of(sc, p);
                    float t[8];
                    gather_features<S>(sc, cn, t);
                    tau = __expf(t[0]);
                    a = tau * rp.delta;
#pragma unroll
                    for (int c = 0; c < 7; ++c) v[c] = sigmoidf_fast(t[c + 1]);
                }
                const float incl = g_scan_incl(a, gl);
                float excl = __shfl_up(incl, 1, kGroup);
                if (gl == 0) excl = 0.0f;
                const float Ti = __expf(-(carry + excl));
                const float Tnext = __expf(-(carry + incl));
                const float w = act ? Ti * (-expm1f(-a)) : 0.0f;
                float gv = 0.0f;
#pragma unroll
                for (int c = 0; c < 7; ++c) gv += g7[c] * v[c];
                const float sincl = carryS + g_scan_incl(w * gv, gl);
                if (act) {
                    const float dLda = Tnext * gv - (gF - sincl) - Tn * gT;
                    float gt[8];
                    gt[0] = dLda * rp.delta * tau;
#pragma unroll
                    for (int c = 0; c < 7; ++c) gt[c + 1] = w * g7[c] * v[c] * (1.0f - v[c]);
                    const uint32_t sy = (uint32_t)sc.Lx, sz = (uint32_t)sc.Lx * (uint32_t)sc.Ly;
                    const float x0 = 1.0f - cn.fx, x1 = cn.fx, y0 = 1.0f - cn.fy, y1 = cn.fy;
                    const float z0 = 1.0f - cn.fz, z1 = cn.fz;
                    F32Scatter::add(gV, cn.g, x0 * y0 * z0, gt);
                    F32Scatter::add(gV, cn.g + 1, x1 * y0 * z0, gt);
                    F32Scatter::add(gV, cn.g + sy, x0 * y1 * z0, gt);
                    F32Scatter::add(gV, cn.g + sy + 1, x1 * y1 * z0, gt);
                    F32Scatter::add(gV, cn.g + sz, x0 * y0 * z1, gt);
                    F32Scatter::add(gV, cn.g + sz + 1, x1 * y0 * z1, gt);
                    F32Scatter::add(gV, cn.g + sz + sy, x0 * y1 * z1, gt);
                    F32Scatter::add(gV, cn.g + sz + sy + 1, x1 * y1 * z1, gt);
                    const float a0 = 1.0f - cn.ux, a1 = cn.ux, b0 = 1.0f - cn.uy, b1 = cn.uy;
                    const float e0 = 1.0f - cn.uz, e1 = cn.uz;
                    const uint32_t nx = (uint32_t)sc.Nx, ny = (uint32_t)sc.Ny;
                    F32Scatter::add(gxy, cn.xy, a0 * b0, gt);
                    F32Scatter::add(gxy, cn.xy + 1, a1 * b0, gt);
                    F32Scatter::add(gxy, cn.xy + nx, a0 * b1, gt);
                    F32Scatter::add(gxy, cn.xy + nx + 1, a1 * b1, gt);
                    F32Scatter::add(gxz, cn.xz, a0 * e0, gt);
                    F32Scatter::add(gxz, cn.xz + 1, a1 * e0, gt);
                    F32Scatter::add(gxz, cn.xz + nx, a0 * e1, gt);
                    F32Scatter::add(gxz, cn.xz + nx + 1, a1 * e1, gt);
                    F32Scatter::add(gyz, cn.yz, b0 * e0, gt);
                    F32Scatter::add(gyz, cn.yz + 1, b1 * e0, gt);
                    F32Scatter::add(gyz, cn.yz + ny, b0 * e1, gt);
                    F32Scatter::add(gyz, cn.yz + ny + 1, b1 * e1, gt);
                }
                carry += __shfl(incl, kGroup - 1, kGroup);
                carryS = __shfl(sincl, kGroup - 1, kGroup);
                done += nb_eff;
                return done >= ne;
            });
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 499; i += kBlock) {
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

hipError_t launch_march_fwd(const SceneDev& sc, bool bf16, const RayParams& rp, const float* o, const float* d,
                            int64_t n, float* F, float* T, int32_t* n_placed, int32_t* n_eval, hipStream_t s) {
    if (bf16)
        hipLaunchKernelGGL(k_march_fwd<BF16Store>, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, rp, o, d, n, F, T,
                           n_placed, n_eval);
    else
        hipLaunchKernelGGL(k_march_fwd<F32Store>, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, rp, o, d, n, F, T,
                           n_placed, n_eval);
    return hipGetLastError();
}

hipError_t launch_march_bwd(const SceneDev& sc, bool bf16, const RayParams& rp, const float* o, const float* d,
                            int64_t n, const float* F, const float* T, const int32_t* n_eval, const float* dC,
                            float* gV, float* gxy, float* gxz, float* gyz, float* gmlp, hipStream_t s) {
    // Persistent blocks, each owning a contiguous chunk of rays, so the MLP
    // weight gradients are reduced in LDS over many rays before one set of
    // global atomics per block.
    const int64_t max_blocks = 4096;
    int64_t nb = (n + kGroupsPerBlock - 1) / kGroupsPerBlock;
    if (nb > max_blocks) nb = max_blocks;
    int64_t chunk = (n + nb - 1) / nb;
    chunk = (chunk + kGroupsPerBlock - 1) / kGroupsPerBlock * kGroupsPerBlock;
    nb = (n + chunk - 1) / chunk;
    if (bf16)
        hipLaunchKernelGGL(k_march_bwd<BF16Store>, dim3((unsigned)nb), dim3(kBlock), 0, s, sc, rp, o, d, n, chunk, F, T,
                           n_eval, dC, gV, gxy, gxz, gyz, gmlp);
    else
        hipLaunchKernelGGL(k_march_bwd<F32Store>, dim3((unsigned)nb), dim3(kBlock), 0, s, sc, rp, o, d, n, chunk, F, T,
                           n_eval, dC, gV, gxy, gxz, gyz, gmlp);
    return hipGetLastError();
}

}  // namespace omerf
