// bake.hip -- 8-bit storage of the features (Sec. 4.4: the baked features
// are kept as 8-bit images).  Channel c of a source is stored as a byte q
// standing for lo_c + q step_c, with lo = the channel minimum and
// step = (max - lo) / 255 over the source.
//
// k_range    : per-channel (min, max) of a float32 [n][8] array; each block
//              reduces a grid-stride slice and merges with float atomics
//              on the order-preserving integer image of the values.
// k_quantize : q = clamp(rint(fl32(fl32(x - lo) * inv)), 0, 255), the code
//              decision taken in binary32 (NaN -> 0).
// k_blocks_* : sparse voxel-block storage of the grid (which blocks to
//              keep, and the copy into the block atlas).
// k_cast_bf16: the bfloat16 shadow of a float32 tensor, rounded to nearest
//              even (the re-cast after each optimiser step of a bfloat16
//              scene with float32 master parameters).
#include "../../include/omerf.h"
#include "omerf_device.h"
#include "omerf_launch.h"

namespace omerf {

// Monotone map of a float's bits to uint32 (and back), so that unsigned
// integer min/max order the floats (no NaN in the reduced data).
__device__ __forceinline__ uint32_t ord_key(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_val(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_range_init(uint32_t* keys) {
    const int i = threadIdx.x;
    if (i < 16) keys[i] = (i & 1) ? 0u : 0xffffffffu;  // (min, max) per channel
}

// One thread per (vertex, channel) pair of a grid-stride sweep; the channel
// of a thread is fixed (the stride is a multiple of 8).
__global__ __launch_bounds__(kBlock) void k_range(const float* __restrict__ x, int64_t count, uint32_t* keys) {
    const int c = threadIdx.x & 7;
    uint32_t kmin = 0xffffffffu, kmax = 0u;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        const uint32_t k = ord_key(x[i]);
        kmin = min(kmin, k);
        kmax = max(kmax, k);
    }
    // reduce the 8 lanes of equal channel in the wave (lanes c, c+8, ...)
#pragma unroll
    for (int off = 8; off < 64; off <<= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
    }
    if ((threadIdx.x & 63) < 8) {
        atomicMin(keys + 2 * c, kmin);
        atomicMax(keys + 2 * c + 1, kmax);
    }
}

__global__ void k_range_final(const uint32_t* keys, float* minmax) {
    const int i = threadIdx.x;
    if (i < 16) minmax[i] = ord_val(keys[i]);
}

hipError_t launch_range(const float* x, int64_t n, float* minmax, uint32_t* keys, hipStream_t s) {
    hipLaunchKernelGGL(k_range_init, dim3(1), dim3(64), 0, s, keys);
    const int64_t count = n * 8;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_range, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, count, keys);
    hipLaunchKernelGGL(k_range_final, dim3(1), dim3(64), 0, s, keys, minmax);
    return hipGetLastError();
}

struct QuantParams {
    float lo[8], inv[8];
};

__global__ __launch_bounds__(kBlock) void k_quantize(const float* __restrict__ x, int64_t n, QuantParams qp,
                                                     uint2* __restrict__ out) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float4 a = reinterpret_cast<const float4*>(x)[2 * i];
    const float4 b = reinterpret_cast<const float4*>(x)[2 * i + 1];
    const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t q[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float y = rintf((v[c] - qp.lo[c]) * qp.inv[c]);
        q[c] = (uint32_t)fminf(fmaxf(y, 0.0f), 255.0f);  // fmaxf(NaN, 0) = 0
    }
    out[i] = make_uint2(q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24),
                        q[4] | (q[5] << 8) | (q[6] << 16) | (q[7] << 24));
}

hipError_t launch_quantize(const float* x, int64_t n, const float* lo, const float* inv, uint8_t* out, hipStream_t s) {
    QuantParams qp;
    for (int c = 0; c < 8; ++c) {
        qp.lo[c] = lo[c];
        qp.inv[c] = inv[c];
    }
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, n, qp, reinterpret_cast<uint2*>(out));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sparse voxel blocks of the grid (Sec. 4.4: the baked grid is stored as
// sparse blocks, chosen from the occupancy plane).  A block covers B^3
// cells; it is kept if some occupancy column overlapping its xy extent (one
// column of padding) has an interval meeting its z extent (one cell of
// padding), which holds for every block that contains a placed sample.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_blocks_mark(SceneDev sc, int shift, int bnx, int bny, int bnz,
                                                        int32_t* __restrict__ mark) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)bnx * bny * bnz) return;
    const int bx = (int)(i % bnx), by = (int)((i / bnx) % bny), bz = (int)(i / ((int64_t)bnx * bny));
    const int B = 1 << shift;
    // vertex ranges of the block's cells
    const int x0 = bx * B, x1 = min(x0 + B, sc.Lx - 1);
    const int y0 = by * B, y1 = min(y0 + B, sc.Ly - 1);
    const int z0 = bz * B, z1 = min(z0 + B, sc.Lz - 1);
    const float hx = (sc.hi0 - sc.lo0) / (float)(sc.Lx - 1), hy = (sc.hi1 - sc.lo1) / (float)(sc.Ly - 1);
    const float hz = (sc.hi2 - sc.lo2) / (float)(sc.Lz - 1);
    const float za = sc.lo2 + (float)(z0 - 1) * hz, zb = sc.lo2 + (float)(z1 + 1) * hz;
    const int cx0 = max(0, (int)floorf((float)x0 * hx * sc.occ_sx) - 1);
    const int cx1 = min(sc.Mx - 1, (int)floorf((float)x1 * hx * sc.occ_sx) + 1);
    const int cy0 = max(0, (int)floorf((float)y0 * hy * sc.occ_sy) - 1);
    const int cy1 = min(sc.My - 1, (int)floorf((float)y1 * hy * sc.occ_sy) + 1);
    int keep = 0;
    for (int cy = cy0; cy <= cy1 && !keep; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) {
            const float2 z = sc.occ[(size_t)cy * sc.Mx + cx];
            if (z.x <= z.y && z.x <= zb && z.y >= za) {
                keep = 1;
                break;
            }
        }
    mark[i] = keep;
}

hipError_t launch_blocks_mark(const SceneDev& sc, int shift, int bnx, int bny, int bnz, int32_t* mark, hipStream_t s) {
    const int64_t n = (int64_t)bnx * bny * bnz;
    hipLaunchKernelGGL(k_blocks_mark, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, sc, shift, bnx,
                       bny, bnz, mark);
    return hipGetLastError();
}

// One workgroup per block-index entry: copies the (B + 1)^3 vertices of a
// kept block (vertices past the grid's last one are zero) into its atlas
// slot; workgroup 0 of the first launch also zeroes atlas block 0.
__global__ __launch_bounds__(kBlock) void k_blocks_fill(SceneDev sc, int shift, int bnx, int bny,
                                                        const int32_t* __restrict__ idx, int64_t n_blocks, int units,
                                                        uint2* __restrict__ atlas) {
    const int64_t e = blockIdx.x;
    const int B = 1 << shift, E = B + 1;
    const int64_t per = (int64_t)E * E * E * units;  // 8-byte units per block
    if (e == 0) {
        for (int64_t u = threadIdx.x; u < per; u += kBlock) atlas[u] = make_uint2(0u, 0u);
    }
    const int32_t id = idx[e];
    if (id <= 0 || id > n_blocks) return;  // ids past the atlas are not written
    const int bx = (int)(e % bnx), by = (int)((e / bnx) % bny), bz = (int)(e / ((int64_t)bnx * bny));
    const uint2* src = reinterpret_cast<const uint2*>(sc.grid);
    uint2* dst = atlas + (int64_t)id * per;
    for (int64_t u = threadIdx.x; u < per; u += kBlock) {
        const int v = (int)(u / units), w = (int)(u - (int64_t)v * units);
        const int lx = v % E, ly = (v / E) % E, lz = v / (E * E);
        const int x = bx * B + lx, y = by * B + ly, z = bz * B + lz;
        uint2 val = make_uint2(0u, 0u);
        if (x < sc.Lx && y < sc.Ly && z < sc.Lz)
            val = src[(((int64_t)z * sc.Ly + y) * sc.Lx + x) * units + w];
        dst[u] = val;
    }
}

hipError_t launch_blocks_fill(const SceneDev& sc, int shift, int bnx, int bny, int bnz, const int32_t* idx,
                              int64_t n_blocks, int units, void* atlas, hipStream_t s) {
    const int64_t n = (int64_t)bnx * bny * bnz;
    hipLaunchKernelGGL(k_blocks_fill, dim3((unsigned)n), dim3(kBlock), 0, s, sc, shift, bnx, bny, idx, n_blocks, units,
                       reinterpret_cast<uint2*>(atlas));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// float32 -> bfloat16 (the upper 16 bits of a binary32), rounded to nearest,
// ties to even: add 0x7fff plus the kept part's lowest bit, then truncate.
// Finite values beyond the largest bfloat16 round to infinity; NaN stays a
// (quiet) NaN with its sign.  Eight values per thread: two 16-byte loads and
// one 16-byte store; the tail of n mod 8 values is converted one per thread.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // NaN: keep it quiet
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__global__ __launch_bounds__(kBlock) void k_cast_bf16(const float4* __restrict__ src, uint4* __restrict__ dst,
                                                      int64_t n8) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n8; i += stride) {
        const float4 a = src[2 * i], b = src[2 * i + 1];
        uint4 o;
        o.x = bf16_rne(a.x) | (bf16_rne(a.y) << 16);
        o.y = bf16_rne(a.z) | (bf16_rne(a.w) << 16);
        o.z = bf16_rne(b.x) | (bf16_rne(b.y) << 16);
        o.w = bf16_rne(b.z) | (bf16_rne(b.w) << 16);
        dst[i] = o;
    }
}

__global__ void k_cast_bf16_tail(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t first,
                                 int64_t n) {
    const int64_t i = first + threadIdx.x;
    if (i < n) dst[i] = (uint16_t)bf16_rne(src[i]);
}

hipError_t launch_cast_bf16(const float* src, int64_t n, uint16_t* dst, hipStream_t s) {
    const int64_t n8 = n / 8;
    if (n8 > 0) {
        int64_t blocks = (n8 + kBlock - 1) / kBlock;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                           reinterpret_cast<const float4*>(src), reinterpret_cast<uint4*>(dst), n8);
    }
    if (n8 * 8 < n) hipLaunchKernelGGL(k_cast_bf16_tail, dim3(1), dim3(8), 0, s, src, dst, n8 * 8, n);
    return hipGetLastError();
}

}  // namespace omerf
