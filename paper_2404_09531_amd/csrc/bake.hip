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

}  // namespace omerf
