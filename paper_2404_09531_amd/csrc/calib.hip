// calib.hip -- calibration kernels for the bench's ceilings (measurement
// only; built into libomcalib.so, not part of the C ABI of
// include/omerf.h): the cache-resident gather rate of the forwards and the
// float-atomic segment rate of the backward.
//
// The forward marches are limited by how fast the vector memory path
// returns gathered 16-byte lane loads to registers, not by HBM: their
// feature rows are re-read from L1/L2 many times per frame.  This kernel
// measures that rate with the same load shape on data that is resident in
// each CU's L1: every lane issues 16-byte loads, lanes in groups of `span`
// (1, 4 or 16) read one contiguous span of span x 16 bytes, and each group
// picks its span with its own linear congruential sequence inside a small
// buffer, so the lanes of one load instruction touch up to 64 / span
// different places, as the gathers do.  Bytes returned = loads x 16.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_l1_gather(const uint4* __restrict__ buf, uint32_t mask, int span_shift,
                                                        int iters, float* __restrict__ sink) {
    const uint32_t tid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t lane_in_span = threadIdx.x & ((1u << span_shift) - 1u);
    uint32_t x = (tid >> span_shift) * 2654435761u + 12345u;  // same sequence for every lane of a span
    float acc0 = 0.0f, acc1 = 0.0f;
    for (int it = 0; it < iters; ++it) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            x = x * 1664525u + 1013904223u;
            const uint32_t base = ((x >> 8) & mask) & ~((1u << span_shift) - 1u);
            v[u] = buf[base + lane_in_span];
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            acc0 += __uint_as_float(v[u].x ^ v[u].w) + __uint_as_float(v[u].y ^ v[u].z);
            acc1 += __uint_as_float(v[u + 1].x ^ v[u + 1].w) + __uint_as_float(v[u + 1].y ^ v[u + 1].z);
        }
    }
    sink[tid] = acc0 + acc1;
}

// Request rate of 64-byte float-atomic segments: each 16-lane group adds
// one float per lane to one 64-byte segment (16 floats) per instruction, the
// shape of the backward's segment flush, at a segment drawn by a hash of
// (group, iteration) from `nseg` segments (a power of two).  One request
// per group and iteration.
__device__ __forceinline__ uint32_t mix32(uint32_t a) {
    a ^= a >> 16;
    a *= 0x7feb352du;
    a ^= a >> 15;
    a *= 0x846ca68bu;
    a ^= a >> 16;
    return a;
}

__global__ __launch_bounds__(kThreads) void k_atomic_segments(float* __restrict__ buf, uint32_t seg_mask, int iters) {
    const uint32_t g = (blockIdx.x * kThreads + threadIdx.x) >> 4, l = threadIdx.x & 15u;
    for (int it = 0; it < iters; ++it) {
        const uint32_t seg = mix32(g * 977u + (uint32_t)it) & seg_mask;
        unsafeAtomicAdd(buf + (size_t)seg * 16 + l, 1.0f);
    }
}

}  // namespace

extern "C" {

// Launches `blocks` blocks of 256 threads; each thread issues 8 * iters
// 16-byte loads from buf (device, nvec 16-byte vectors, nvec a power of two,
// every index below nvec readable) and writes one float to sink (device,
// blocks * 256 floats).  span = 1, 2, 4, 8 or 16.  Returns 0, or -1 for bad
// arguments (nothing launched), or the HIP error code of the launch.
int omcalib_l1_gather(const void* buf, int64_t nvec, int span, int blocks, int iters, float* sink, void* stream) {
    if (!buf || !sink || nvec < 16 || (nvec & (nvec - 1)) || blocks < 1 || iters < 1) return -1;
    int shift = 0;
    while ((1 << shift) < span) ++shift;
    if ((1 << shift) != span || shift > 4 || nvec > (int64_t)1 << 24) return -1;
    hipLaunchKernelGGL(k_l1_gather, dim3((unsigned)blocks), dim3(kThreads), 0, (hipStream_t)stream,
                       static_cast<const uint4*>(buf), (uint32_t)(nvec - 1), shift, iters, sink);
    return (int)hipGetLastError();
}

// Launches `blocks` blocks of 256 threads; each 16-lane group issues
// `iters` float-atomic adds of one 64-byte segment of buf (device, nseg
// segments of 16 floats, nseg a power of two <= 2^26; the values grow by
// 1.0 per add).  Requests = blocks * 16 * iters.  Returns 0, -1 for bad
// arguments (nothing launched), or the HIP error code of the launch.
int omcalib_atomic_segments(float* buf, int64_t nseg, int blocks, int iters, void* stream) {
    if (!buf || nseg < 1 || (nseg & (nseg - 1)) || nseg > ((int64_t)1 << 26) || blocks < 1 || iters < 1) return -1;
    hipLaunchKernelGGL(k_atomic_segments, dim3((unsigned)blocks), dim3(kThreads), 0, (hipStream_t)stream, buf,
                       (uint32_t)(nseg - 1), iters);
    return (int)hipGetLastError();
}

}  // extern "C"
