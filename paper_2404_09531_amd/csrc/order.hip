// order.hip -- a locality order for a batch of rays, and row gathers and
// scatters to apply it.  Scheduling only: every ray is rendered on its own,
// so no result depends on the order.  The march reads the grid and plane
// rows around each sample; rays that cross the scene close to one another
// read the same rows, and when they sit in the same waves and blocks those
// rows are fetched once into L1/L2 instead of once per ray.
//
// Key: the point where the ray meets the horizontal plane halfway up the
// scene box, on a 256 x 256 lattice over the box's ground footprint, as a
// 16-bit Morton code (x in the even bits).  Points outside the footprint
// are clamped to its edge; a ray parallel to the plane, or one whose key
// point is not finite, gets the cell of its own origin or cell 0.
//
// k_okey_clear   : zero the 65,536-bin histogram (a fill kernel, so the
//                  call can be captured in a graph).
// k_okey_hist    : per ray its key (kept in the workspace for the
//                  scatter); each run of equal keys among consecutive rays
//                  of a wave adds its length once.
// k_okey_scan    : exclusive prefix sum of the histogram, in place (one
//                  block; 64 bins per thread).
// k_okey_scatter : reads the stored keys, so its runs are those the
//                  histogram counted and every slot lies in [0, n); each
//                  run reserves its slots in its bin with one atomic
//                  and its rays take consecutive slots in input order;
//                  writes order[slot] = ray and the ray's origin and
//                  direction at that slot.  Runs of one bin land in the
//                  order their atomics are served.
// k_rows_gather / k_rows_scatter : dst[i] = src[idx[i]] and
//                  dst[idx[i]] = src[i] on rows of `cols` floats; indices
//                  outside the rows are skipped.
#include "../../include/omerf.h"
#include "omerf_launch.h"

namespace omerf {

namespace {

constexpr int kOrderBlock = 256;
constexpr int kAxisBits = 8;
constexpr int kKeyBins = 1 << (2 * kAxisBits);
constexpr int kScanThreads = 1024;
constexpr int kBinsPerThread = kKeyBins / kScanThreads;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// The key's lattice: footprint origin, cells per unit length, and the
// height of the key plane.
struct KeyFrame {
    float lo_x, lo_y, cells_x, cells_y, z_mid;
};

__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {
    v &= 0xFFu;
    v = (v | (v << 4)) & 0x0F0Fu;
    v = (v | (v << 2)) & 0x3333u;
    v = (v | (v << 1)) & 0x5555u;
    return v;
}

// Lattice cell of a coordinate already scaled to cells (NaN and values
// below the footprint -> 0, values past it -> the last cell).
__device__ __forceinline__ uint32_t axis_cell(float u) {
    if (!(u > 0.0f)) return 0u;
    if (u >= (float)(1 << kAxisBits)) return (1u << kAxisBits) - 1u;
    return (uint32_t)u;
}

__device__ __forceinline__ uint32_t ray_key(const float* o, const float* d, int64_t i, const KeyFrame& kf) {
    const float ox = o[3 * i], oy = o[3 * i + 1], oz = o[3 * i + 2];
    const float dx = d[3 * i], dy = d[3 * i + 1], dz = d[3 * i + 2];
    float t = dz != 0.0f ? (kf.z_mid - oz) / dz : 0.0f;
    if (!(fabsf(t) < INFINITY)) t = 0.0f;
    const float x = fmaf(t, dx, ox), y = fmaf(t, dy, oy);
    return spread_bits(axis_cell((x - kf.lo_x) * kf.cells_x)) |
           (spread_bits(axis_cell((y - kf.lo_y) * kf.cells_y)) << 1);
}

// Runs of equal keys among the lanes of a wave: `heads` has a bit for each
// lane that starts a run (lane 0, a lane whose key differs from the lane
// below, and every lane past the end of the input, which has kNoKey).
__device__ __forceinline__ uint64_t run_heads(uint32_t key, int lane) {
    const uint32_t below = (uint32_t)__shfl_up((int)key, 1);
    return __ballot(lane == 0 || key == kNoKey || below != key);
}

__device__ __forceinline__ int run_length(uint64_t heads, int lane) {
    const uint64_t above = lane == 63 ? 0ull : heads & ~((2ull << lane) - 1ull);
    return (above ? __builtin_ctzll(above) : 64) - lane;
}

}  // namespace

// Kernels sit outside the unnamed namespace so that profiles show their names.
__global__ void __launch_bounds__(kOrderBlock) k_okey_clear(int* hist) {
    const int i = blockIdx.x * kOrderBlock + threadIdx.x;
    if (i < kKeyBins) hist[i] = 0;
}

__global__ void __launch_bounds__(kOrderBlock) k_okey_hist(const float* __restrict__ o, const float* __restrict__ d,
                                                            int64_t n, KeyFrame kf, uint16_t* __restrict__ keys,
                                                            int* __restrict__ hist) {
    const int64_t i = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint32_t key = i < n ? ray_key(o, d, i, kf) : kNoKey;
    if (i < n) keys[i] = (uint16_t)key;
    const uint64_t heads = run_heads(key, lane);
    if (key != kNoKey && ((heads >> lane) & 1ull)) atomicAdd(&hist[key], run_length(heads, lane));
}

__global__ void __launch_bounds__(kScanThreads) k_okey_scan(int* hist) {
    __shared__ int part[kScanThreads];
    const int t = threadIdx.x;
    int* bins = hist + t * kBinsPerThread;
    int sum = 0;
    for (int j = 0; j < kBinsPerThread; ++j) sum += bins[j];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    for (int j = 0; j < kBinsPerThread; ++j) {
        const int c = bins[j];
        bins[j] = run;
        run += c;
    }
}

__global__ void __launch_bounds__(kOrderBlock) k_okey_scatter(const float* __restrict__ o, const float* __restrict__ d,
                                                               int64_t n, const uint16_t* __restrict__ keys,
                                                               int* __restrict__ cursor,
                                                               int32_t* __restrict__ order, float* __restrict__ o_out,
                                                               float* __restrict__ d_out) {
    const int64_t i = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint32_t key = i < n ? (uint32_t)keys[i] : kNoKey;
    const uint64_t heads = run_heads(key, lane);
    int base = 0;
    if (key != kNoKey && ((heads >> lane) & 1ull)) base = atomicAdd(&cursor[key], run_length(heads, lane));
    const int head = 63 - __builtin_clzll(heads & (lane == 63 ? ~0ull : (2ull << lane) - 1ull));
    base = __shfl(base, head);
    const int64_t slot = (int64_t)base + (lane - head);
    if (key == kNoKey || slot >= n) return;
    order[slot] = (int32_t)i;
    for (int c = 0; c < 3; ++c) {
        o_out[3 * slot + c] = o[3 * i + c];
        d_out[3 * slot + c] = d[3 * i + c];
    }
}

__global__ void __launch_bounds__(kOrderBlock) k_rows_gather(const float* __restrict__ src, int64_t src_rows, int cols,
                                                              const int32_t* __restrict__ idx, int64_t n,
                                                              float* __restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    if (e >= n * cols) return;
    const int64_t i = e / cols;
    const int c = (int)(e - i * cols);
    const int64_t r = idx[i];
    if (r >= 0 && r < src_rows) dst[e] = src[r * cols + c];
}

__global__ void __launch_bounds__(kOrderBlock) k_rows_scatter(const float* __restrict__ src, int cols,
                                                               const int32_t* __restrict__ idx, int64_t n,
                                                               float* __restrict__ dst, int64_t dst_rows) {
    const int64_t e = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    if (e >= n * cols) return;
    const int64_t i = e / cols;
    const int c = (int)(e - i * cols);
    const int64_t r = idx[i];
    if (r >= 0 && r < dst_rows) dst[r * cols + c] = src[e];
}

namespace {
unsigned blocks_for(int64_t items) { return (unsigned)((items + kOrderBlock - 1) / kOrderBlock); }
}  // namespace

int64_t order_hist_bytes() { return (int64_t)kKeyBins * (int64_t)sizeof(int); }

hipError_t launch_order_rays(const float* box_lo, const float* box_hi, const float* o, const float* d, int64_t n,
                             int32_t* order, float* o_out, float* d_out, int* hist, uint16_t* keys, hipStream_t s) {
    const float cells = (float)(1 << kAxisBits);
    const KeyFrame kf{box_lo[0], box_lo[1], cells / (box_hi[0] - box_lo[0]), cells / (box_hi[1] - box_lo[1]),
                      0.5f * (box_lo[2] + box_hi[2])};
    hipLaunchKernelGGL(k_okey_clear, dim3(blocks_for(kKeyBins)), dim3(kOrderBlock), 0, s, hist);
    hipLaunchKernelGGL(k_okey_hist, dim3(blocks_for(n)), dim3(kOrderBlock), 0, s, o, d, n, kf, keys, hist);
    hipLaunchKernelGGL(k_okey_scan, dim3(1), dim3(kScanThreads), 0, s, hist);
    hipLaunchKernelGGL(k_okey_scatter, dim3(blocks_for(n)), dim3(kOrderBlock), 0, s, o, d, n, keys, hist, order, o_out,
                       d_out);
    return hipGetLastError();
}

hipError_t launch_rows_gather(const float* src, int64_t src_rows, int cols, const int32_t* idx, int64_t n,
                              float* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_gather, dim3(blocks_for(n * cols)), dim3(kOrderBlock), 0, s, src, src_rows, cols, idx, n,
                       dst);
    return hipGetLastError();
}

hipError_t launch_rows_scatter(const float* src, int cols, const int32_t* idx, int64_t n, float* dst,
                               int64_t dst_rows, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_scatter, dim3(blocks_for(n * cols)), dim3(kOrderBlock), 0, s, src, cols, idx, n, dst,
                       dst_rows);
    return hipGetLastError();
}

}  // namespace omerf
