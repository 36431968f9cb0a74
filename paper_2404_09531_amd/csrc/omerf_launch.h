// omerf_launch.h -- host-side launchers shared between the translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "omerf_device.h"

namespace omerf {

hipError_t launch_place(const SceneDev& sc, const RayParams& rp, const float* o, const float* d, int64_t n,
                        int32_t* k_out, int32_t* n_placed, hipStream_t s);
hipError_t launch_mark(const SceneDev& sc, const RayParams& rp, const float* o, const float* d, int64_t n,
                       const int32_t* n_eval, uint8_t* fg, uint8_t* fxy, uint8_t* fxz, uint8_t* fyz, hipStream_t s);
hipError_t launch_march_fwd(const SceneDev& sc, int dtype, const RayParams& rp, const float* o, const float* d,
                            int64_t n, float* F, float* T, int32_t* n_placed, int32_t* n_eval, float* batch_wv,
                            hipStream_t s);
// Scheduling words (int32) of the march backward in its workspace: the
// ray-order histogram, its cursors and the hand-out counter.
constexpr int kBwdSchedWords = 256;
hipError_t launch_march_bwd(const SceneDev& sc, bool bf16, const RayParams& rp, const float* o, const float* d,
                            int64_t n, const float* T, const int32_t* n_eval, const float* batch_wv, const float* G8,
                            int32_t* order, int* sched, float* gV, float* gxy, float* gxz, float* gyz, float* gocc,
                            hipStream_t s);
hipError_t launch_mlp_bwd(const float* W, int mlp_in, const RayParams& rp, const float* F, const float* d,
                          const int32_t* n_eval, const float* dC, const float* dF, int64_t n, float* G8, float* gmlp,
                          hipStream_t s);
hipError_t launch_smooth(const float* W, int mlp_in, const float* F, const float* d, int64_t n, const float* perturb,
                         int P, float weight, float* loss, float* dF, float* gmlp, hipStream_t s);
hipError_t launch_mlp(const float* W, int mlp_in, bool bf16, const RayParams& rp, const float* d, int64_t n, const float* F,
                      const float* T, const int32_t* n_eval, float* C, hipStream_t s);
hipError_t launch_occ_pyramid(const float2* occ, int Mx, int My, float2* mips, int levels, hipStream_t s);
hipError_t launch_occ_loss(const float* occ, int64_t cells, float weight, float* loss, float* grad, hipStream_t s);
hipError_t launch_range(const float* x, int64_t n, float* minmax, uint32_t* keys, hipStream_t s);
hipError_t launch_quantize(const float* x, int64_t n, const float* lo, const float* inv, uint8_t* out, hipStream_t s);
hipError_t launch_blocks_mark(const SceneDev& sc, int shift, int bnx, int bny, int bnz, int32_t* mark, hipStream_t s);
hipError_t launch_blocks_fill(const SceneDev& sc, int shift, int bnx, int bny, int bnz, const int32_t* idx,
                              int64_t n_blocks, int units, void* atlas, hipStream_t s);
hipError_t launch_cast_bf16(const float* src, int64_t n, uint16_t* dst, hipStream_t s);
hipError_t launch_l2(const float* C, const float* tgt, int64_t n, float* dC, float* loss, hipStream_t s);
// Ray locality order (order.hip): histogram bytes of its workspace, the
// order with the reordered rays, and row gathers / scatters.
int64_t order_hist_bytes();
hipError_t launch_order_rays(const float* box_lo, const float* box_hi, const float* o, const float* d, int64_t n,
                             int32_t* order, float* o_out, float* d_out, int* hist, uint16_t* keys,
                             hipStream_t s);
hipError_t launch_rows_gather(const float* src, int64_t src_rows, int cols, const int32_t* idx, int64_t n,
                              float* dst, hipStream_t s);
hipError_t launch_rows_scatter(const float* src, int cols, const int32_t* idx, int64_t n, float* dst,
                               int64_t dst_rows, hipStream_t s);
hipError_t launch_l2_fp64(const float* C, const float* tgt, int64_t n, double* loss, hipStream_t s);

}  // namespace omerf
