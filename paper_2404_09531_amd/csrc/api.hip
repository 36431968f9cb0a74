// api.hip -- C ABI of the ray marcher (declared in include/omerf.h):
// argument validation, scene handles, launch sequencing and error strings.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/omerf.h"
#include "omerf_device.h"
#include "omerf_launch.h"

using namespace omerf;

struct om_scene {
    om_scene_desc desc;
    SceneDev dev;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return OM_OK;
}

bool pow2(double v) {
    if (!(v > 0.0) || !std::isfinite(v)) return false;
    int e;
    return std::frexp(v, &e) == 0.5;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// u = p * (n - 1)/(hi - lo) - lo * (n - 1)/(hi - lo), split as p * s + (ci + cf).
int make_axis(float lo, float hi, int n, const char* name, AxisMap* m) {
    const double ext = (double)hi - (double)lo;
    const double s = (double)(n - 1) / ext;
    const double c = -(double)lo * s;
    if ((double)(float)s != s) return fail(OM_ERR_UNSUPPORTED, "%s: scale (n-1)/extent not exact in binary32", name);
    if ((double)(float)c != c) return fail(OM_ERR_UNSUPPORTED, "%s: offset -lo*(n-1)/extent not exact in binary32", name);
    if (std::fmax(std::fabs((double)lo), std::fabs((double)hi)) * s >= 4194304.0)
        return fail(OM_ERR_UNSUPPORTED, "%s: coordinate range too large for exact splitting", name);
    m->s = (float)s;
    const double ci = std::floor(c);
    m->ci = (int)ci;
    m->cf = (float)(c - ci);
    m->n = n;
    return OM_OK;
}

int validate_desc(const om_scene_desc* d, SceneDev* out) {
    if (!d) return fail(OM_ERR_INVALID, "scene descriptor is NULL");
    const float* lo = d->box_lo;
    const float* hi = d->box_hi;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] > lo[a]))
            return fail(OM_ERR_INVALID, "box axis %d: need finite lo < hi", a);
        if (!pow2((double)hi[a] - (double)lo[a]))
            return fail(OM_ERR_UNSUPPORTED, "box axis %d: extent must be a power of two", a);
        if (d->grid_dims[a] < 2 || d->plane_dims[a] < 2)
            return fail(OM_ERR_INVALID, "axis %d: grid and plane dims must be >= 2", a);
    }
    const int64_t nv = (int64_t)d->grid_dims[0] * d->grid_dims[1] * d->grid_dims[2];
    const int64_t nxy = (int64_t)d->plane_dims[0] * d->plane_dims[1];
    const int64_t nxz = (int64_t)d->plane_dims[0] * d->plane_dims[2];
    const int64_t nyz = (int64_t)d->plane_dims[1] * d->plane_dims[2];
    if (nv >= (int64_t)1 << 31 || nxy >= (int64_t)1 << 31 || nxz >= (int64_t)1 << 31 || nyz >= (int64_t)1 << 31)
        return fail(OM_ERR_UNSUPPORTED, "feature sources must have fewer than 2^31 vertices");
    for (int a = 0; a < 2; ++a) {
        const int m = d->occ_dims[a];
        if (m < 1) return fail(OM_ERR_INVALID, "occupancy dim %d must be >= 1", a);
        const double s = (double)m / ((double)hi[a] - (double)lo[a]);
        const double o = (double)lo[a] * s;
        if (!pow2(s)) return fail(OM_ERR_UNSUPPORTED, "occupancy axis %d: cells per unit length must be a power of two", a);
        if (o != std::floor(o) || std::fabs(o) >= 16777216.0)
            return fail(OM_ERR_UNSUPPORTED, "occupancy axis %d: box low corner must be an integer number of cells", a);
    }
    if ((int64_t)d->occ_dims[0] * d->occ_dims[1] >= (int64_t)1 << 31)
        return fail(OM_ERR_UNSUPPORTED, "occupancy plane too large");
    if (d->dtype != OM_F32 && d->dtype != OM_BF16 && d->dtype != OM_U8)
        return fail(OM_ERR_UNSUPPORTED, "dtype must be OM_F32, OM_BF16 or OM_U8");
    if (d->dtype == OM_U8) {
        for (int i = 0; i < 32; ++i) {
            const float lo = (&d->quant_lo[0][0])[i], st = (&d->quant_step[0][0])[i];
            if (!std::isfinite(lo) || !std::isfinite(st) || st < 0.0f)
                return fail(OM_ERR_INVALID, "quant_lo / quant_step must be finite with quant_step >= 0");
        }
    }
    if (d->dir_freqs != 0 && d->dir_freqs != 4) return fail(OM_ERR_UNSUPPORTED, "dir_freqs must be 0 or 4");
    if (d->block_shift < 0 || d->block_shift > 5) return fail(OM_ERR_INVALID, "block_shift must be in 0 .. 5");
    if (d->block_shift > 0) {
        const int64_t E = ((int64_t)1 << d->block_shift) + 1;
        if (!d->grid_blocks || ((uintptr_t)d->grid_blocks & 3u))
            return fail(OM_ERR_INVALID, "grid_blocks must be a 4-byte aligned device pointer");
        if (d->n_blocks < 0 || ((int64_t)d->n_blocks + 1) * E * E * E >= ((int64_t)1 << 31))
            return fail(OM_ERR_UNSUPPORTED, "n_blocks must be >= 0 with (n_blocks + 1) (B + 1)^3 < 2^31");
    }
    const void* ptrs[6] = {d->grid, d->plane_xy, d->plane_xz, d->plane_yz, d->occ, d->mlp};
    const char* names[6] = {"grid", "plane_xy", "plane_xz", "plane_yz", "occ", "mlp"};
    for (int i = 0; i < 6; ++i) {
        if (!ptrs[i]) return fail(OM_ERR_INVALID, "%s pointer is NULL", names[i]);
        if (!aligned16(ptrs[i])) return fail(OM_ERR_INVALID, "%s pointer is not 16-byte aligned", names[i]);
    }
    SceneDev s;
    s.mips = nullptr;  // no pyramid until om_build_occupancy_mips attaches one
    s.mip_levels = 0;
    s.grid = d->grid;
    s.pxy = d->plane_xy;
    s.pxz = d->plane_xz;
    s.pyz = d->plane_yz;
    s.occ = reinterpret_cast<const float2*>(d->occ);
    s.mlp = d->mlp;
    s.mlp_in = 10 + 6 * d->dir_freqs;
    s.gsy = (uint32_t)d->grid_dims[0];
    s.gsz = (uint32_t)d->grid_dims[0] * (uint32_t)d->grid_dims[1];
    s.blk_idx = nullptr;
    s.blk_shift = 0;
    s.bnx = s.bny = 0;
    s.blk_verts = 0;
    s.n_blocks = 0;
    if (d->block_shift > 0) {
        const int B = 1 << d->block_shift;
        s.blk_shift = d->block_shift;
        s.blk_idx = d->grid_blocks;
        s.bnx = (d->grid_dims[0] - 2) / B + 1;  // ceil((L - 1) / B)
        s.bny = (d->grid_dims[1] - 2) / B + 1;
        s.gsy = (uint32_t)(B + 1);
        s.gsz = (uint32_t)((B + 1) * (B + 1));
        s.blk_verts = (uint32_t)((B + 1) * (B + 1) * (B + 1));
        s.n_blocks = (uint32_t)d->n_blocks;
    }
    for (int i = 0; i < 32; ++i) {
        s.qlo[i] = d->dtype == OM_U8 ? (&d->quant_lo[0][0])[i] : 0.0f;
        s.qstep[i] = d->dtype == OM_U8 ? (&d->quant_step[0][0])[i] : 0.0f;
    }
    s.Lx = d->grid_dims[0];
    s.Ly = d->grid_dims[1];
    s.Lz = d->grid_dims[2];
    s.Nx = d->plane_dims[0];
    s.Ny = d->plane_dims[1];
    s.Nz = d->plane_dims[2];
    s.Mx = d->occ_dims[0];
    s.My = d->occ_dims[1];
    s.lo0 = lo[0];
    s.lo1 = lo[1];
    s.lo2 = lo[2];
    s.hi0 = hi[0];
    s.hi1 = hi[1];
    s.hi2 = hi[2];
    s.occ_sx = (float)((double)s.Mx / ((double)hi[0] - (double)lo[0]));
    s.occ_sy = (float)((double)s.My / ((double)hi[1] - (double)lo[1]));
    s.occ_ox = (float)((double)lo[0] * s.occ_sx);
    s.occ_oy = (float)((double)lo[1] * s.occ_sy);
    int rc;
    if ((rc = make_axis(lo[0], hi[0], s.Lx, "grid x", &s.gx)) != OM_OK) return rc;
    if ((rc = make_axis(lo[1], hi[1], s.Ly, "grid y", &s.gy)) != OM_OK) return rc;
    if ((rc = make_axis(lo[2], hi[2], s.Lz, "grid z", &s.gz)) != OM_OK) return rc;
    if ((rc = make_axis(lo[0], hi[0], s.Nx, "plane x", &s.px)) != OM_OK) return rc;
    if ((rc = make_axis(lo[1], hi[1], s.Ny, "plane y", &s.py)) != OM_OK) return rc;
    if ((rc = make_axis(lo[2], hi[2], s.Nz, "plane z", &s.pz)) != OM_OK) return rc;
    *out = s;
    return OM_OK;
}

int validate_params(const om_params* p, RayParams* rp) {
    if (!p) return fail(OM_ERR_INVALID, "params pointer is NULL");
    if (!pow2((double)p->delta)) return fail(OM_ERR_INVALID, "delta must be a positive power of two");
    if (!std::isfinite((double)p->delta * 16777216.0)) return fail(OM_ERR_INVALID, "delta too large");
    if (p->n_max < 1 || p->n_max > OM_MAX_SAMPLES)
        return fail(OM_ERR_UNSUPPORTED, "n_max must be in [1, %d]", OM_MAX_SAMPLES);
    if (!std::isfinite(p->t_term) || p->t_term < 0.0f) return fail(OM_ERR_INVALID, "t_term must be finite and >= 0");
    if (p->mlp_bf16 < -1 || p->mlp_bf16 > 1) return fail(OM_ERR_INVALID, "mlp_bf16 must be -1, 0 or 1");
    if (!std::isfinite(p->occ_eps) || p->occ_eps < 0.0f) return fail(OM_ERR_INVALID, "occ_eps must be finite and >= 0");
    const float inv = p->occ_eps > 0.0f ? 1.0f / p->occ_eps : 0.0f;
    if (!std::isfinite(inv)) return fail(OM_ERR_INVALID, "occ_eps too small");
    rp->occ_inv_eps = inv;
    rp->delta = p->delta;
    rp->n_max = p->n_max;
    rp->t_term = p->t_term;
    rp->bg0 = p->c_bg[0];
    rp->bg1 = p->c_bg[1];
    rp->bg2 = p->c_bg[2];
    return OM_OK;
}

int check_rays(const om_scene* sc, const float* o, const float* d, int64_t n) {
    if (!sc) return fail(OM_ERR_INVALID, "scene handle is NULL");
    if (n < 0) return fail(OM_ERR_INVALID, "n must be >= 0");
    if (n > ((int64_t)1 << 31) - 1) return fail(OM_ERR_UNSUPPORTED, "n must be below 2^31");
    if (n > 0 && (!o || !d)) return fail(OM_ERR_INVALID, "ray pointers are NULL");
    return OM_OK;
}

int hip_status(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(OM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

}  // namespace

extern "C" {

int om_scene_create(const om_scene_desc* desc, om_scene** out) {
    if (!out) return fail(OM_ERR_INVALID, "output handle pointer is NULL");
    *out = nullptr;
    SceneDev dev;
    int rc = validate_desc(desc, &dev);
    if (rc != OM_OK) return rc;
    om_scene* s = new (std::nothrow) om_scene;
    if (!s) return fail(OM_ERR_INVALID, "out of host memory");
    s->desc = *desc;
    s->dev = dev;
    *out = s;
    return ok();
}

int om_scene_update(om_scene* scene, const om_scene_desc* desc) {
    if (!scene) return fail(OM_ERR_INVALID, "scene handle is NULL");
    SceneDev dev;
    int rc = validate_desc(desc, &dev);
    if (rc != OM_OK) return rc;
    scene->desc = *desc;
    scene->dev = dev;
    return ok();
}

int om_scene_destroy(om_scene* scene) {
    delete scene;
    return ok();
}

int64_t om_occupancy_mips_size(const om_scene* scene, int levels) {
    if (!scene) {
        fail(OM_ERR_INVALID, "scene handle is NULL");
        return -1;
    }
    const int Mx = scene->dev.Mx, My = scene->dev.My;
    if (levels < 0 || levels > kMaxMipLevels || (Mx % (1 << levels)) || (My % (1 << levels))) {
        fail(OM_ERR_UNSUPPORTED, "levels must be in [0, %d] with both occupancy dims divisible by 2^levels",
             kMaxMipLevels);
        return -1;
    }
    int64_t cells = 0;
    for (int l = 1; l <= levels; ++l) cells += (int64_t)(Mx >> l) * (My >> l);
    return cells * (int64_t)sizeof(float2);
}

int om_build_occupancy_mips(om_scene* scene, void* mips, int64_t mips_bytes, int levels, void* stream) {
    const int64_t need = om_occupancy_mips_size(scene, levels);
    if (need < 0) return OM_ERR_INVALID;
    SceneDev& dev = scene->dev;
    dev.mips = nullptr;
    dev.mip_levels = 0;
    if (levels == 0) return ok();
    if (!mips || ((uintptr_t)mips & 7u)) return fail(OM_ERR_INVALID, "mips must be non-NULL and 8-byte aligned");
    if (mips_bytes < need)
        return fail(OM_ERR_INVALID, "mips holds %lld bytes, %lld needed", (long long)mips_bytes, (long long)need);
    hipError_t e = launch_occ_pyramid(dev.occ, dev.Mx, dev.My, static_cast<float2*>(mips), levels, (hipStream_t)stream);
    if (e != hipSuccess) return hip_status(e, "om_build_occupancy_mips");
    dev.mips = static_cast<const float2*>(mips);
    dev.mip_levels = levels;
    return ok();
}

int om_place_samples(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                     int32_t* k_out, int32_t* n_placed, void* stream) {
    int rc = check_rays(scene, o, d, n);
    if (rc != OM_OK) return rc;
    RayParams rp;
    if ((rc = validate_params(p, &rp)) != OM_OK) return rc;
    if (n == 0) return ok();
    if (!k_out || !n_placed) return fail(OM_ERR_INVALID, "output pointers are NULL");
    if ((int64_t)n * rp.n_max >= ((int64_t)1 << 62)) return fail(OM_ERR_INVALID, "k_out too large");
    return hip_status(launch_place(scene->dev, rp, o, d, n, k_out, n_placed, (hipStream_t)stream), "om_place_samples");
}

int om_mark_rows(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                 const int32_t* n_eval, uint8_t* grid_flags, uint8_t* xy_flags, uint8_t* xz_flags,
                 uint8_t* yz_flags, void* stream) {
    int rc = check_rays(scene, o, d, n);
    if (rc != OM_OK) return rc;
    RayParams rp;
    if ((rc = validate_params(p, &rp)) != OM_OK) return rc;
    if (n == 0) return ok();
    if (!grid_flags || !xy_flags || !xz_flags || !yz_flags) return fail(OM_ERR_INVALID, "flag buffers are NULL");
    return hip_status(launch_mark(scene->dev, rp, o, d, n, n_eval, grid_flags, xy_flags, xz_flags, yz_flags,
                                  (hipStream_t)stream),
                      "om_mark_rows");
}

}  // extern "C"

namespace {

int check_fwd(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
              const om_fwd_out* out, bool need_o, bool need_C, RayParams* rp) {
    int rc = check_rays(scene, need_o ? o : d, d, n);
    if (rc != OM_OK) return rc;
    if ((rc = validate_params(p, rp)) != OM_OK) return rc;
    if (!out) return fail(OM_ERR_INVALID, "output struct is NULL");
    if (n == 0) return OM_OK;
    if ((need_C && !out->C) || (need_o && !out->n_placed) || !out->T || !out->F || !out->n_eval)
        return fail(OM_ERR_INVALID, "required om_fwd_out buffers are NULL");
    if (out->batch_wv && ((uintptr_t)out->batch_wv & 3u))
        return fail(OM_ERR_INVALID, "batch_wv must be 4-byte aligned");
    if (out->batch_wv && (scene->desc.dtype == OM_U8 || scene->desc.block_shift > 0))
        return fail(OM_ERR_UNSUPPORTED, "8-bit and sparse-block scenes are render-only: batch_wv must be NULL");
    return OM_OK;
}

bool mlp_in_bf16(const om_scene* scene, const om_params* p) {
    return p->mlp_bf16 < 0 ? scene->desc.dtype == OM_BF16 : p->mlp_bf16 == 1;
}

}  // namespace

extern "C" {

int om_march(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
             const om_fwd_out* out, void* stream) {
    RayParams rp;
    int rc = check_fwd(scene, o, d, n, p, out, true, false, &rp);
    if (rc != OM_OK || n == 0) return rc == OM_OK ? ok() : rc;
    return hip_status(launch_march_fwd(scene->dev, scene->desc.dtype, rp, o, d, n, out->F, out->T, out->n_placed, out->n_eval,
                                       out->batch_wv, (hipStream_t)stream), "om_march");
}

int om_deferred_mlp(const om_scene* scene, const float* d, int64_t n, const om_params* p, const om_fwd_out* out,
                    void* stream) {
    RayParams rp;
    int rc = check_fwd(scene, nullptr, d, n, p, out, false, true, &rp);
    if (rc != OM_OK || n == 0) return rc == OM_OK ? ok() : rc;
    return hip_status(launch_mlp(scene->dev.mlp, scene->dev.mlp_in, mlp_in_bf16(scene, p), rp, d, n, out->F, out->T, out->n_eval,
                                 out->C, (hipStream_t)stream), "om_deferred_mlp");
}

int om_render(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
              const om_fwd_out* out, void* stream) {
    RayParams rp;
    int rc = check_fwd(scene, o, d, n, p, out, true, true, &rp);
    if (rc != OM_OK || n == 0) return rc == OM_OK ? ok() : rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_march_fwd(scene->dev, scene->desc.dtype, rp, o, d, n, out->F, out->T, out->n_placed,
                                    out->n_eval, out->batch_wv, s);
    if (e != hipSuccess) return hip_status(e, "om_render (march)");
    e = launch_mlp(scene->dev.mlp, scene->dev.mlp_in, mlp_in_bf16(scene, p), rp, d, n, out->F, out->T, out->n_eval, out->C, s);
    return hip_status(e, "om_render (mlp)");
}

int64_t om_render_backward_workspace_size(int64_t n) {
    if (n < 0) {
        fail(OM_ERR_INVALID, "n must be >= 0");
        return -1;
    }
    // G8 (8 floats per ray), the ray order (one int32 per ray), the
    // scheduling words; each part 256-byte aligned.  No rays, no work.
    if (n == 0) return 0;
    return (n * 8 * (int64_t)sizeof(float) + 255) / 256 * 256 + (n * (int64_t)sizeof(int32_t) + 255) / 256 * 256 +
           kBwdSchedWords * (int64_t)sizeof(int32_t);
}

namespace {

int check_backward(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                   const om_fwd_out* saved, const float* dL_dC, const om_grads* g, RayParams* rp) {
    int rc = check_rays(scene, o, d, n);
    if (rc != OM_OK) return rc;
    if ((rc = validate_params(p, rp)) != OM_OK) return rc;
    if (scene->desc.dtype == OM_U8 || scene->desc.block_shift > 0)
        return fail(OM_ERR_UNSUPPORTED, "8-bit and sparse-block scenes are render-only");
    if (!saved || !g) return fail(OM_ERR_INVALID, "saved / grads struct is NULL");
    if (n == 0) return OM_OK;
    if (!saved->F || !saved->T || !saved->n_eval) return fail(OM_ERR_INVALID, "saved F, T and n_eval are required");
    if (saved->batch_wv && ((uintptr_t)saved->batch_wv & 3u))
        return fail(OM_ERR_INVALID, "batch_wv must be 4-byte aligned");
    if (!dL_dC) return fail(OM_ERR_INVALID, "dL_dC is NULL");
    if (!g->grid || !g->plane_xy || !g->plane_xz || !g->plane_yz || !g->mlp)
        return fail(OM_ERR_INVALID, "all gradient buffers are required");
    return OM_OK;
}

// MLP backward into G8 (per-ray dL/dF and background term), then the march
// backward that reads it.  `ws` is the backward workspace
// (om_render_backward_workspace_size(n) bytes, 256-byte aligned).
hipError_t backward_launch(const om_scene* scene, const RayParams& rp, const float* o, const float* d, int64_t n,
                           const float* F, const float* T, const int32_t* n_eval, const float* batch_wv,
                           const float* dC, const float* dF, void* ws, const om_grads* g, hipStream_t s) {
    char* p = static_cast<char*>(ws);
    float* G8 = reinterpret_cast<float*>(p);
    int32_t* order = reinterpret_cast<int32_t*>(p + (n * 8 * (int64_t)sizeof(float) + 255) / 256 * 256);
    int* sched = reinterpret_cast<int*>(reinterpret_cast<char*>(order) +
                                        (n * (int64_t)sizeof(int32_t) + 255) / 256 * 256);
    hipError_t e = launch_mlp_bwd(scene->dev.mlp, scene->dev.mlp_in, rp, F, d, n_eval, dC, dF, n, G8, g->mlp, s);
    if (e != hipSuccess) return e;
    return launch_march_bwd(scene->dev, scene->desc.dtype == OM_BF16, rp, o, d, n, T, n_eval, batch_wv, G8, order,
                            sched, g->grid, g->plane_xy, g->plane_xz, g->plane_yz, g->occ, s);
}

}  // namespace

int om_render_backward(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                       const om_fwd_out* saved, const float* dL_dC, void* workspace, int64_t workspace_bytes,
                       const om_grads* g, void* stream) {
    return om_render_backward_ex(scene, o, d, n, p, saved, dL_dC, nullptr, workspace, workspace_bytes, g, stream);
}

int om_render_backward_ex(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                          const om_fwd_out* saved, const float* dL_dC, const float* dL_dF, void* workspace,
                          int64_t workspace_bytes, const om_grads* g, void* stream) {
    RayParams rp;
    int rc = check_backward(scene, o, d, n, p, saved, dL_dC, g, &rp);
    if (rc != OM_OK) return rc;
    if (n == 0) return ok();
    const int64_t need = om_render_backward_workspace_size(n);
    if (!workspace || ((uintptr_t)workspace & 255u)) return fail(OM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < need)
        return fail(OM_ERR_INVALID, "workspace holds %lld bytes, %lld needed", (long long)workspace_bytes,
                    (long long)need);
    const hipError_t e = backward_launch(scene, rp, o, d, n, saved->F, saved->T, saved->n_eval, saved->batch_wv, dL_dC,
                                         dL_dF, workspace, g, (hipStream_t)stream);
    return hip_status(e, "om_render_backward");
}

int64_t om_render_fwd_bwd_l2_workspace_size(int64_t n, const om_params* p) {
    RayParams rp;
    if (n < 0) {
        fail(OM_ERR_INVALID, "n must be >= 0");
        return -1;
    }
    if (validate_params(p, &rp) != OM_OK) return -1;
    const int64_t slots = (p->n_max + kGroup - 1) / kGroup;
    const int64_t dc = (n * 3 * (int64_t)sizeof(float) + 255) / 256 * 256;
    return dc + om_render_backward_workspace_size(n) + n * slots * 7 * (int64_t)sizeof(float);
}

// Workspace of om_render_fwd_bwd_l2_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress returns for the current
// device, looked up once per device on the entry point's first call there.
constexpr int64_t kNoAllocScratchBytes = 64ll << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// Validation shared by the fused L2 step and its no-alloc variant.
int check_fwd_bwd_l2(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                     const float* target, const om_fwd_out* out, const om_grads* g, RayParams* rp) {
    int rc = check_fwd(scene, o, d, n, p, out, true, true, rp);
    if (rc != OM_OK) return rc;
    if (scene->desc.dtype == OM_U8 || scene->desc.block_shift > 0)
        return fail(OM_ERR_UNSUPPORTED, "8-bit and sparse-block scenes are render-only");
    if (n == 0) return OM_OK;
    if (!target || !g) return fail(OM_ERR_INVALID, "target / grads is NULL");
    if (!g->grid || !g->plane_xy || !g->plane_xz || !g->plane_yz || !g->mlp)
        return fail(OM_ERR_INVALID, "all gradient buffers are required");
    return OM_OK;
}

// The step itself over a workspace laid out as [dL/dC, 256-byte aligned |
// the backward's workspace (om_render_backward_workspace_size: per-ray dL/dF
// and background term, ray order, scheduling words) | per-batch sums of
// w v]: forward with per-batch sums, loss gradient, MLP backward, march
// backward.
int fwd_bwd_l2_launch(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                      const RayParams& rp, const float* target, const om_fwd_out* out, void* workspace, float* loss,
                      const om_grads* g, hipStream_t s, const char* who) {
    char* base = static_cast<char*>(workspace);
    float* dC = reinterpret_cast<float*>(base);
    char* bws = base + (n * 3 * (int64_t)sizeof(float) + 255) / 256 * 256;
    float* bw = reinterpret_cast<float*>(bws + om_render_backward_workspace_size(n));
    hipError_t e = launch_march_fwd(scene->dev, scene->desc.dtype, rp, o, d, n, out->F, out->T, out->n_placed,
                                    out->n_eval, bw, s);
    if (e != hipSuccess) return hip_status(e, who);
    e = launch_mlp(scene->dev.mlp, scene->dev.mlp_in, mlp_in_bf16(scene, p), rp, d, n, out->F, out->T, out->n_eval, out->C, s);
    if (e != hipSuccess) return hip_status(e, who);
    e = launch_l2(out->C, target, n, dC, loss, s);
    if (e != hipSuccess) return hip_status(e, who);
    e = backward_launch(scene, rp, o, d, n, out->F, out->T, out->n_eval, bw, dC, nullptr, bws, g, s);
    return hip_status(e, who);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(void** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "om_render_fwd_bwd_l2_noalloc (hipGetDevice)");
    if (dev < 0 || dev >= kMaxDevices) return fail(OM_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "om_render_fwd_bwd_l2_noalloc (hipGetSymbolAddress)");
        if (!p) return fail(OM_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return OM_OK;
}

}  // namespace

int om_render_fwd_bwd_l2(const om_scene* scene, const float* o, const float* d, int64_t n, const om_params* p,
                         const float* target, const om_fwd_out* out, void* workspace, int64_t workspace_bytes,
                         float* loss, const om_grads* g, void* stream) {
    RayParams rp;
    int rc = check_fwd_bwd_l2(scene, o, d, n, p, target, out, g, &rp);
    if (rc != OM_OK) return rc;
    if (n == 0) return ok();
    const int64_t need = om_render_fwd_bwd_l2_workspace_size(n, p);
    if (!workspace || ((uintptr_t)workspace & 255u)) return fail(OM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < need)
        return fail(OM_ERR_INVALID, "workspace holds %lld bytes, %lld needed", (long long)workspace_bytes,
                    (long long)need);
    return fwd_bwd_l2_launch(scene, o, d, n, p, rp, target, out, workspace, loss, g, (hipStream_t)stream,
                             "om_render_fwd_bwd_l2");
}

int64_t om_render_fwd_bwd_l2_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int om_render_fwd_bwd_l2_noalloc(const om_scene* scene, const float* o, const float* d, int64_t n,
                                 const om_params* p, const float* target, const om_fwd_out* out, float* loss,
                                 const om_grads* g, void* stream) {
    RayParams rp;
    int rc = check_fwd_bwd_l2(scene, o, d, n, p, target, out, g, &rp);
    if (rc != OM_OK) return rc;
    if (n == 0) return ok();
    const int64_t need = om_render_fwd_bwd_l2_workspace_size(n, p);
    if (need > kNoAllocScratchBytes)
        return fail(OM_ERR_UNSUPPORTED,
                    "om_render_fwd_bwd_l2_noalloc: %lld rays at n_max %d need %lld bytes of workspace, above the "
                    "library's fixed %lld; use om_render_fwd_bwd_l2 with a caller workspace",
                    (long long)n, p->n_max, (long long)need, (long long)kNoAllocScratchBytes);
    void* ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc != OM_OK) return rc;
    return fwd_bwd_l2_launch(scene, o, d, n, p, rp, target, out, ws, loss, g, (hipStream_t)stream,
                             "om_render_fwd_bwd_l2_noalloc");
}

int om_smooth_loss(const om_scene* scene, const float* F, const float* d, int64_t n, const float* perturb, int32_t P,
                   float weight, float* loss, float* dL_dF, float* grad_mlp, void* stream) {
    if (!scene) return fail(OM_ERR_INVALID, "scene is NULL");
    if (n < 0) return fail(OM_ERR_INVALID, "n must be >= 0");
    if (P < 1 || P > 64) return fail(OM_ERR_INVALID, "P must be in 1 .. 64");
    if (!std::isfinite(weight)) return fail(OM_ERR_INVALID, "weight must be finite");
    if (n > 0 && (!F || !d || !perturb)) return fail(OM_ERR_INVALID, "F, d and perturb are required");
    if (!loss && !dL_dF && !grad_mlp) return ok();
    if (n == 0 && !loss) return ok();
    return hip_status(launch_smooth(scene->dev.mlp, scene->dev.mlp_in, F, d, n, perturb, P, weight, loss, dL_dF,
                                    grad_mlp, (hipStream_t)stream),
                      "om_smooth_loss");
}

int om_occ_interval_loss(const float* occ, int64_t cells, float weight, float* loss, float* grad_occ,
                         void* stream) {
    if (cells <= 0) return fail(OM_ERR_INVALID, "cells must be > 0");
    if (!occ) return fail(OM_ERR_INVALID, "occ is NULL");
    if (!std::isfinite(weight)) return fail(OM_ERR_INVALID, "weight must be finite");
    if (!loss && !grad_occ) return ok();
    return hip_status(launch_occ_loss(occ, cells, weight, loss, grad_occ, (hipStream_t)stream),
                      "om_occ_interval_loss");
}

int om_feature_range(const float* x, int64_t n, float* minmax, void* stream) {
    if (n <= 0) return fail(OM_ERR_INVALID, "n must be > 0");
    if (!x || !minmax) return fail(OM_ERR_INVALID, "NULL pointer");
    if (((uintptr_t)x & 15u) || ((uintptr_t)minmax & 3u))
        return fail(OM_ERR_INVALID, "x must be 16-byte and minmax 4-byte aligned");
    const char* xb = reinterpret_cast<const char*>(x);
    const char* mb = reinterpret_cast<const char*>(minmax);
    if (mb + 64 > xb && mb < xb + n * 32) return fail(OM_ERR_INVALID, "minmax must not alias x");
    return hip_status(launch_range(x, n, minmax, reinterpret_cast<uint32_t*>(minmax), (hipStream_t)stream),
                      "om_feature_range");
}

int om_quant_params(const float* minmax_host, float* lo, float* step) {
    if (!minmax_host || !lo || !step) return fail(OM_ERR_INVALID, "NULL pointer");
    for (int c = 0; c < 8; ++c) {
        const float mn = minmax_host[2 * c], mx = minmax_host[2 * c + 1];
        if (!std::isfinite(mn) || !std::isfinite(mx) || mx < mn)
            return fail(OM_ERR_INVALID, "channel %d: need finite min <= max", c);
    }
    for (int c = 0; c < 8; ++c) {
        const float mn = minmax_host[2 * c], mx = minmax_host[2 * c + 1];
        const float span = mx - mn;  // binary32 arithmetic, as the codes are decided in it
        lo[c] = mn;
        step[c] = span / 255.0f;
        if (!std::isfinite(step[c])) return fail(OM_ERR_UNSUPPORTED, "channel %d: range overflows float32", c);
    }
    return ok();
}

int om_quantize_u8(const float* x, int64_t n, const float* lo, const float* step, uint8_t* out, void* stream) {
    if (n <= 0) return fail(OM_ERR_INVALID, "n must be > 0");
    if (!x || !lo || !step || !out) return fail(OM_ERR_INVALID, "NULL pointer");
    if (((uintptr_t)x & 15u) || ((uintptr_t)out & 7u))
        return fail(OM_ERR_INVALID, "x must be 16-byte and out 8-byte aligned");
    float inv[8];
    for (int c = 0; c < 8; ++c) {
        if (!std::isfinite(lo[c]) || !std::isfinite(step[c]) || step[c] < 0.0f)
            return fail(OM_ERR_INVALID, "lo / step must be finite with step >= 0");
        inv[c] = step[c] > 0.0f ? 1.0f / step[c] : 0.0f;
        if (!std::isfinite(inv[c])) return fail(OM_ERR_UNSUPPORTED, "step %g too small to invert in float32", step[c]);
    }
    return hip_status(launch_quantize(x, n, lo, inv, out, (hipStream_t)stream), "om_quantize_u8");
}

namespace {
int sparse_dims(const om_scene* scene, int block_shift, int* bn) {
    if (!scene) return fail(OM_ERR_INVALID, "scene is NULL");
    if (block_shift < 1 || block_shift > 5) return fail(OM_ERR_INVALID, "block_shift must be in 1 .. 5");
    if (scene->desc.block_shift > 0) return fail(OM_ERR_INVALID, "the scene's grid is already sparse");
    const int B = 1 << block_shift;
    for (int a = 0; a < 3; ++a) bn[a] = (scene->desc.grid_dims[a] - 2) / B + 1;
    return OM_OK;
}
}  // namespace

int64_t om_sparse_grid_index(const om_scene* scene, int block_shift, int32_t* grid_blocks, int64_t idx_len,
                             void* stream) {
    int bn[3];
    if (sparse_dims(scene, block_shift, bn) != OM_OK) return -1;
    const int64_t n = (int64_t)bn[0] * bn[1] * bn[2];
    if (!grid_blocks || idx_len != n) {
        fail(OM_ERR_INVALID, "grid_blocks must hold %lld entries", (long long)n);
        return -1;
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_blocks_mark(scene->dev, block_shift, bn[0], bn[1], bn[2], grid_blocks, s);
    std::vector<int32_t> mark((size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(mark.data(), grid_blocks, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hip_status(e, "om_sparse_grid_index");
        return -1;
    }
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) mark[(size_t)i] = mark[(size_t)i] ? (int32_t)(++kept) : 0;
    e = hipMemcpyAsync(grid_blocks, mark.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hip_status(e, "om_sparse_grid_index");
        return -1;
    }
    ok();
    return kept;
}

int om_sparse_grid_fill(const om_scene* scene, int block_shift, const int32_t* grid_blocks, int64_t n_blocks,
                        void* atlas, void* stream) {
    int bn[3];
    int rc = sparse_dims(scene, block_shift, bn);
    if (rc != OM_OK) return rc;
    if (!grid_blocks || !atlas || ((uintptr_t)atlas & 15u))
        return fail(OM_ERR_INVALID, "grid_blocks and a 16-byte aligned atlas are required");
    const int64_t E = ((int64_t)1 << block_shift) + 1;
    if (n_blocks < 0 || (n_blocks + 1) * E * E * E >= ((int64_t)1 << 31))
        return fail(OM_ERR_UNSUPPORTED, "n_blocks must be >= 0 with (n_blocks + 1) (B + 1)^3 < 2^31");
    const int units = scene->desc.dtype == OM_F32 ? 4 : scene->desc.dtype == OM_BF16 ? 2 : 1;
    return hip_status(launch_blocks_fill(scene->dev, block_shift, bn[0], bn[1], bn[2], grid_blocks, n_blocks, units,
                                         atlas, (hipStream_t)stream),
                      "om_sparse_grid_fill");
}

int om_cast_bf16(const float* src, int64_t n, uint16_t* dst, void* stream) {
    if (n < 0) return fail(OM_ERR_INVALID, "n must be >= 0");
    if (n == 0) return ok();
    if (!src || !dst) return fail(OM_ERR_INVALID, "NULL pointer");
    if (((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
        return fail(OM_ERR_INVALID, "src and dst must be 16-byte aligned");
    const char* sb = reinterpret_cast<const char*>(src);
    const char* db = reinterpret_cast<const char*>(dst);
    if (db < sb + n * 4 && sb < db + n * 2) return fail(OM_ERR_INVALID, "dst must not overlap src");
    return hip_status(launch_cast_bf16(src, n, dst, (hipStream_t)stream), "om_cast_bf16");
}

namespace {
static int64_t order_keys_offset() { return (order_hist_bytes() + 255) / 256 * 256; }
}  // namespace

int64_t om_order_rays_workspace_size(int64_t n) {
    if (n < 0 || n > INT32_MAX) {
        fail(OM_ERR_INVALID, "n must lie in [0, 2^31 - 1]");
        return -1;
    }
    // The key histogram, then one 16-bit key per ray.  No rays, no work.
    if (n == 0) return 0;
    return order_keys_offset() + (n * (int64_t)sizeof(uint16_t) + 255) / 256 * 256;
}

int om_order_rays(const om_scene* scene, const float* o, const float* d, int64_t n, int32_t* order, float* o_sorted,
                  float* d_sorted, void* workspace, int64_t workspace_bytes, void* stream) {
    if (!scene) return fail(OM_ERR_INVALID, "NULL scene");
    if (n < 0 || n > INT32_MAX) return fail(OM_ERR_INVALID, "n must lie in [0, 2^31 - 1]");
    if (n == 0) return ok();
    if (!o || !d || !order || !o_sorted || !d_sorted || !workspace) return fail(OM_ERR_INVALID, "NULL pointer");
    if ((uintptr_t)workspace & 255u) return fail(OM_ERR_INVALID, "workspace must be 256-byte aligned");
    const int64_t need = om_order_rays_workspace_size(n);
    if (workspace_bytes < need)
        return fail(OM_ERR_INVALID, "workspace of %lld bytes, %lld needed", (long long)workspace_bytes, (long long)need);
    const char* ob = reinterpret_cast<const char*>(o);
    const char* db = reinterpret_cast<const char*>(d);
    const int64_t rb = n * 3 * (int64_t)sizeof(float);
    for (const float* w : {(const float*)o_sorted, (const float*)d_sorted}) {
        const char* wb = reinterpret_cast<const char*>(w);
        if ((wb < ob + rb && ob < wb + rb) || (wb < db + rb && db < wb + rb))
            return fail(OM_ERR_INVALID, "o_sorted and d_sorted must not overlap o or d");
    }
    int* hist = static_cast<int*>(workspace);
    uint16_t* keys = reinterpret_cast<uint16_t*>(static_cast<char*>(workspace) + order_keys_offset());
    return hip_status(launch_order_rays(scene->desc.box_lo, scene->desc.box_hi, o, d, n, order, o_sorted, d_sorted,
                                        hist, keys, (hipStream_t)stream),
                      "om_order_rays");
}

namespace {
static int rows_args(const float* src, int cols, const int32_t* idx, int64_t n, const float* dst, int64_t src_rows,
              int64_t dst_rows) {
    if (n < 0 || n > INT32_MAX) return fail(OM_ERR_INVALID, "n must lie in [0, 2^31 - 1]");
    if (cols < 1 || cols > 64) return fail(OM_ERR_INVALID, "cols must lie in [1, 64]");
    if (src_rows < 0 || dst_rows < 0) return fail(OM_ERR_INVALID, "row counts must be >= 0");
    if (n > 0 && (!src || !idx || !dst)) return fail(OM_ERR_INVALID, "NULL pointer");
    const char* sb = reinterpret_cast<const char*>(src);
    const char* db = reinterpret_cast<const char*>(dst);
    const int64_t s_bytes = src_rows * cols * (int64_t)sizeof(float), d_bytes = dst_rows * cols * (int64_t)sizeof(float);
    if (n > 0 && db < sb + s_bytes && sb < db + d_bytes) return fail(OM_ERR_INVALID, "dst must not overlap src");
    return OM_OK;
}
}  // namespace

int om_gather_rows(const float* src, int64_t src_rows, int cols, const int32_t* idx, int64_t n, float* dst,
                   void* stream) {
    const int st = rows_args(src, cols, idx, n, dst, src_rows, n);
    if (st != OM_OK || n == 0) return st == OM_OK ? ok() : st;
    return hip_status(launch_rows_gather(src, src_rows, cols, idx, n, dst, (hipStream_t)stream), "om_gather_rows");
}

int om_scatter_rows(const float* src, int cols, const int32_t* idx, int64_t n, float* dst, int64_t dst_rows,
                    void* stream) {
    const int st = rows_args(src, cols, idx, n, dst, n, dst_rows);
    if (st != OM_OK || n == 0) return st == OM_OK ? ok() : st;
    return hip_status(launch_rows_scatter(src, cols, idx, n, dst, dst_rows, (hipStream_t)stream), "om_scatter_rows");
}

int om_l2_loss_fp64(const float* C, const float* target, int64_t n, double* out, void* stream) {
    if (n <= 0) return fail(OM_ERR_INVALID, "n must be > 0");
    if (!C || !target || !out) return fail(OM_ERR_INVALID, "NULL pointer");
    return hip_status(launch_l2_fp64(C, target, n, out, (hipStream_t)stream), "om_l2_loss_fp64");
}

int om_l2_loss_grad(const float* C, const float* target, int64_t n, float* dL_dC, float* loss_out, void* stream) {
    if (n <= 0) return fail(OM_ERR_INVALID, "n must be > 0");
    if (!C || !target || !dL_dC) return fail(OM_ERR_INVALID, "NULL pointer");
    if (dL_dC == C || dL_dC == target) return fail(OM_ERR_INVALID, "dL_dC must not alias C or target");
    return hip_status(launch_l2(C, target, n, dL_dC, loss_out, (hipStream_t)stream), "om_l2_loss_grad");
}

const char* om_last_error(void) { return g_err.c_str(); }

const char* om_status_str(int status) {
    switch (status) {
        case OM_OK: return "ok";
        case OM_ERR_INVALID: return "invalid argument";
        case OM_ERR_UNSUPPORTED: return "unsupported shape or dtype";
        case OM_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

int om_version(void) { return 110; }

}  // extern "C"
