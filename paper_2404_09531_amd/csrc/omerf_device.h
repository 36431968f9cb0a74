// omerf_device.h -- device-side building blocks of the gfx950 ray marcher.
//
// Work decomposition: one ray per GROUP of 16 lanes (a DPP row of a
// wave64), four rays per wavefront.  A group tests 16 consecutive lattice
// candidates at once, compacts the accepted ones through a small per-group
// LDS queue (ballot + prefix popcount), then shades full batches of 16
// samples: one sample per lane, a 16-lane inclusive scan of the optical
// depth gives each lane its transmittance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omerf {

constexpr int kGroup = 16;            // lanes per ray
constexpr int kBlock = 256;           // threads per block (4 waves)
constexpr int kGroupsPerBlock = kBlock / kGroup;
constexpr int kQueue = 2 * kGroup;    // per-group LDS queue capacity
constexpr int kKCap = 1 << 24;        // lattice indices k in [0, 2^24)
constexpr int kMaxMipLevels = 8;      // occupancy pyramid levels above the plane

// Vertex-aligned coordinate along one axis: u = p * s + (ci + cf) with
// s = (n - 1) / (hi - lo) a power-of-two scaling of an integer, ci integer,
// cf in [0, 1).  n = number of vertices / texels on the axis.
struct AxisMap {
    float s;
    float cf;
    int ci;
    int n;
};

struct SceneDev {
    const void* grid;   // [Lz][Ly][Lx][8]
    const void* pxy;    // [Ny][Nx][8]
    const void* pxz;    // [Nz][Nx][8]
    const void* pyz;    // [Nz][Ny][8]
    const float2* occ;  // [My][Mx] (z_min, z_max)
    const float* mlp;   // packed 499
    int Lx, Ly, Lz, Nx, Ny, Nz, Mx, My;
    float lo0, lo1, lo2, hi0, hi1, hi2;
    float occ_sx, occ_sy, occ_ox, occ_oy;  // cell = floor(p * s) - o
    AxisMap gx, gy, gz, px, py, pz;
    // Optional occupancy pyramid: levels l = 1..mip_levels one after the
    // other, (My >> l) x (Mx >> l) blocks of 2^l x 2^l cells each holding
    // (min z_min, max z_max) over its non-empty cells; level l starts at
    // entry (Mx My - (Mx >> (l-1)) (My >> (l-1))) / 3 (a geometric sum).
    const float2* mips;
    int mip_levels;
    int mlp_in;  // deferred-MLP input width: 10 or 34
    // 8-bit storage: channel c of source s (grid, XY, XZ, YZ) decodes as
    // qlo[8 s + c] + q qstep[8 s + c]; indexed with constants only.
    float qlo[32], qstep[32];
    // Grid row strides in vertices: (Lx, Lx Ly) for the dense grid,
    // (B + 1, (B + 1)^2) inside a sparse block.
    uint32_t gsy, gsz;
    // Sparse voxel blocks (blk_shift > 0): the grid is an atlas of
    // (B + 1)^3-vertex blocks (B = 2^blk_shift cells per edge, one vertex
    // of overlap so a cell never straddles blocks); blk_idx[bz][by][bx]
    // names the block of each B^3 cell region, 0 being an all-zero block.
    const int32_t* blk_idx;
    int blk_shift, bnx, bny;
    uint32_t blk_verts, n_blocks;
};

struct RayParams {
    float delta;
    int n_max;
    float t_term;
    float bg0, bg1, bg2;
    float occ_inv_eps;  // 1 / epsilon of the soft occupancy value (Eq. 6); 0: hard interval
};

// Deferred MLP of Eq. 4, NIN -> 16 -> 16 -> 3, packed [W1 (16 x NIN), b1,
// W2 (16 x 16), b2, W3 (3 x 16), b3], weights row-major (out, in).  NIN is
// 10 (7 features + the raw view direction) or 34 (the direction with four
// sine/cosine frequencies).
template <int NIN>
struct MlpLayout {
    static constexpr int W1 = 0, B1 = 16 * NIN, W2 = B1 + 16, B2 = W2 + 256, W3 = B2 + 16, B3 = W3 + 48;
    static constexpr int SIZE = B3 + 3;
};
constexpr int kMlpMaxSize = MlpLayout<34>::SIZE;  // 883

// ---------------------------------------------------------------------------
// Lattice point and placement predicate (Sec. 4.1 Eq. 6-7 at epsilon = 0).
// p = fl32(o + fl32(t_k * d)) with two roundings: contraction into an FMA is
// switched off here so the discrete decision matches the binary32 definition.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 lattice_point(int k, float3 o, float3 d, float delta) {
#pragma clang fp contract(off)
    const float t = (float)k * delta;  // exact: k < 2^24, delta a power of two
    float3 p;
    p.x = o.x + t * d.x;
    p.y = o.y + t * d.y;
    p.z = o.z + t * d.z;
    return p;
}

__device__ __forceinline__ bool accept_point(const SceneDev& sc, float3 p) {
    const bool inb = p.x >= sc.lo0 && p.x <= sc.hi0 && p.y >= sc.lo1 && p.y <= sc.hi1 &&
                     p.z >= sc.lo2 && p.z <= sc.hi2;
    // p * s is exact (s a power of two); fmaxf maps NaN to 0, so the index
    // is always in range.
    const float fi = fminf(fmaxf(floorf(p.x * sc.occ_sx) - sc.occ_ox, 0.0f), (float)(sc.Mx - 1));
    const float fj = fminf(fmaxf(floorf(p.y * sc.occ_sy) - sc.occ_oy, 0.0f), (float)(sc.My - 1));
    const float2 z = sc.occ[(int)fj * sc.Mx + (int)fi];
    return inb && p.z >= z.x && p.z <= z.y;
}

// Empty-space skipping over occupancy columns (the bounding-box jump of
// Sec. 4.4), at pyramid level lv (0 = the occupancy plane itself): may any
// lattice sample k in [ka, ka + len - 1] be accepted?  The binary32 points
// of those samples lie within the segment between the two end points padded
// by eps (rounding is bounded by 2^-22 of the coordinate magnitudes; eps is
// 2^-20 of them), so the segment may hold an accepted sample only if its
// padded box meets the scene box and some level-lv block it overlaps has an
// interval [z_min, z_max] meeting its padded z range.  A block's interval
// contains those of all its cells, and the containing-cell map is monotone,
// so the overlapped blocks are those of the padded x and y bounds.  More
// than 3 x 3 blocks: answer "maybe".
__device__ __forceinline__ bool column_maybe(const SceneDev& sc, float3 o, float3 d, float delta, int ka, int len,
                                             int lv) {
    const float ta = (float)ka * delta, tb = (float)(ka + len - 1) * delta;
    const float xa = o.x + ta * d.x, xb = o.x + tb * d.x;
    const float ya = o.y + ta * d.y, yb = o.y + tb * d.y;
    const float za = o.z + ta * d.z, zb = o.z + tb * d.z;
    const float ex = ldexpf(1.0f + fabsf(o.x) + fabsf(tb * d.x), -20);
    const float ey = ldexpf(1.0f + fabsf(o.y) + fabsf(tb * d.y), -20);
    const float ez = ldexpf(1.0f + fabsf(o.z) + fabsf(tb * d.z), -20);
    const float x0 = fminf(xa, xb) - ex, x1 = fmaxf(xa, xb) + ex;
    const float y0 = fminf(ya, yb) - ey, y1 = fmaxf(ya, yb) + ey;
    const float z0 = fminf(za, zb) - ez, z1 = fmaxf(za, zb) + ez;
    if (x1 < sc.lo0 || x0 > sc.hi0 || y1 < sc.lo1 || y0 > sc.hi1 || z1 < sc.lo2 || z0 > sc.hi2) return false;
    const float mx = (float)(sc.Mx - 1), my = (float)(sc.My - 1);
    const int i0 = (int)fminf(fmaxf(floorf(x0 * sc.occ_sx) - sc.occ_ox, 0.0f), mx) >> lv;
    const int i1 = (int)fminf(fmaxf(floorf(x1 * sc.occ_sx) - sc.occ_ox, 0.0f), mx) >> lv;
    const int j0 = (int)fminf(fmaxf(floorf(y0 * sc.occ_sy) - sc.occ_oy, 0.0f), my) >> lv;
    const int j1 = (int)fminf(fmaxf(floorf(y1 * sc.occ_sy) - sc.occ_oy, 0.0f), my) >> lv;
    if (i1 - i0 > 2 || j1 - j0 > 2) return true;
    const float2* z_of =
        lv == 0 ? sc.occ : sc.mips + (sc.Mx * sc.My - (sc.Mx >> (lv - 1)) * (sc.My >> (lv - 1))) / 3;
    const int w = sc.Mx >> lv;
    bool maybe = false;
    for (int j = j0; j <= j1; ++j)
        for (int i = i0; i <= i1; ++i) {
            const float2 z = z_of[j * w + i];
            maybe |= (z.x <= z1) && (z.y >= z0) && (z.x <= z.y);
        }
    return maybe;
}

// Soft occupancy value of Eq. 6 (q = 2) at a placed sample p, read at the
// cell containing p's xy (Eq. 7), in the form min(rise^2, fall^2) with
// rise = clamp((z - z_min) / eps, 0, 1) and fall = clamp((z_max - z) / eps,
// 0, 1), which equals the four cases of Eq. 6 whenever z_max - z_min >= 2 eps
// and stays continuous when the buffer zones overlap.  Also returns
// dM/dz_min and dM/dz_max, with the conventions of a float64 autograd of
// that expression: a clamp passes the derivative on its closed range, and a
// tie of the minimum splits it between the two sides.
struct OccValue {
    float m, dzmin, dzmax;
    int cell;
};

__device__ __forceinline__ OccValue occ_value(const SceneDev& sc, float3 p, float inv_eps) {
    const float fi = fminf(fmaxf(floorf(p.x * sc.occ_sx) - sc.occ_ox, 0.0f), (float)(sc.Mx - 1));
    const float fj = fminf(fmaxf(floorf(p.y * sc.occ_sy) - sc.occ_oy, 0.0f), (float)(sc.My - 1));
    OccValue v;
    v.cell = (int)fj * sc.Mx + (int)fi;
    const float2 z = sc.occ[v.cell];
    const float ur = (p.z - z.x) * inv_eps, uf = (z.y - p.z) * inv_eps;
    const float r = fminf(fmaxf(ur, 0.0f), 1.0f), f = fminf(fmaxf(uf, 0.0f), 1.0f);
    const float mr = r * r, mf = f * f;
    v.m = fminf(mr, mf);
    const float sr = mr < mf ? 1.0f : (mr == mf ? 0.5f : 0.0f);
    const float dr = (ur >= 0.0f && ur <= 1.0f) ? 2.0f * r * inv_eps : 0.0f;
    const float df = (uf >= 0.0f && uf <= 1.0f) ? 2.0f * f * inv_eps : 0.0f;
    v.dzmin = -sr * dr;
    v.dzmax = (1.0f - sr) * df;
    return v;
}

// Conservative candidate range [k_lo, k_hi] for the closed box: every k whose
// binary32 point lies in the box is inside it (the exact predicate is applied
// to each candidate afterwards).  Rounding of p is bounded by 2^-22 of the
// magnitudes involved; the slab bounds are widened by 2^-20 of them and the
// t range by a relative 2^-20 plus two lattice steps.
struct KRange {
    int lo, hi;
};

__device__ __forceinline__ void slab(float oa, float da, float lo, float hi, float& t0, float& t1, bool& empty) {
    if (da == 0.0f) {
        if (oa < lo || oa > hi) empty = true;
        return;
    }
    const float eps = ldexpf(fabsf(oa) + fmaxf(fabsf(lo), fabsf(hi)) + 1.0f, -20);
    const float inv = 1.0f / da;
    float a = (lo - eps - oa) * inv;
    float b = (hi + eps - oa) * inv;
    if (da < 0.0f) {
        const float s = a;
        a = b;
        b = s;
    }
    t0 = fmaxf(t0, a);
    t1 = fminf(t1, b);
}

__device__ __forceinline__ KRange candidate_range(const SceneDev& sc, float3 o, float3 d, float delta) {
    KRange r{0, -1};
    const bool finite = isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(d.x) &&
                        isfinite(d.y) && isfinite(d.z);
    if (!finite) return r;
    float t0 = 0.0f, t1 = (float)kKCap * delta;
    bool empty = false;
    slab(o.x, d.x, sc.lo0, sc.hi0, t0, t1, empty);
    slab(o.y, d.y, sc.lo1, sc.hi1, t0, t1, empty);
    slab(o.z, d.z, sc.lo2, sc.hi2, t0, t1, empty);
    if (empty) return r;
    t0 = t0 - fabsf(t0) * 0x1p-20f - 2.0f * delta;
    t1 = t1 + fabsf(t1) * 0x1p-20f + 2.0f * delta;
    if (!(t0 <= t1)) return r;
    const float kmax = (float)(kKCap - 1);
    const float klo = fminf(fmaxf(floorf(t0 / delta), 0.0f), kmax);
    const float khi = fminf(fmaxf(ceilf(t1 / delta), -1.0f), kmax);
    r.lo = (int)klo;
    r.hi = (int)khi;
    return r;
}

// ---------------------------------------------------------------------------
// Interpolation coordinates, with the fractional part kept to ~1e-7 absolute
// even on 4096-texel axes: the product p * s is split into its rounded value
// and the exact FMA remainder before the integer part is removed.  Automatic
// contraction is off here: fusing p * s into (hi - floor(hi)) would count the
// remainder twice.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void axis_coord(float p, const AxisMap& m, int& i0, float& f) {
#pragma clang fp contract(off)
    const float hi = p * m.s;
    const float lo = __builtin_fmaf(p, m.s, -hi);
    const float ih = floorf(hi);
    const float fr = ((hi - ih) + m.cf) + lo;
    const float fl = floorf(fr);
    const int i = (int)ih + m.ci + (int)fl;
    const int ic = min(max(i, 0), m.n - 2);
    f = (fr - fl) + (float)(i - ic);
    i0 = ic;
}

// Storage policies.  A corner is 8 channels: two 16-byte loads (float32) or
// one (bfloat16).  load() only issues the loads; acc() consumes them, so a
// whole source's corners can be in flight before the first is used.
struct F32Store {
    struct Row {
        float4 a, b;
    };
    static __device__ __forceinline__ Row load(const void* base, uint32_t idx) {
        const float4* q = reinterpret_cast<const float4*>(base) + (size_t)idx * 2;
        return Row{q[0], q[1]};
    }
    static __device__ __forceinline__ void acc(const Row& r, float w, float* t) {
        t[0] += w * r.a.x; t[1] += w * r.a.y; t[2] += w * r.a.z; t[3] += w * r.a.w;
        t[4] += w * r.b.x; t[5] += w * r.b.y; t[6] += w * r.b.z; t[7] += w * r.b.w;
    }
};

struct BF16Store {
    typedef uint4 Row;
    static __device__ __forceinline__ float lo16(uint32_t v) { return __uint_as_float(v << 16); }
    static __device__ __forceinline__ float hi16(uint32_t v) { return __uint_as_float(v & 0xffff0000u); }
    static __device__ __forceinline__ Row load(const void* base, uint32_t idx) {
        return reinterpret_cast<const uint4*>(base)[idx];
    }
    static __device__ __forceinline__ void acc(const Row& v, float w, float* t) {
        t[0] += w * lo16(v.x); t[1] += w * hi16(v.x); t[2] += w * lo16(v.y); t[3] += w * hi16(v.y);
        t[4] += w * lo16(v.z); t[5] += w * hi16(v.z); t[6] += w * lo16(v.w); t[7] += w * hi16(v.w);
    }
};

// 8-bit storage (Sec. 4.4): one vertex or texel is 8 bytes, channel c in
// byte c.  Interpolation weights of one source sum to one, so a source adds
// lo + step * sum_corners w q per channel; acc accumulates sum w q.
struct U8Store {
    typedef uint2 Row;
    static __device__ __forceinline__ Row load(const void* base, uint32_t idx) {
        return reinterpret_cast<const uint2*>(base)[idx];
    }
    static __device__ __forceinline__ void acc(const Row& v, float w, float* a) {
        a[0] += w * (float)(v.x & 0xffu);
        a[1] += w * (float)((v.x >> 8) & 0xffu);
        a[2] += w * (float)((v.x >> 16) & 0xffu);
        a[3] += w * (float)(v.x >> 24);
        a[4] += w * (float)(v.y & 0xffu);
        a[5] += w * (float)((v.y >> 8) & 0xffu);
        a[6] += w * (float)((v.y >> 16) & 0xffu);
        a[7] += w * (float)(v.y >> 24);
    }
};

// Corner set of one sample: 8 grid vertices + 3 x 4 plane texels.
struct Corners {
    uint32_t g, xy, xz, yz;  // base vertex / texel indices
    int ix, iy, iz;          // grid base vertex
    int jx, jy, jz;          // plane base texel per axis
    float fx, fy, fz;        // grid fractions
    float ux, uy, uz;        // plane fractions
};

// kSparse: the grid is the atlas of sparse voxel blocks (a separate
// specialisation, so the dense kernels carry no block lookup).
template <bool kSparse = false>
__device__ __forceinline__ Corners corners_of(const SceneDev& sc, float3 p) {
    Corners c;
    axis_coord(p.x, sc.gx, c.ix, c.fx);
    axis_coord(p.y, sc.gy, c.iy, c.fy);
    axis_coord(p.z, sc.gz, c.iz, c.fz);
    axis_coord(p.x, sc.px, c.jx, c.ux);
    axis_coord(p.y, sc.py, c.jy, c.uy);
    axis_coord(p.z, sc.pz, c.jz, c.uz);
    if (kSparse) {
        const int m = (1 << sc.blk_shift) - 1;
        const int32_t id = sc.blk_idx[((c.iz >> sc.blk_shift) * sc.bny + (c.iy >> sc.blk_shift)) * sc.bnx +
                                      (c.ix >> sc.blk_shift)];
        const uint32_t b = min((uint32_t)id, sc.n_blocks);  // a stray id reads a stored block, never past the atlas
        c.g = b * sc.blk_verts + ((uint32_t)(c.iz & m) * sc.gsy + (uint32_t)(c.iy & m)) * sc.gsy + (uint32_t)(c.ix & m);
    } else {
        c.g = ((uint32_t)c.iz * (uint32_t)sc.Ly + (uint32_t)c.iy) * (uint32_t)sc.Lx + (uint32_t)c.ix;
    }
    c.xy = (uint32_t)c.jy * (uint32_t)sc.Nx + (uint32_t)c.jx;
    c.xz = (uint32_t)c.jz * (uint32_t)sc.Nx + (uint32_t)c.jx;
    c.yz = (uint32_t)c.jz * (uint32_t)sc.Ny + (uint32_t)c.jy;
    return c;
}

// Eq. 2: t = trilinear(V) + bilinear(P_xy) + bilinear(P_xz) + bilinear(P_yz),
// one lane per sample, with at most 12 corners in flight (grid first, then
// planes), for kernels that carry more live state than the forward march.
template <class S>
__device__ __forceinline__ void gather_features_split(const SceneDev& sc, const Corners& c, float* t) {
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = 0.0f;
    const uint32_t sy = sc.gsy, sz = sc.gsz;
    const uint32_t nx = (uint32_t)sc.Nx, ny = (uint32_t)sc.Ny;
    // two rows (one pair adjacent along the row axis) in flight for 32-byte
    // rows, four for 16-byte rows
    constexpr int kPerGroup = sizeof(typename S::Row) > 16 ? 1 : 2;
    const float x0 = 1.0f - c.fx, x1 = c.fx, y0 = 1.0f - c.fy, y1 = c.fy, z0 = 1.0f - c.fz, z1 = c.fz;
#pragma unroll
    for (int p0 = 0; p0 < 4; p0 += kPerGroup) {
        typename S::Row r[2 * kPerGroup];
#pragma unroll
        for (int k = 0; k < kPerGroup; ++k) {
            const int p = p0 + k;  // (dy, dz) = (p & 1, p >> 1)
            const uint32_t base = c.g + ((p & 1) ? sy : 0u) + ((p >> 1) ? sz : 0u);
            r[2 * k] = S::load(sc.grid, base);
            r[2 * k + 1] = S::load(sc.grid, base + 1);
        }
#pragma unroll
        for (int k = 0; k < kPerGroup; ++k) {
            const int p = p0 + k;
            const float wyz = ((p & 1) ? y1 : y0) * ((p >> 1) ? z1 : z0);
            S::acc(r[2 * k], x0 * wyz, t);
            S::acc(r[2 * k + 1], x1 * wyz, t);
        }
    }
    const float a0 = 1.0f - c.ux, a1 = c.ux, b0 = 1.0f - c.uy, b1 = c.uy, e0 = 1.0f - c.uz, e1 = c.uz;
#pragma unroll
    for (int p0 = 0; p0 < 6; p0 += kPerGroup) {
        typename S::Row r[2 * kPerGroup];
#pragma unroll
        for (int k = 0; k < kPerGroup; ++k) {
            const int p = p0 + k;  // plane p >> 1, second-axis offset p & 1
            const int q = p >> 1;
            const void* P = q == 0 ? sc.pxy : q == 1 ? sc.pxz : sc.pyz;
            const uint32_t base = (q == 0 ? c.xy : q == 1 ? c.xz : c.yz) + ((p & 1) ? (q == 2 ? ny : nx) : 0u);
            r[2 * k] = S::load(P, base);
            r[2 * k + 1] = S::load(P, base + 1);
        }
#pragma unroll
        for (int k = 0; k < kPerGroup; ++k) {
            const int p = p0 + k;
            const int q = p >> 1;
            const float u0 = q == 2 ? b0 : a0, u1 = q == 2 ? b1 : a1;
            const float v = (p & 1) ? (q == 0 ? b1 : e1) : (q == 0 ? b0 : e0);
            S::acc(r[2 * k], u0 * v, t);
            S::acc(r[2 * k + 1], u1 * v, t);
        }
    }
}

__device__ __forceinline__ float sigmoidf_fast(float x) {
    return __builtin_amdgcn_rcpf(1.0f + __expf(-x));
}

// ---------------------------------------------------------------------------
// 16-lane group collectives.  All lanes of a group take the same branches,
// so group members are always active together.
// ---------------------------------------------------------------------------
// DPP move within a 16-lane row (= one group); out-of-row sources read 0.
template <int CTRL>
__device__ __forceinline__ float dpp_row(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}
constexpr int kRowShr = 0x110, kRowShl = 0x100;

// Inclusive scan over the group: lane i gets x_0 + ... + x_i (row_shr DPP).
__device__ __forceinline__ float g_scan_incl(float x, int /*gl*/) {
    x += dpp_row<kRowShr | 1>(x);
    x += dpp_row<kRowShr | 2>(x);
    x += dpp_row<kRowShr | 4>(x);
    x += dpp_row<kRowShr | 8>(x);
    return x;
}

// Value of the neighbouring lane of the pair (lane ^ 1), via DPP quad_perm.
__device__ __forceinline__ float pair_swap(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xf, 0xf, false));  // [1,0,3,2]
}

template <int CTRL>
__device__ __forceinline__ int dpp_row_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, true);
}


// Value of lane 0 of the lane's quad (DPP quad_perm [0,0,0,0]).
__device__ __forceinline__ float quad_bcast0(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x00, 0xf, 0xf, false));
}

// Value of the next lower lane (0 for lane 0).
__device__ __forceinline__ float g_shift_up1(float x) { return dpp_row<kRowShr | 1>(x); }

// Value of the next higher lane (0 for lane 15).
__device__ __forceinline__ float g_shift_down1(float x) { return dpp_row<kRowShl | 1>(x); }


// Group min / max in every lane: DPP butterflies over the quad, then
// rotations of the 16-lane row by 4 and 8 (no LDS crossbar).
template <class Op>
__device__ __forceinline__ int g_reduce(int x, Op op) {
    x = op(x, __builtin_amdgcn_mov_dpp(x, 0xB1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    x = op(x, __builtin_amdgcn_mov_dpp(x, 0x4E, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    x = op(x, __builtin_amdgcn_mov_dpp(x, 0x124, 0xf, 0xf, false));  // row_ror:4
    x = op(x, __builtin_amdgcn_mov_dpp(x, 0x128, 0xf, 0xf, false));  // row_ror:8
    return x;
}
__device__ __forceinline__ int g_min(int x) {
    return g_reduce(x, [](int a, int b) { return min(a, b); });
}
__device__ __forceinline__ int g_max(int x) {
    return g_reduce(x, [](int a, int b) { return max(a, b); });
}

// Group sum, returned in every lane: scan, then broadcast lane 15.
__device__ __forceinline__ float g_sum(float x) { return __shfl(g_scan_incl(x, 0), kGroup - 1, kGroup); }

__device__ __forceinline__ uint32_t g_ballot(bool pred, int lane) {
    const unsigned long long m = __ballot(pred);
    return (uint32_t)(m >> (lane & (64 - kGroup))) & 0xffffu;
}

// Keeps the compiler from moving LDS accesses across this point; the
// hardware executes one wave's LDS instructions in order.
__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Eq. 2 for 8-bit storage, one lane per sample: the 4 grid corner pairs
// (16 bytes each), then the 2 XY pairs, then the 4 XZ and YZ pairs, each
// group loaded before its weighted code sums are decoded with the source's
// per-channel (lo, step).  Three load groups keep the kernel at 78 VGPRs,
// 6 waves per SIMD (two groups, grid and planes: 86, 5 waves; one group of
// 10: 97, 4 waves).
__device__ __forceinline__ void decode_add(const SceneDev& sc, int src, const float* a, float* t) {
#pragma unroll
    for (int c = 0; c < 8; ++c) t[c] += fmaf(sc.qstep[8 * src + c], a[c], sc.qlo[8 * src + c]);
}

__device__ __forceinline__ void gather_u8(const SceneDev& sc, const Corners& c, float* t) {
    const uint32_t sy = sc.gsy, sz = sc.gsz;
    const uint32_t nx = (uint32_t)sc.Nx, ny = (uint32_t)sc.Ny;
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = 0.0f;
    float a[8];
    {
        uint4 r[4];
        const uint8_t* G = static_cast<const uint8_t*>(sc.grid);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint32_t base = c.g + ((p & 1) ? sy : 0u) + ((p >> 1) ? sz : 0u);
            __builtin_memcpy(&r[p], G + (size_t)base * 8, 16);
        }
        const float x0 = 1.0f - c.fx, x1 = c.fx, y0 = 1.0f - c.fy, y1 = c.fy, z0 = 1.0f - c.fz, z1 = c.fz;
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = 0.0f;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float wyz = ((p & 1) ? y1 : y0) * ((p >> 1) ? z1 : z0);
            U8Store::acc(make_uint2(r[p].x, r[p].y), x0 * wyz, a);
            U8Store::acc(make_uint2(r[p].z, r[p].w), x1 * wyz, a);
        }
        decode_add(sc, 0, a, t);
    }
    const uint8_t* P[3] = {static_cast<const uint8_t*>(sc.pxy), static_cast<const uint8_t*>(sc.pxz),
                           static_cast<const uint8_t*>(sc.pyz)};
    const uint32_t pb[3] = {c.xy, c.xz, c.yz}, ps[3] = {nx, nx, ny};
    const float u0 = 1.0f - c.ux, u1 = c.ux, v0 = 1.0f - c.uy, v1 = c.uy, e0 = 1.0f - c.uz, e1 = c.uz;
    const float wa[3][2] = {{u0, u1}, {u0, u1}, {v0, v1}};  // first axis: x, x, y
    const float wb[3][2] = {{v0, v1}, {e0, e1}, {e0, e1}};  // second axis: y, z, z
#pragma unroll
    for (int g = 0; g < 2; ++g) {  // planes [q0, q1): XY, then XZ and YZ
        const int q0 = g == 0 ? 0 : 1, q1 = g == 0 ? 1 : 3;
        uint4 r[4];
#pragma unroll
        for (int q = q0; q < q1; ++q) {
            __builtin_memcpy(&r[2 * (q - q0)], P[q] + (size_t)pb[q] * 8, 16);
            __builtin_memcpy(&r[1 + 2 * (q - q0)], P[q] + (size_t)(pb[q] + ps[q]) * 8, 16);
        }
#pragma unroll
        for (int q = q0; q < q1; ++q) {
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = 0.0f;
            const uint4 lo = r[2 * (q - q0)], hi = r[1 + 2 * (q - q0)];
            U8Store::acc(make_uint2(lo.x, lo.y), wa[q][0] * wb[q][0], a);
            U8Store::acc(make_uint2(lo.z, lo.w), wa[q][1] * wb[q][0], a);
            U8Store::acc(make_uint2(hi.x, hi.y), wa[q][0] * wb[q][1], a);
            U8Store::acc(make_uint2(hi.z, hi.w), wa[q][1] * wb[q][1], a);
            decode_add(sc, 1 + q, a, t);
        }
    }
}

// Block index -> virtual block index such that the blocks the hardware
// places on one XCD (round-robin over 8 XCDs) cover one contiguous range of
// rays, keeping neighbouring rays in the same L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    const uint32_t per = nb / 8, rem = nb % 8, x = b % 8, i = b / 8;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// ---------------------------------------------------------------------------
// Deferred MLP input, shared by the MLP forward kernels, the MLP backward
// and the view-smoothness loss.
// ---------------------------------------------------------------------------
// x = [F (7), enc(d)]: enc(d) = d, or [d, sin(2^0 d), cos(2^0 d), ...,
// sin(2^3 d), cos(2^3 d)] (each term a 3-vector) for NIN = 34.
template <int NIN>
__device__ __forceinline__ void mlp_input(const float* F7, float3 d, float* x) {
#pragma unroll
    for (int c = 0; c < 7; ++c) x[c] = F7[c];
    x[7] = d.x;
    x[8] = d.y;
    x[9] = d.z;
    if (NIN == 34) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float sc = (float)(1 << k);  // exact scaling
            sincosf(sc * d.x, &x[10 + 6 * k + 0], &x[13 + 6 * k + 0]);
            sincosf(sc * d.y, &x[10 + 6 * k + 1], &x[13 + 6 * k + 1]);
            sincosf(sc * d.z, &x[10 + 6 * k + 2], &x[13 + 6 * k + 2]);
        }
    }
}


// ---------------------------------------------------------------------------
// Candidate driver shared by the forward, placement and backward kernels.
// ---------------------------------------------------------------------------
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

}  // namespace omerf

