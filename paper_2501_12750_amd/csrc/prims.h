// Primitives as the binning and resolve kernels read them: fetching a
// primitive's inputs by source index, its view-space record, and its
// conservative pixel rectangle (paper, Methods, "Meshless Representations":
// one screen footprint per atom sphere or bond cylinder).
#pragma once

#include "vtx_internal.h"

namespace vtx {

// Raw inputs of one primitive.
struct Item {
    float4 a;          // atom: centre and radius | bond: end A (w unused)
    float4 b;          // bond: end B
    uint32_t id;       // primitive id (atoms i, bonds n_atoms + b, in the caller's numbering)
    uint32_t src;      // source index the primitive is fetched by again (see fetch_src)
    uint32_t kind;     // kNone, kAtom, kBond, kBadBond
};
constexpr uint32_t kNone = 0, kAtom = 1, kBond = 2, kBadBond = 3;

__device__ inline Item empty_item() {
    return Item{make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f), 0u, 0u, kNone};
}

// Primitive p of the caller's arrays (atoms first, then bonds): the plain
// path's source index is p itself.
__device__ inline Item fetch_plain(const global_t<const float>* __restrict__ pos,
                                   const global_t<const float>* __restrict__ rad,
                                   const global_t<const uint32_t>* __restrict__ bonds, uint32_t n_atoms, uint64_t p) {
    Item it = empty_item();
    it.id = (uint32_t)p;
    it.src = (uint32_t)p;
    if (p < n_atoms) {
        it.a = make_float4(pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], rad[p]);
        it.kind = kAtom;
        return it;
    }
    const size_t bi = p - n_atoms;
    const uint32_t ia = bonds[2 * bi], ib = bonds[2 * bi + 1];
    if (ia >= n_atoms || ib >= n_atoms) {
        it.kind = kBadBond;
        return it;
    }
    if (ia == ib) return it;
    it.a = make_float4(pos[3 * (size_t)ia], pos[3 * (size_t)ia + 1], pos[3 * (size_t)ia + 2], 0.f);
    it.b = make_float4(pos[3 * (size_t)ib], pos[3 * (size_t)ib + 1], pos[3 * (size_t)ib + 2], 0.f);
    it.kind = kBond;
    return it;
}

// Stored atom i (< n_atoms) or stored bond n_atoms + j of a resident scene.
__device__ inline Item fetch_scene(const SceneDev& S, uint32_t src) {
    Item it = empty_item();
    it.src = src;
    const global_t<const float4>* __restrict__ const xyzr = to_global(S.xyzr);
    if (src < S.n_atoms) {
        it.a = xyzr[src];
        it.id = to_global(S.atom_id)[src];
        it.kind = kAtom;
        return it;
    }
    const uint32_t j = src - S.n_atoms;
    if (j >= S.n_bonds) return it;
    const uint4 br = to_global(S.bond_rec)[j];
    if (br.x == br.y) return it;
    it.a = xyzr[br.x];
    it.b = xyzr[br.y];
    it.id = S.n_atoms + br.z;
    it.kind = kBond;
    return it;
}

// A job's primitive by source index (resident scene or the caller's arrays).
__device__ inline Item fetch_src(const Job& J, uint32_t src) {
    if (J.S.xyzr) return fetch_scene(J.S, src);
    return fetch_plain(to_global(J.pos), to_global(J.rad), to_global(J.bonds), J.F.n_atoms, src);
}

// View-space record of an item (FP64 view transform rounded once to FP32,
// see PrimRec) and its FP64 view coordinates v (sphere: centre, radius in
// r; bond: ends A = v[0..2], B = v[3..5]).  False when the item cannot show:
// degenerate, or outside the view volume by the FP32 frustum test (kCull;
// without it, for items that have passed the test before).
template <bool kCull = true>
__device__ inline bool item_view(const Frame& F, const Item& it, PrimRec& rec, double* v, double& r) {
    if (it.kind == kAtom) {
        to_view(F, it.a.x, it.a.y, it.a.z, v[0], v[1], v[2]);
        r = (double)atom_radius(F, it.a.w);
        if (!(r > 0.0) || (kCull && !sphere_in_frustum(F, v[0], v[1], v[2], r))) return false;
        rec.g0 = make_float4((float)v[0], (float)v[1], (float)v[2], (float)r);
        rec.g1 = make_uint4(0u, 0u, it.id, 0u);
        return true;
    }
    if (it.kind != kBond) return false;
    if (it.a.x == it.b.x && it.a.y == it.b.y && it.a.z == it.b.z) return false;
    to_view(F, it.a.x, it.a.y, it.a.z, v[0], v[1], v[2]);
    to_view(F, it.b.x, it.b.y, it.b.z, v[3], v[4], v[5]);
    r = F.bond_radius;
    // the difference B - A is kept from FP64, so the axis is accurate however
    // far the bond is
    const double dx = v[3] - v[0], dy = v[4] - v[1], dz = v[5] - v[2];
    // the half length only enters the frustum test, whose margin (1e-4
    // relative) far exceeds the FP32 square root's error
    if (kCull) {
        const double half = 0.5 * (double)__builtin_amdgcn_sqrtf((float)(dx * dx + dy * dy + dz * dz));
        if (!sphere_in_frustum(F, v[0] + 0.5 * dx, v[1] + 0.5 * dy, v[2] + 0.5 * dz, half + r)) return false;
    }
    rec.g0 = make_float4((float)v[0], (float)v[1], (float)v[2], (float)dx);
    rec.g1 = make_uint4(__float_as_uint((float)dy), __float_as_uint((float)dz), it.id, 0u);
    return true;
}

// Conservative pixel rectangle of a sphere in front of the eye plane
// (perspective), in FP32: the tangent-plane interval of each axis with a
// margin of 0.02 pixel, about ten times the bound on its rounding error for
// spheres with vz >= 1.05 r; nearer the eye plane (where vz^2 - r^2 loses
// its digits), orthographic views and everything else take the FP64 path.
// A rectangle only has to contain the footprint: a larger one adds pixels
// whose ray test misses.
// Pixel-space extent [ax, bx] x [ay, by] (unclamped, pixel centres at
// i + 1/2) of a sphere with vz >= 1.05 r, perspective, in FP32.
__device__ inline void sphere_extent_f32(const Frame& F, double vx, double vy, double vz, double r, float& ax,
                                         float& bx, float& ay, float& by) {
    const float x = (float)vx, y = (float)vy, z = (float)vz, rf = (float)r;
    const float den = fmaf(z, z, -rf * rf);
    const float inv = __builtin_amdgcn_rcpf(den);
    const float sx = rf * __builtin_amdgcn_sqrtf(fmaf(x, x, den));
    const float sy = rf * __builtin_amdgcn_sqrtf(fmaf(y, y, den));
    const float kx = inv * F.itxf * 0.5f * (float)F.W, ky = inv * F.ityf * 0.5f * (float)F.H;
    ax = fmaf(fmaf(x, z, -sx), kx, 0.5f * (float)F.W);
    bx = fmaf(fmaf(x, z, sx), kx, 0.5f * (float)F.W);
    ay = fmaf(-fmaf(y, z, sy), ky, 0.5f * (float)F.H);
    by = fmaf(-fmaf(y, z, -sy), ky, 0.5f * (float)F.H);
}

// Pixel rectangle from an FP32 extent, widened by the margin and clamped to
// the image.
__device__ inline bool extent_pixels(const Frame& F, float ax, float bx, float ay, float by, int& x0, int& y0,
                                     int& x1, int& y1) {
    constexpr float kMargin = 0.02f;
    const float fw = (float)F.W, fh = (float)F.H;
    x0 = (int)fminf(fmaxf(ceilf(ax - 0.5f - kMargin), 0.0f), fw);
    x1 = (int)fmaxf(fminf(floorf(bx - 0.5f + kMargin), fw - 1.0f), -1.0f);
    y0 = (int)fminf(fmaxf(ceilf(ay - 0.5f - kMargin), 0.0f), fh);
    y1 = (int)fmaxf(fminf(floorf(by - 0.5f + kMargin), fh - 1.0f), -1.0f);
    return x0 <= x1 && y0 <= y1;
}

__device__ inline bool sphere_rect_fast(const Frame& F, double vx, double vy, double vz, double r, int& x0, int& y0,
                                        int& x1, int& y1) {
    if (F.proj != 0 || !(vz >= 1.05 * r) || vz - r > F.zfar) return sphere_rect(F, vx, vy, vz, r, x0, y0, x1, y1);
    if (vz + r < F.znear) return false;
    float ax, bx, ay, by;
    sphere_extent_f32(F, vx, vy, vz, r, ax, bx, ay, by);
    return extent_pixels(F, ax, bx, ay, by, x0, y0, x1, y1);
}

// The same for a capped cylinder of radius rho between view points A and B:
// its projection lies in the union of the two end balls' extents (the
// capsule's), taken unclamped and then clamped, when both balls are at
// least 1.05 rho in front of the eye; otherwise bond_rect in FP64.
__device__ inline bool bond_rect_fast(const Frame& F, const double* A, const double* B, double rho, int& x0,
                                      int& y0, int& x1, int& y1) {
    if (F.proj != 0 || !(A[2] >= 1.05 * rho) || !(B[2] >= 1.05 * rho)) return bond_rect(F, A, B, rho, x0, y0, x1, y1);
    const double zlo = fmin(A[2], B[2]) - rho, zhi = fmax(A[2], B[2]) + rho;
    if (zhi < F.znear || zlo > F.zfar) return false;
    float ax, bx, ay, by, cx, dx, cy, dy;
    sphere_extent_f32(F, A[0], A[1], A[2], rho, ax, bx, ay, by);
    sphere_extent_f32(F, B[0], B[1], B[2], rho, cx, dx, cy, dy);
    return extent_pixels(F, fminf(ax, cx), fmaxf(bx, dx), fminf(ay, cy), fmaxf(by, dy), x0, y0, x1, y1);
}

}  // namespace vtx
