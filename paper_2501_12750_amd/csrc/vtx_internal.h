// Internal declarations of the HIP renderer: frame constants, device counters,
// geometry helpers shared by the kernels, and the host launch wrappers.
//
// Method: paper, Methods, "Molecular Graphics Engine" (spheres for atoms,
// cylinders for bonds, one screen footprint per primitive, then a ray-cast of
// the implicit surface per pixel) and "High Quality Rendering" (deferred
// shading with screen-space ambient occlusion).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vtx {

constexpr int kBlock = 256;                  // threads per workgroup (4 waves of 64)
constexpr int kBinThreads = 1024;            // binning workgroups (16 waves)
constexpr int kMaxLdsTiles = 15360;          // tile histogram of one binning workgroup (< 64 KiB of LDS)
constexpr uint32_t kMaxBinGroups = 512;
constexpr uint32_t kBackground = 0xFFFFFFFFu;
// A resolve winner whose FP32 depth may miss the depth tolerance (1e-5 of the
// depth) carries kRefineBit in its id until the refine pass has recomputed the
// depth in FP64 and cleared it.  Frames with 2^31 - 1 primitives or more have
// no room for the bit and refine every hit.
constexpr uint32_t kRefineBit = 0x80000000u;
// The FP32 sphere root is off by at most about 32 u |c| / (n.V) (u = 2^-24,
// c the record's view-space centre, rounded once from FP64): the centre's
// rounding moves the entry by u |c| / (n.V), the discriminant's rounding
// (a dozen u r |c|) moves its root by that over 2 r (n.V), and the rest is a
// few u |c|.  Hits with n.V >= kGrazeCos and r <= z / 4 (so |c| <= 1.25 z)
// are therefore within 6e-6 of the depth; the others are refined.
constexpr float kGrazeCos = 0.4f;
constexpr int kMaxSamples = 64;
// Resident scenes bin their visible clusters front to back: the frustum test
// files each cluster under one of kDepthBuckets depth classes (log spacing
// from znear to zfar), and the tile lists keep the order of kLayers
// consecutive ranges of binning workgroups.
constexpr int kDepthBuckets = 64;
constexpr int kLayers = 32;
// Occlusion pre-pass of resident scenes: the nearest 1 / kFrontShare of the
// depth-ordered visible clusters (rounded up to the end of its depth class
// unless that would pass half of them) is binned and resolved first; of the
// rest only the clusters not behind its 16x16-pixel block depths are binned.
constexpr int kFrontShare = 8;
constexpr int kHzCell = 16;
enum Phase : int { kPhaseAll = 0, kPhaseFront = 1, kPhaseRest = 2 };

// Per-frame constants, passed by value to every kernel.
struct Frame {
    double eye[3], s[3], u[3], f[3];   // world -> view basis (x right, y up, z forward)
    double tx, ty;                     // perspective: tan(fovy/2) * W/H, tan(fovy/2)
    double hx, hy;                     // orthographic: h * W/H, h
    double itx, ity, ihx, ihy;         // their inverses
    float txf, tyf, hxf, hyf;
    float itxf, ityf;                  // 1 / tx, 1 / ty
    float sxf, syf;                    // perspective: sqrt(1 + tx^2), sqrt(1 + ty^2)
    float inv_w2, inv_h2;              // 2/W, 2/H
    float ssao_fpx, ssao_osc;          // view to pixel scale of SSAO samples: 0.5 H / ty, 0.5 H / hy (FP32)
    double inv_w2d, inv_h2d;           // the same in FP64
    float znear, zfar;
    float bond_radius;
    int32_t proj;                      // 0 perspective, 1 orthographic
    int32_t W, H;
    int32_t tile, tiles_x, tiles_y;
    int32_t tile_shift;                // tile = 1 << tile_shift
    uint32_t n_atoms, n_bonds;         // n_bonds: bonds drawn (0 when the representation has none)
    uint32_t flags;
    int32_t rep;                       // VTX_REP_* : radius of the atom spheres
    float probe;                       // VTX_REP_SAS probe radius
    int32_t shading;                   // VTX_SHADE_*
    float fog_start, fog_inv;          // fog factor (z - fog_start) * fog_inv; fog_inv = 0: no fog
    float fog_rgb[3];
    float outline_t;                   // relative depth step of an outline; 0: none
    uint32_t outline_rgba;             // packed RGBA8 of outline pixels (alpha 255)
    int32_t clip_on;                   // a clip plane is set
    int32_t refine_flag;               // ids leave room for kRefineBit (fewer than 2^31 - 1 primitives)
    float clip[4];                     // the plane in view coordinates: kept where clip . (x, y, z, 1) >= 0
    // depth class of a front depth z (resident scenes; orders the lists, never
    // changes the image): floor(log2(z / cls_z0) * cls_k), clamped to the classes
    float cls_z0, cls_k;
};

// Sphere radius of an atom of given radius r under the frame's representation.
__host__ __device__ inline float atom_radius(const Frame& F, float r) {
    return F.rep == 2 ? F.bond_radius : F.rep == 3 ? r + F.probe : r;
}

// SSAO sample set: h[k].xyz is sample k's offset in the frame (tangent,
// bitangent, normal) of the surface point, already scaled to its length
// (the radius times the sample's scale), h[k].w that length.
struct SampleKernel {
    float4 h[kMaxSamples];
    // noise form (options.ssao_noise): the turn of the tangent frame of a
    // pixel of 4x4-tile rank b, (cos, sin) of 2 pi (b + 1/2) / 16
    float2 rot[16];
    int32_t count;
    float radius, bias;
    uint32_t background;
    int32_t noise;
};

// Device-side counters of one frame.  The scatter's first workgroup
// publishes the binning counters to host-mapped memory; on counting frames
// the resolve's tail launch publishes the fragment counters.
struct Counters {
    unsigned int vis_count;
    unsigned int overflow;
    unsigned int bad_bonds;
    unsigned int overflow_tiles;
    unsigned long long pairs;
    unsigned long long frag_tested;
    unsigned long long frag_hit;
    unsigned long long frag_hit_bond;
    // counting frames: ray tests on bonds, tests skipped by the per-pixel
    // depth test, records culled by block depths, lists and depth-ordered
    // chunks ended early
    unsigned long long frag_tested_bond;
    unsigned long long frag_skipped;
    unsigned long long rec_culled;
    unsigned long long lists_stopped;
    unsigned long long chunks_stopped;
    unsigned int done_blocks;
    unsigned int vis_bucket[kDepthBuckets];   // resident scenes: clusters that passed the frustum test, per depth class
    // resident scenes: per pass (one pass or the front pass; the rest) and
    // layer, float bits of a lower bound of the resolve's cull depth of every
    // primitive its workgroups binned (+inf: none; 0: not positive)
    unsigned int layer_zlo[2][kLayers];
    unsigned long long pairs_counted;   // total of the tile counts, added by the count kernel
};

// View-space record of one visible primitive (32 bytes), computed from FP64
// and rounded to FP32; the resolve rebuilds it from the 8-byte tile-list
// entry (source index, footprint).
//   sphere: g0 = (centre x, y, z, radius),      g1 = (0, 0, id, footprint)
//   bond:   g0 = (A x, y, z, (B - A).x),         g1 = ((B - A).y, (B - A).z, id, footprint)
// id >= n_atoms marks a bond.  The footprint word is the primitive's pixel
// rectangle clipped to the tile, x0 | y0 << 8 | w << 16 | h << 24 in
// tile-local pixels.
struct PrimRec {
    float4 g0;
    uint4 g1;
};

// ---------------------------------------------------------------------------
// geometry helpers (device)
// ---------------------------------------------------------------------------
__device__ inline void to_view(const Frame& F, float px, float py, float pz, double& vx, double& vy,
                               double& vz) {
    const double rx = (double)px - F.eye[0], ry = (double)py - F.eye[1], rz = (double)pz - F.eye[2];
    vx = rx * F.s[0] + ry * F.s[1] + rz * F.s[2];
    vy = rx * F.u[0] + ry * F.u[1] + rz * F.u[2];
    vz = rx * F.f[0] + ry * F.f[1] + rz * F.f[2];
}

// Interval of NDC coordinates along one image axis covered by a sphere of
// view-space centre (c, vz) (c = x or y) and radius r in front of the eye
// plane (perspective, vz > r): the two planes through the eye tangent to the
// sphere have slopes (c vz -+ r sqrt(c^2 + vz^2 - r^2)) / (vz^2 - r^2).
// `den` = vz^2 - r^2 and `scale` = 1 / (den tan) for the axis' tangent `tan`
// (one division per sphere serves both axes).
__device__ inline void persp_interval(double c, double vz, double r, double den, double scale, double& lo,
                                      double& hi) {
    const double sq = r * sqrt(c * c + den);
    lo = (c * vz - sq) * scale;
    hi = (c * vz + sq) * scale;
}

// Inclusive pixel index range of the pixel centres whose NDC lies in [lo, hi]
// along an axis of n pixels; `flip` for the y axis (row 0 at the top).
__device__ inline void ndc_to_pixels(double lo, double hi, int n, bool flip, int& p0, int& p1) {
    const double eps = 1e-3;
    double a, b;
    if (!flip) {
        a = (lo + 1.0) * 0.5 * n;
        b = (hi + 1.0) * 0.5 * n;
    } else {
        a = (1.0 - hi) * 0.5 * n;
        b = (1.0 - lo) * 0.5 * n;
    }
    a = ceil(a - 0.5 - eps);
    b = floor(b - 0.5 + eps);
    a = fmax(a, 0.0);
    b = fmin(b, (double)(n - 1));
    p0 = (int)fmin(a, (double)n);
    p1 = (int)fmax(b, -1.0);
}

// NDC interval along one axis covered by the view-space box
// [c_lo, c_hi] x [z_lo, z_hi] with z_lo > 0 (perspective): the projection of
// a box in front of the eye is the convex hull of its projected corners.
__device__ inline void box_ndc_interval(double c_lo, double c_hi, double z_lo, double z_hi, double tscale,
                                        double& lo, double& hi) {
    lo = fmin(c_lo / z_lo, c_lo / z_hi) / tscale;
    hi = fmax(c_hi / z_lo, c_hi / z_hi) / tscale;
}

// Conservative pixel rectangle of a sphere of view centre v and radius r.
// Returns false when no pixel can hold a hit with znear <= z <= zfar.  A
// sphere that reaches the eye plane has an unbounded projection, but only its
// part with z >= znear can be hit: that part lies in its bounding box cut at
// znear, whose projected corners bound it.
__device__ inline bool sphere_rect(const Frame& F, double vx, double vy, double vz, double r, int& x0,
                                   int& y0, int& x1, int& y1) {
    if (!(r > 0.0)) return false;
    if (vz + r < F.znear || vz - r > F.zfar) return false;
    double lo, hi;
    if (F.proj != 0) {
        ndc_to_pixels((vx - r) * F.ihx, (vx + r) * F.ihx, F.W, false, x0, x1);
        ndc_to_pixels((vy - r) * F.ihy, (vy + r) * F.ihy, F.H, true, y0, y1);
    } else if (vz > r) {
        const double den = vz * vz - r * r, inv = 1.0 / den;
        persp_interval(vx, vz, r, den, inv * F.itx, lo, hi);
        ndc_to_pixels(lo, hi, F.W, false, x0, x1);
        persp_interval(vy, vz, r, den, inv * F.ity, lo, hi);
        ndc_to_pixels(lo, hi, F.H, true, y0, y1);
    } else {
        const double zl = F.znear, zh = vz + r;
        box_ndc_interval(vx - r, vx + r, zl, zh, F.tx, lo, hi);
        ndc_to_pixels(lo, hi, F.W, false, x0, x1);
        box_ndc_interval(vy - r, vy + r, zl, zh, F.ty, lo, hi);
        ndc_to_pixels(lo, hi, F.H, true, y0, y1);
    }
    return x0 <= x1 && y0 <= y1;
}

// Conservative pixel rectangle of a capped cylinder of radius rho between
// view points A and B: it lies inside the capsule (the convex hull of the two
// end balls), whose projection's bounding box is the union of the two balls'
// boxes when both lie in front of the eye plane; otherwise its part with
// z >= znear lies in the capsule's bounding box cut at znear.
__device__ inline bool bond_rect(const Frame& F, const double* A, const double* B, double rho, int& x0,
                                 int& y0, int& x1, int& y1) {
    const double zlo = fmin(A[2], B[2]) - rho, zhi = fmax(A[2], B[2]) + rho;
    if (zhi < F.znear || zlo > F.zfar) return false;
    if (F.proj == 0 && !(zlo > 0.0)) {
        double lo, hi;
        box_ndc_interval(fmin(A[0], B[0]) - rho, fmax(A[0], B[0]) + rho, F.znear, zhi, F.tx, lo, hi);
        ndc_to_pixels(lo, hi, F.W, false, x0, x1);
        box_ndc_interval(fmin(A[1], B[1]) - rho, fmax(A[1], B[1]) + rho, F.znear, zhi, F.ty, lo, hi);
        ndc_to_pixels(lo, hi, F.H, true, y0, y1);
        return x0 <= x1 && y0 <= y1;
    }
    double la, ha, lb, hb;
    if (F.proj != 0) {
        ndc_to_pixels((fmin(A[0], B[0]) - rho) * F.ihx, (fmax(A[0], B[0]) + rho) * F.ihx, F.W, false, x0, x1);
        ndc_to_pixels((fmin(A[1], B[1]) - rho) * F.ihy, (fmax(A[1], B[1]) + rho) * F.ihy, F.H, true, y0, y1);
        return x0 <= x1 && y0 <= y1;
    }
    // both end balls lie in front of the eye plane (zlo > 0)
    const double da = A[2] * A[2] - rho * rho, db = B[2] * B[2] - rho * rho;
    const double ia = 1.0 / da, ib = 1.0 / db;
    persp_interval(A[0], A[2], rho, da, ia * F.itx, la, ha);
    persp_interval(B[0], B[2], rho, db, ib * F.itx, lb, hb);
    ndc_to_pixels(fmin(la, lb), fmax(ha, hb), F.W, false, x0, x1);
    persp_interval(A[1], A[2], rho, da, ia * F.ity, la, ha);
    persp_interval(B[1], B[2], rho, db, ib * F.ity, lb, hb);
    ndc_to_pixels(fmin(la, lb), fmax(ha, hb), F.H, true, y0, y1);
    return x0 <= x1 && y0 <= y1;
}

// Cheap conservative frustum test of a view-space bounding sphere, in FP32
// (the margin covers the rounding of the view coordinates): false when no
// point of the sphere is inside the view volume.
__device__ inline bool sphere_in_frustum(const Frame& F, double vx, double vy, double vz, double r) {
    const float z = (float)vz, x = (float)vx, y = (float)vy;
    const float rr = (float)r + 1e-4f * (fabsf(x) + fabsf(y) + fabsf(z) + (float)r);
    if (z + rr < F.znear || z - rr > F.zfar) return false;
    if (F.proj == 0) {
        const float ex = rr * F.sxf, ey = rr * F.syf;
        return !(x - F.txf * z > ex || -x - F.txf * z > ex || y - F.tyf * z > ey || -y - F.tyf * z > ey);
    }
    return !(fabsf(x) > F.hxf + rr || fabsf(y) > F.hyf + rr);
}

// A bounding sphere wholly inside the view volume, by a margin of 1e-3 of
// its coordinates' magnitudes (FP64): every primitive inside it passes
// sphere_in_frustum, so the count kernel skips that test for its atoms.
__device__ inline bool sphere_inside_frustum(const Frame& F, double vx, double vy, double vz, double r) {
    const double m = 1e-3 * (fabs(vx) + fabs(vy) + fabs(vz) + r) + 1e-3;
    if (!(vz - r >= (double)F.znear + m) || !(vz + r <= (double)F.zfar - m)) return false;
    if (F.proj == 0) {
        const double rx = r * sqrt(1.0 + F.tx * F.tx) + m, ry = r * sqrt(1.0 + F.ty * F.ty) + m;
        return fabs(vx) + rx <= F.tx * vz && fabs(vy) + ry <= F.ty * vz;
    }
    return fabs(vx) + r + m <= F.hx && fabs(vy) + r + m <= F.hy;
}
// Flag of a visible-cluster entry whose sphere is wholly inside the view
// volume (cluster indices stay below 2^31).
constexpr uint32_t kClusterInside = 0x80000000u;

// A device buffer typed in the global address space.  A pointer a batch
// reads from its job table is generic to the compiler, which then emits flat
// accesses (a 64-bit address each, and waits shared with LDS); through this
// type they take the global form (a scalar base and a 32-bit offset), as
// accesses through kernel arguments do.  Every buffer the kernels are given
// is device or host-mapped memory, never LDS or scratch.  (The host pass,
// which only parses device code, takes the plain type.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using global_t = __attribute__((address_space(1))) T;
#else
template <class T>
using global_t = T;
#endif
template <class T>
__device__ inline global_t<T>* to_global(T* p) { return (global_t<T>*)p; }

// Hardware dispatch places workgroup b on XCD (b mod 8).  Give each XCD one
// contiguous range of work items so neighbouring tiles share an L2.
__device__ inline int xcd_contiguous(int b, int nblocks) {
    const int per = (nblocks + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

inline int xcd_grid(int nblocks) { return ((nblocks + 7) >> 3) << 3; }

// Binning workgroup b of `groups` belongs to layer b * layers / groups; layer
// g holds the workgroups [layer_first(g), layer_first(g + 1)).
__device__ inline uint32_t layer_of(uint32_t b, uint32_t groups, uint32_t layers) {
    return (uint32_t)(((uint64_t)b * layers) / groups);
}
__device__ inline uint32_t layer_first(uint32_t g, uint32_t groups, uint32_t layers) {
    return (uint32_t)(((uint64_t)g * groups + layers - 1) / layers);
}

// ---------------------------------------------------------------------------
// host launch wrappers (one per kernel file)
// ---------------------------------------------------------------------------
// Kernel clock of a timed frame: while one is set on the host thread, every
// frame kernel is dispatched with a start and a stop event of its own
// (hipExtLaunchKernel), which take the dispatch's own begin and end
// timestamps, so the time of each kernel excludes launch gaps and event
// packets.  `cur` is the time category of the launches queued next.
struct KernelClock {
    static constexpr int kMax = 24;
    hipEvent_t start[kMax], stop[kMax];
    int cat[kMax];
    int used;
    int cur;
};
KernelClock*& kernel_clock();

// Dispatches kernel `k` on `stream`, timed when a kernel clock is set.
template <class... Params, class... Args>
hipError_t dispatch(void (*k)(Params...), dim3 grid, dim3 block, uint32_t lds, hipStream_t stream, Args... args) {
    KernelClock* c = kernel_clock();
    hipEvent_t a = nullptr, b = nullptr;
    if (c && c->used < KernelClock::kMax) {
        const int i = c->used++;
        c->cat[i] = c->cur;
        a = c->start[i];
        b = c->stop[i];
    }
    hipExtLaunchKernelGGL(k, grid, block, lds, stream, a, b, 0u, static_cast<Params>(args)...);
    return hipGetLastError();
}

// Binning scratch.  The `groups` binning workgroups each own `chunk`
// consecutive primitives and the same range of the visible-list arrays.
struct BinBuffers {
    uint32_t* tile_cnt;     // T
    uint64_t* tile_off;     // T
    uint32_t* tile_fill;    // layers * T: next free entry of each layer's run of each tile list
    uint32_t* layer_off;    // layers * T: start of each layer's run within each tile list
    uint32_t* layer_sum;    // layers * T: entries of each layer in each tile list, added up by the
                            // count kernel, read and re-zeroed by the layer kernel
    uint32_t* vis_src;      // groups * chunk: source index of each visible primitive
    uint2* vis_rect;        // groups * chunk, pixel rectangle packed (x0 | y0 << 16, x1 | y1 << 16)
    uint32_t* vis_cnt;      // groups: visible primitives of each workgroup
    uint2* vis_box;         // groups: tile-space bounding box of each workgroup's visible
                            // primitives, packed like vis_rect (empty: x0 > x1)
    uint32_t* hist;         // groups * T: tile histogram of each workgroup
    uint2* list;            // capacity entries (source index, tile-local footprint), each tile's contiguous
    uint64_t capacity;
    uint32_t groups, chunk;
    uint32_t layers;        // 1, or kLayers for a resident scene (workgroup ranges of increasing depth)
    uint32_t* hz16;         // two-pass frames: float bits of the farthest depth of each 16x16-pixel
                            // cell after the front pass (+inf while a pixel is empty), hz16_w per row
    int32_t hz16_w;
    Counters* ctr;
    Counters* host_ctr;     // device address of host-mapped counters (may be null)
};

// Binning grid for n primitives (groups <= kMaxBinGroups, groups * chunk >= n).
void bin_grid(uint64_t nprim, uint32_t* groups, uint32_t* chunk);

// Resident scene (device arrays owned by the library).  Atoms are stored in
// Morton order as an xyzr stream, grouped in clusters of kCluster; bonds are
// re-indexed to those positions and sorted by their first atom.
constexpr int kCluster = 256;
struct SceneDev {
    uint32_t n_atoms, n_bonds;          // n_bonds: valid bonds (both indices < n_atoms)
    uint32_t n_bonds_total;             // bonds as given (ids run over these)
    uint32_t atom_clusters, bond_clusters;
    const float4* xyzr;                 // n_atoms, Morton order
    const uint32_t* atom_id;            // n_atoms: original index of each stored atom
    const uint4* bond_rec;              // n_bonds: (stored index a, stored index b, original bond index, 0)
    const float4* cluster_box;          // 2 per cluster: (min xyz, -), (max xyz, -); bond boxes exclude the radius
    uint32_t* vis_clusters;             // kDepthBuckets regions of atom_clusters + bond_clusters entries:
                                        // visible cluster ids per depth class (per render)
};
// Stable radix sort (sort.hip) of n (key, value) pairs by the low end_bit
// bits of the keys, 8 bits per pass.  keys/vals hold the input and are
// overwritten, like keys_alt/vals_alt; the sorted values go to vals_out,
// which may be vals when the number of passes is even, vals_alt when it is
// odd.  scratch holds radix_sort_scratch_words(n) words.
size_t radix_sort_scratch_words(size_t n);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt,
                            uint32_t* vals_out, size_t n, int end_bit, uint32_t* scratch, hipStream_t stream);
// Original index of each stored atom and of each stored bond (device
// arrays; either may be null).
hipError_t scene_order(const SceneDev& S, uint32_t* atom_order, uint32_t* bond_order, hipStream_t stream);
size_t scene_build_temp_bytes(uint64_t n, uint64_t m);
hipError_t scene_build(const float* pos, const float* rad, const uint32_t* bonds, uint64_t n, uint64_t m,
                       SceneDev& S, float4* xyzr, uint32_t* atom_id, uint4* bond_rec, float4* cluster_box,
                       void* tmp, size_t tmp_bytes, uint32_t* m_valid, uint32_t* n_bad, uint32_t* box_bits,
                       hipStream_t stream);
hipError_t scene_update_positions(const float* pos, SceneDev& S, float4* xyzr, float4* cluster_box,
                                  hipStream_t stream);

// Zeroes n 32-bit words (used when scratch is allocated; the frame kernels
// leave the tile counts and the counters zeroed for the next frame).
hipError_t launch_zero(uint32_t* p, size_t n, hipStream_t stream);

// ---------------------------------------------------------------------------
// jobs: one render (camera, image, primitives, scratch, outputs)
// ---------------------------------------------------------------------------
struct Job {
    Frame F;
    // primitives in the caller's order: the plain path bins them, and the
    // deferred pass reads every render's primitives through them by id
    const float* pos;
    const float* rad;
    const uint32_t* col;
    const uint32_t* bonds;
    SceneDev S;              // resident scene (scene path only)
    BinBuffers bb;           // this render's binning scratch
    float* depth;
    uint32_t* id;
    uint32_t* rgba;
    float* normal;           // optional deferred outputs (may be null)
    uint32_t* albedo;
    float* ao;
};

// Per-kernel work-block counts of a job (the grid of a launch is the sum over
// its jobs, padded to a multiple of 8 for the XCD mapping).
inline uint32_t cull_blocks(const SceneDev& S) {
    const uint32_t nc = S.atom_clusters + S.bond_clusters;
    return (nc + kBlock - 1) / kBlock;
}
inline uint32_t shade_blocks(const Frame& F) { return (uint32_t)(((F.W + 15) / 16) * ((F.H + 15) / 16)); }

// A launch over one render: the job travels in the kernel arguments.
struct OneJob {
    Job j;
    SampleKernel K;
    static constexpr bool kMany = false;
    uint32_t blocks;         // work blocks of the launch (the grid may be padded past it)
    __device__ int find(uint32_t g, uint32_t& local) const {
        local = g;
        return g < blocks ? 0 : -1;
    }
    __device__ const Job& job(int) const { return j; }
    __device__ const SampleKernel& samples(int) const { return K; }
    __device__ uint32_t count() const { return 1; }
    // the work block after (i, local): the next one of the job, else -1
    __device__ void next(int& i, uint32_t& local) const {
        if (i >= 0 && ++local >= blocks) i = -1;
    }
};

// A launch over several renders, described by device tables: job i owns the
// work blocks [start[i], start[i + 1]).
struct JobList {
    static constexpr bool kMany = true;   // a batch launch (see resolve_tile's kInline)
    const Job* jobs;
    const SampleKernel* K;
    const uint32_t* start;   // n + 1 entries
    uint32_t n;
    uint32_t per;            // when every job has this many blocks (else 0): job g / per
    uint32_t no_bonds;       // no job's scene holds bonds (the count's atom-only instantiation)
    __device__ int find(uint32_t g, uint32_t& local) const {
        if (per) {
            if (g >= n * per) return -1;
            const uint32_t i = g / per;
            local = g - i * per;
            return (int)i;
        }
        if (g >= start[n]) return -1;
        uint32_t lo = 0, hi = n;   // the last i with start[i] <= g (jobs without blocks are skipped)
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (start[mid] <= g) lo = mid;
            else hi = mid;
        }
        local = g - start[lo];
        return (int)lo;
    }
    __device__ const Job& job(int i) const { return jobs[i]; }
    __device__ const SampleKernel& samples(int i) const { return K[i]; }
    __device__ uint32_t count() const { return n; }
    // the work block after (i, local): the next one of job i, else the first
    // of the next job that has any, else -1 (no search)
    __device__ void next(int& i, uint32_t& local) const {
        if (i < 0) return;
        ++local;
        while ((uint32_t)i < n && local >= (per ? per : start[i + 1] - start[i])) {
            ++i;
            local = 0;
        }
        if ((uint32_t)i >= n) i = -1;
    }
};

// Launch wrappers, one overload per job source.  `grid` is the number of
// work blocks (sum over the jobs); `max_tiles` the largest tile grid of the
// jobs (LDS of the binning kernels).  `tile` selects the resolve
// instantiation: every job of one resolve launch has that tile size; `count`
// selects the one that counts fragments (needed when any job sets
// VTX_FLAG_STATS).
hipError_t launch_cluster_cull(const OneJob& js, uint32_t grid, hipStream_t stream);
hipError_t launch_cluster_cull(const JobList& js, uint32_t grid, hipStream_t stream);
// `phase` (resident scenes): kPhaseAll bins every visible cluster; a
// two-pass frame runs count to resolve with kPhaseFront, then again with
// kPhaseRest, whose resolve starts from the front pass's G-buffer.
hipError_t launch_count(const OneJob& js, bool scene, int phase, uint32_t grid, int max_tiles, hipStream_t stream);
hipError_t launch_count(const JobList& js, bool scene, int phase, uint32_t grid, int max_tiles, hipStream_t stream);
// Layer starts of every tile list from the count kernel's histograms (jobs
// with layers > 1; runs on the binning grid).
hipError_t launch_layers(const OneJob& js, uint32_t grid, hipStream_t stream);
hipError_t launch_layers(const JobList& js, uint32_t grid, hipStream_t stream);
// List offsets of every tile (exclusive prefix sum of the counts), the list
// total and the overflow flag, one workgroup per job.
hipError_t launch_tile_offsets(const OneJob& js, hipStream_t stream);
hipError_t launch_tile_offsets(const JobList& js, hipStream_t stream);
hipError_t launch_scatter(const OneJob& js, int phase, uint32_t grid, int max_tiles, hipStream_t stream);
hipError_t launch_scatter(const JobList& js, int phase, uint32_t grid, int max_tiles, hipStream_t stream);
// The resolve is a main launch plus a small tail launch for the tiles whose
// lists overflowed: `ovf` holds at least `grid` entries and ovf_n two zeroed
// counters (both left zeroed again).
hipError_t launch_resolve(const OneJob& js, int tile, int phase, uint32_t grid, bool count, unsigned long long* ovf,
                          uint32_t* ovf_n, hipStream_t stream);
hipError_t launch_resolve(const JobList& js, int tile, int phase, uint32_t grid, bool count, unsigned long long* ovf,
                          uint32_t* ovf_n, hipStream_t stream);
// Supersampled render: output pixel (x, y) of W x H from its S x S samples
// of the (S W) x (S H) images (channel means rounded half up, nearest
// (depth, id)).
hipError_t launch_downsample(const float* sdepth, const uint32_t* sid, const uint32_t* srgba, int W, int H, int S,
                             float* depth, uint32_t* id, uint32_t* rgba, hipStream_t stream);
// `noise`: some job asks for the noise form of the ambient occlusion.
// FP64 depths of the pixels the resolve marked, over the shade's 16x16
// blocks (resolve.hip); runs after the last resolve of a frame.
hipError_t launch_refine(const OneJob& js, uint32_t grid, hipStream_t stream);
hipError_t launch_refine(const JobList& js, uint32_t grid, hipStream_t stream);
hipError_t launch_shade(const OneJob& js, uint32_t grid, bool noise, hipStream_t stream);
hipError_t launch_shade(const JobList& js, uint32_t grid, bool noise, hipStream_t stream);

// In-place exclusive prefix sum of n counts (scan.hip); bsum needs
// scan_scratch_words(n) words; *total (may be null) gets the sum.
size_t scan_scratch_words(size_t n);
hipError_t exclusive_scan(uint32_t* v, size_t n, uint32_t* bsum, unsigned long long* total, hipStream_t stream);

// Solvent excluded surface (ses.hip): scratch of one call, sized by
// ses_scratch_words, and the passes (queued on `stream`; field may not be
// null).
struct SesScratch {
    uint8_t* mark;          // grid points: 1 inside the solvent-accessible region
    int32_t* ga;            // squared distances, x and z passes
    int32_t* gb;            // squared distances, y pass
    uint32_t* cnt;          // triangles per cube, then their offsets
    uint32_t* bsum;         // block sums of the scan
};
size_t ses_scratch_words(const int dims[3], size_t* mark_words, size_t* g_words, size_t* cnt_words,
                         size_t* bsum_words);
hipError_t ses_run(const float* pos, const float* rad, uint64_t n, float probe, const float origin[3], float spacing,
                   const int dims[3], float* field, float* tri, uint64_t capacity, unsigned long long* n_tri,
                   SesScratch& s, hipStream_t stream);

}  // namespace vtx
