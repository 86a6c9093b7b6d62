// Per-tile visibility resolve: ray-cast every pixel of a tile against the
// primitives binned to it and keep the nearest hit (paper, Methods,
// "Meshless Representations": ray-casting evaluates the implicit equation of
// each primitive, which makes the display pixel-exact).
//
// One workgroup owns one tile.  The tile's list holds 8-byte entries (source
// index, footprint clipped to the tile); each chunk of 256 entries is turned
// back into view-space records from the sources and staged in LDS.  The
// records' footprint pixel counts are prefix-summed and the resulting
// (record, pixel) fragments are dealt to the 256 lanes round-robin, so the
// load is balanced whatever the mix of tiny and large primitives, and lanes of
// one wave work on neighbouring pixels of the same few records.  A hit is
// folded into the tile's depth buffer in LDS with one 64-bit atomicMin of the
// packed key (float bits of z) << 32 | id: positive floats order like their
// bit patterns, so the minimum key is the nearest hit and equal depths go to
// the smaller id, in any order of evaluation.
//
// Depth early-outs, all conservative (statistics frames switch them off):
// a record whose nearest possible depth lies behind everything the 4x4-pixel
// blocks under its footprint hold is dropped; a fragment whose pixel holds a
// nearer hit is skipped; chunks of large footprints run front to back in
// small sub-chunks and end once the depth bucket they reached lies behind the
// whole tile; a resident scene's list, ordered front to back by layers, ends
// once every layer left lies behind the whole tile.
#include "prims.h"

namespace vtx {

namespace {

constexpr int kChunk = kBlock;
constexpr unsigned kTailBlocks = 256;   // grid of the overflow (tail) launch
constexpr int kBuckets = 64;      // depth buckets of the front-to-back record order
static_assert(kBuckets <= 64, "one wave scans and searches the buckets");
constexpr int kSortArea = 64;     // order a chunk when its kept records average more pixels than this
constexpr int kKeptShift = 21;    // packed scan: footprint area (<= 256 * 64 * 64) below, kept count above
constexpr uint32_t kAreaMask = (1u << kKeptShift) - 1u;
constexpr int kLaterSub = 8;      // records per depth-ordered sub-chunk after the first (4 to 64, a power of 2)
static_assert(kBlock == kChunk, "one 64-slot window per wave in the order array");
template <int TS>
struct HzGrid {
    static constexpr int kBlocks = (TS / 4) * (TS / 4);
};

struct Rec {
    float4 a;          // sphere: centre (view), radius | cylinder: A (view), radius
    float4 b;          // cylinder: unit axis (view), length
    float zcull;       // lower bound of the depth of any hit of this record
    uint32_t id;
    uint32_t rect;     // tile-local x0 | y0 << 8 | w << 16 | h << 24
    float inv_w;       // 1 / w (hardware reciprocal): splits a footprint offset into row and column
};

__device__ inline float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Inclusive max-scan over the 64 lanes of a wave by DPP row shifts and row
// broadcasts (lanes shifted in from outside a row read 0, the identity).
__device__ inline uint32_t wave_incl_max(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return v;
}

// Inclusive sum-scan over the 64 lanes of a wave, the same DPP steps.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// Sphere: front root of |o + t D - c| = r with D = (Dx, Dy, 1), so t is the
// view depth.  Stable form: b = (c-o).D / D.D, q = (c-o) - b D,
// t = b - sqrt((r^2 - q.q) / D.D).
// The hardware reciprocal and square root (<= 1 ulp) are used throughout:
// their error is a few parts in 1e7 of the distance, far inside the 1e-5
// depth tolerance and the grazing band the oracle allows.
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// graze: the hit's n.V (the half chord sqrt(disc) over r) is below
// kGrazeCos, or the sphere is large against its depth (r > z / 4): where the
// FP32 root may miss the depth tolerance (see kGrazeCos).
__device__ inline float hit_sphere(const float4 s, float ox, float oy, float Dx, float Dy, bool& graze) {
    const float cx = s.x - ox, cy = s.y - oy, cz = s.z;
    const float inv_dd = fast_rcp(fmaf(Dx, Dx, fmaf(Dy, Dy, 1.0f)));
    const float b = fmaf(cx, Dx, fmaf(cy, Dy, cz)) * inv_dd;
    const float qx = fmaf(-b, Dx, cx), qy = fmaf(-b, Dy, cy), qz = cz - b;
    const float disc = fmaf(s.w, s.w, -fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
    if (disc < 0.0f) return INFINITY;
    const float t = b - fast_sqrt(disc * inv_dd);
    graze = disc < kGrazeCos * kGrazeCos * (s.w * s.w) || 4.0f * s.w > t;
    return t;
}

// Closed cylinder of radius rho from A along unit axis a for length L: the
// entry point is the lateral front root with 0 <= s <= L, or the plane hit of
// the cap the ray enters through (cap A when D.a > 0, cap B when D.a < 0) if
// it lies within rho of the axis.
__device__ inline float hit_cylinder(const float4 ca, const float4 cb, float ox, float oy, float Dx,
                                     float Dy) {
    const float wx = ox - ca.x, wy = oy - ca.y, wz = -ca.z;
    const float rho2 = ca.w * ca.w;
    const float da = fmaf(Dx, cb.x, fmaf(Dy, cb.y, cb.z));
    const float wa = fmaf(wx, cb.x, fmaf(wy, cb.y, wz * cb.z));
    const float px = fmaf(-da, cb.x, Dx), py = fmaf(-da, cb.y, Dy), pz = fmaf(-da, cb.z, 1.0f);
    const float qx = fmaf(-wa, cb.x, wx), qy = fmaf(-wa, cb.y, wy), qz = fmaf(-wa, cb.z, wz);
    const float k = fmaf(px, px, fmaf(py, py, pz * pz));
    float t = INFINITY;
    if (k > 0.0f) {
        const float inv_k = fast_rcp(k);
        const float tc = -fmaf(qx, px, fmaf(qy, py, qz * pz)) * inv_k;
        const float rx = fmaf(tc, px, qx), ry = fmaf(tc, py, qy), rz = fmaf(tc, pz, qz);
        const float disc = rho2 - fmaf(rx, rx, fmaf(ry, ry, rz * rz));
        if (disc >= 0.0f) {
            const float ts = tc - fast_sqrt(disc * inv_k);
            const float s = fmaf(ts, da, wa);
            if (s >= 0.0f && s <= cb.w) t = ts;
        }
    }
    if (da != 0.0f) {
        const float tp = (da > 0.0f ? -wa : cb.w - wa) * fast_rcp(da);
        const float off = da > 0.0f ? 0.0f : cb.w;
        const float ex = fmaf(tp, Dx, wx) - off * cb.x;
        const float ey = fmaf(tp, Dy, wy) - off * cb.y;
        const float ez = (tp + wz) - off * cb.z;
        if (fmaf(ex, ex, fmaf(ey, ey, ez * ez)) <= rho2) t = fminf(t, tp);
    }
    return t;
}

// Depth of primitive `id` at pixel (px, py), recomputed in FP64 from the
// caller's FP32 inputs.  The FP32 ray test decides which primitive a pixel
// shows; its depth is only good to a few ulps of the distance divided by n.V,
// so towards a silhouette it drifts past any fixed relative tolerance (at
// n.V = 0.01 about 1e-5 of the depth).  The FP64 root loses the same digits
// relative to 2^-53, and rounding it once gives the depth to half an FP32 ulp
// wherever the hit is not within ~1e-7 of grazing.  Where FP64 finds no
// entry (an FP32 hit at the silhouette that FP64 places just outside), the
// depth is the surface's closest approach to the ray: the front root with
// the discriminant taken as zero, or the cap plane's crossing, whichever is
// nearest the FP32 depth.
__device__ inline float refine_depth_at(const Frame& F, const global_t<const float>* __restrict__ pos,
                                       const global_t<const float>* __restrict__ rad,
                                       const global_t<const uint32_t>* __restrict__ bonds, uint32_t id, int px, int py,
                                       float z32) {
    const double ndx = fma((double)px + 0.5, F.inv_w2d, -1.0);
    const double ndy = fma(-((double)py + 0.5), F.inv_h2d, 1.0);
    // ray o + t D with D.z = 1, so t is the view depth
    double ox = 0.0, oy = 0.0, Dx = 0.0, Dy = 0.0;
    if (F.proj == 0) {
        Dx = ndx * F.tx;
        Dy = ndy * F.ty;
    } else {
        ox = ndx * F.hx;
        oy = ndy * F.hy;
    }
    const double dd = fma(Dx, Dx, fma(Dy, Dy, 1.0)), idd = 1.0 / dd;
    double t = (double)z32;
    if (id < F.n_atoms) {
        const size_t i = id;
        double cx, cy, cz;
        to_view(F, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], cx, cy, cz);
        const double r = (double)atom_radius(F, rad[i]);
        cx -= ox;
        cy -= oy;
        const double b = fma(cx, Dx, fma(cy, Dy, cz)) * idd;
        const double qx = fma(-b, Dx, cx), qy = fma(-b, Dy, cy), qz = cz - b;
        const double disc = fma(r, r, -fma(qx, qx, fma(qy, qy, qz * qz)));
        t = b - sqrt(fmax(disc, 0.0) * idd);
    } else {
        const size_t bi = id - F.n_atoms;
        const uint32_t ia = bonds[2 * bi], ib = bonds[2 * bi + 1];
        double A[3], B[3];
        to_view(F, pos[3 * (size_t)ia], pos[3 * (size_t)ia + 1], pos[3 * (size_t)ia + 2], A[0], A[1], A[2]);
        to_view(F, pos[3 * (size_t)ib], pos[3 * (size_t)ib + 1], pos[3 * (size_t)ib + 2], B[0], B[1], B[2]);
        const double rho = (double)F.bond_radius;
        double ax = B[0] - A[0], ay = B[1] - A[1], az = B[2] - A[2];
        const double L = sqrt(fma(ax, ax, fma(ay, ay, az * az)));
        ax /= L;
        ay /= L;
        az /= L;
        const double wx = ox - A[0], wy = oy - A[1], wz = -A[2];
        const double da = fma(Dx, ax, fma(Dy, ay, az)), wa = fma(wx, ax, fma(wy, ay, wz * az));
        const double px_ = fma(-da, ax, Dx), py_ = fma(-da, ay, Dy), pz_ = fma(-da, az, 1.0);
        const double qx = fma(-wa, ax, wx), qy = fma(-wa, ay, wy), qz = fma(-wa, az, wz);
        const double k = fma(px_, px_, fma(py_, py_, pz_ * pz_));
        double entry = INFINITY, near = INFINITY;
        auto consider = [&](double tt, bool valid) {
            if (valid) entry = fmin(entry, tt);
            if (fabs(tt - (double)z32) < fabs(near - (double)z32)) near = tt;
        };
        if (k > 0.0) {
            const double tc = -fma(qx, px_, fma(qy, py_, qz * pz_)) / k;
            const double rx = fma(tc, px_, qx), ry = fma(tc, py_, qy), rz = fma(tc, pz_, qz);
            const double disc = fma(rho, rho, -fma(rx, rx, fma(ry, ry, rz * rz)));
            const double ts = tc - sqrt(fmax(disc, 0.0) / k);
            const double s = fma(ts, da, wa);
            consider(ts, disc >= 0.0 && s >= 0.0 && s <= L);
        }
        if (da != 0.0) {
            const double cap[2] = {0.0, L};
            for (int c = 0; c < 2; ++c) {
                const double tp = (cap[c] - wa) / da;
                const double ex = fma(tp, Dx, wx) - cap[c] * ax, ey = fma(tp, Dy, wy) - cap[c] * ay,
                             ez = (tp + wz) - cap[c] * az;
                const bool front = c == 0 ? da > 0.0 : da < 0.0;
                consider(tp, front && fma(ex, ex, fma(ey, ey, ez * ez)) <= rho * rho);
            }
        }
        t = entry < INFINITY ? entry : near;
    }
    const float z = (float)t;
    return z > 0.0f && z < INFINITY ? z : z32;
}

__device__ inline float refine_depth(const Job& J, uint32_t id, int px, int py, float z32) {
    return refine_depth_at(J.F, to_global(J.pos), to_global(J.rad), to_global(J.bonds), id, px, py, z32);
}

// Expand a list record into the LDS form.
__device__ inline Rec make_rec(const Frame& F, const PrimRec& p) {
    Rec r;
    r.id = p.g1.z;
    r.rect = p.g1.w;
    r.inv_w = __builtin_amdgcn_rcpf((float)((r.rect >> 16) & 0xFF));
    if (r.id < F.n_atoms) {
        r.a = p.g0;
        r.b = make_float4(0.f, 0.f, 0.f, 0.f);
        r.zcull = (p.g0.z - p.g0.w) * (1.0f - 1e-5f);
    } else {
        const float dx = p.g0.w, dy = __uint_as_float(p.g1.x), dz = __uint_as_float(p.g1.y);
        const float L = fast_sqrt(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        const float inv = fast_rcp(L);
        const float rho = F.bond_radius;
        r.a = make_float4(p.g0.x, p.g0.y, p.g0.z, rho);
        r.b = make_float4(dx * inv, dy * inv, dz * inv, L);
        r.zcull = (fminf(p.g0.z, p.g0.z + dz) - rho) * (1.0f - 1e-5f) - 1e-6f;
    }
    return r;
}

// View-space record of a visible primitive, rebuilt from its source (the
// tile lists hold only source indices and footprints).  The count pass has
// culled it already, so the frustum test is not repeated.
__device__ inline bool source_record(const Job& J, uint32_t src, PrimRec& pr) {
    double v[6], rr;
    return item_view<false>(J.F, fetch_src(J, src), pr, v, rr);
}

// Resolves tile t of job J, whose list holds n records from offset o
// (kTail: the list overflowed and the tile is rebuilt from every binning
// workgroup's visible list).  Re-arms the tile's count and cursor for the next
// frame.  The workgroup's LDS holds the tile's depth buffer, one chunk of
// records and their prefix.  Two-pass frames: the front pass also stores the
// farthest depth of each 16x16 cell of the tile; the rest pass starts from the
// front pass's depth and id.
// kInline: the write-out recomputes the marked winners' depths in FP64 itself
// (single renders); otherwise it leaves them to the refine pass (batches,
// whose instantiations have no registers to spare for it).
template <int TS, bool kCount, bool kTail, bool kTwo, bool kInline>
__device__ inline void resolve_tile(const Job& J, int t, uint32_t n, uint64_t o, int phase_arg) {
    const int phase = kTwo ? phase_arg : (int)kPhaseAll;   // one-pass instantiations drop the two-pass code
    __shared__ unsigned long long keys[TS * TS];
    __shared__ Rec recs[kChunk];
    __shared__ uint32_t pref[kChunk + 1];
    __shared__ uint32_t wsum[kBlock / 64];
    constexpr int kHzBlocks = HzGrid<TS>::kBlocks;
    __shared__ uint32_t hz[kHzBlocks];
    __shared__ float red_lo[kBlock / 64], red_hi[kBlock / 64];
    __shared__ uint32_t bcnt[kBuckets], bbase[kBuckets];
    // resident scenes: list position where each layer starts, and the least
    // cull depth (float bits) of the layers from there on
    __shared__ uint32_t lay_start[kLayers], lay_zrest[kLayers];
    // depth-ordered chunk: record slots front to back.  Chunks resolved in
    // list order use it instead as 64 slots per wave, slot i holding j when
    // record j's first fragment is the i-th of the 64 the wave resolves
    // next, else 0 (all 0 between uses).
    __shared__ __align__(16) uint8_t ord[kChunk];

    // record slot j < kChunk, addressed with a 24-bit multiply (full rate)
    auto rec_at = [&](uint32_t j) -> const Rec& {
        return *reinterpret_cast<const Rec*>(reinterpret_cast<const char*>(recs) + __umul24(j, (uint32_t)sizeof(Rec)));
    };
    const Frame F = J.F;
    uint32_t* __restrict__ const cnt = J.bb.tile_cnt;
    const global_t<const uint2>* __restrict__ const list = to_global(J.bb.list);
    const global_t<const uint32_t>* __restrict__ const vis_src = to_global(J.bb.vis_src);
    const global_t<const uint2>* __restrict__ const vis_rect = to_global(J.bb.vis_rect);
    const uint32_t* __restrict__ const vis_cnt = J.bb.vis_cnt;
    const uint2* __restrict__ const vis_box = J.bb.vis_box;
    const uint32_t chunk = J.bb.chunk, groups = J.bb.groups;
    uint32_t* __restrict__ const fill = J.bb.tile_fill;
    Counters* const ctr = J.bb.ctr;
    global_t<float>* __restrict__ const depth = to_global(J.depth);
    global_t<uint32_t>* __restrict__ const out_id = to_global(J.id);

    const int tid = threadIdx.x, lane = __lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool stats = kCount && (F.flags & 1u) != 0;
    // counting frames (statistics, or VTX_FLAG_COUNT with the early-outs on):
    // ray tests and hits, and how often each early-out fired
    const bool counting = kCount && (F.flags & (1u | 16u)) != 0;
    unsigned long long n_tested = 0, n_hit = 0, n_hit_bond = 0, n_tested_bond = 0, n_skipped = 0, n_culled = 0;
    uint32_t n_list_stop = 0, n_chunk_stop = 0;

    {
        const int tx = t % F.tiles_x, ty = t / F.tiles_x;
        const int px0 = tx * TS, py0 = ty * TS;
        const int tw = min(TS, F.W - px0), th = min(TS, F.H - py0);
        for (int i = tid; i < TS * TS; i += kBlock) {
            unsigned long long k0 = ~0ull;
            const int ly = i / TS, lx = i - ly * TS;
            if (phase == kPhaseRest && lx < tw && ly < th) {
                const size_t p = (size_t)(py0 + ly) * F.W + (px0 + lx);
                const uint32_t id0 = out_id[p];
                if (id0 != kBackground) k0 = ((unsigned long long)__float_as_uint(depth[p]) << 32) | id0;
            }
            keys[i] = k0;
        }
        if (tid < kChunk / 4) reinterpret_cast<uint32_t*>(ord)[tid] = 0u;
        const uint64_t nsrc = kTail ? (uint64_t)groups * chunk : n;
        const bool persp = F.proj == 0;
        __syncthreads();
        // every wave has read the tile's count (it sets the trip count of the
        // barrier loop below): re-arm it for the next frame's count kernel
        if (tid == 0) cnt[t] = 0;
        if ((uint32_t)tid < J.bb.layers) fill[(size_t)tid * F.tiles_x * F.tiles_y + t] = 0;

        // one (record, pixel) ray test folded into the tile's LDS depth buffer
        auto test_pixel = [&](const Rec& rc, int lx, int ly) {
            const int slot = ly * TS + lx;
            if (!stats) {
                const unsigned long long cur = keys[slot];
                if (__uint_as_float((uint32_t)(cur >> 32)) < rc.zcull) {
                    if (counting) n_skipped += 1;
                    return;
                }
            }
            const float ndx = fmaf((float)(px0 + lx) + 0.5f, F.inv_w2, -1.0f);
            const float ndy = fmaf(-((float)(py0 + ly) + 0.5f), F.inv_h2, 1.0f);
            float ox, oy, Dx, Dy;
            if (persp) {
                ox = 0.f; oy = 0.f; Dx = ndx * F.txf; Dy = ndy * F.tyf;
            } else {
                ox = ndx * F.hxf; oy = ndy * F.hyf; Dx = 0.f; Dy = 0.f;
            }
            // cylinder hits are always refined; sphere hits only when grazing
            bool graze = true;
            const bool sphere = rc.id < F.n_atoms;   // ids past the atoms are bonds
            const float z = sphere ? hit_sphere(rc.a, ox, oy, Dx, Dy, graze)
                                         : hit_cylinder(rc.a, rc.b, ox, oy, Dx, Dy);
            bool hit = z >= F.znear && z <= F.zfar;
            // clip plane: the hit point (ox + z Dx, oy + z Dy, z) on the cut side draws nothing
            if (F.clip_on && hit)
                hit = fmaf(F.clip[0], fmaf(z, Dx, ox), fmaf(F.clip[1], fmaf(z, Dy, oy), fmaf(F.clip[2], z, F.clip[3]))) >= 0.0f;
            if (counting) {
                n_tested += 1;
                n_tested_bond += sphere ? 0 : 1;
                n_hit += hit ? 1 : 0;
                n_hit_bond += (hit && !sphere) ? 1 : 0;
            }
            if (hit)
                atomicMin(&keys[slot], ((unsigned long long)__float_as_uint(z) << 32) |
                                           (rc.id | (graze && F.refine_flag ? kRefineBit : 0u)));
        };
        // entry k of the visible lists (tiles whose list overflowed): the
        // record is rebuilt from its source
        auto fetch_overflow = [&](uint64_t k, PrimRec& pr) -> bool {
            if constexpr (!kTail) return false;
            const uint32_t g = (uint32_t)(k / chunk);
            if ((uint32_t)(k - (uint64_t)g * chunk) >= vis_cnt[g]) return false;
            const uint2 gb = vis_box[g];    // skip workgroups whose primitives cannot touch this tile
            if (tx < (int)(gb.x & 0xFFFF) || tx > (int)(gb.y & 0xFFFF) || ty < (int)(gb.x >> 16) ||
                ty > (int)(gb.y >> 16))
                return false;
            const uint2 r = vis_rect[k];
            const int x0 = max((int)(r.x & 0xFFFF), px0) - px0, y0 = max((int)(r.x >> 16), py0) - py0;
            const int x1 = min((int)(r.y & 0xFFFF), px0 + TS - 1) - px0;
            const int y1 = min((int)(r.y >> 16), py0 + TS - 1) - py0;
            if (x0 > x1 || y0 > y1) return false;
            if (!source_record(J, vis_src[k], pr)) return false;
            pr.g1.w = (uint32_t)x0 | ((uint32_t)y0 << 8) | ((uint32_t)(x1 - x0 + 1) << 16) |
                      ((uint32_t)(y1 - y0 + 1) << 24);
            return true;
        };

        // hz[b]: float bits of the farthest depth held by 4x4-pixel block b
        // (+inf while any of its pixels is empty).  It only decreases during
        // the frame, so a stale value is a safe bound.
        for (int i = tid; i < kHzBlocks; i += kBlock) hz[i] = 0x7F800000u;
        // The tile's list is staged 256 records at a time; the next chunk's
        // records are loaded while this chunk is resolved.
        // A list's next chunk is loaded while this one is resolved; the
        // overflow path loads each chunk when it starts.
        uint2 nxt = make_uint2(0u, 0u);
        bool nxt_ok = !kTail && (uint64_t)tid < nsrc;
        if (nxt_ok) nxt = list[o + tid];
        __syncthreads();
        // record cull against the block depths: its nearest possible depth
        // lies behind everything the 4x4 blocks under its footprint hold
        auto hz_culled = [&](const Rec& rc) -> bool {
            const int x0 = (int)(rc.rect & 0xFF), y0 = (int)((rc.rect >> 8) & 0xFF);
            const int x1 = x0 + (int)((rc.rect >> 16) & 0xFF) - 1, y1 = y0 + (int)(rc.rect >> 24) - 1;
            uint32_t m = 0;
            for (int by = y0 >> 2; by <= (y1 >> 2); ++by)
                for (int bx = x0 >> 2; bx <= (x1 >> 2); ++bx) m = max(m, hz[by * (TS / 4) + bx]);
            return __float_as_uint(rc.zcull) > m && rc.zcull > 0.0f;
        };
        auto rect_area = [](uint32_t rect) -> uint32_t { return ((rect >> 16) & 0xFF) * (rect >> 24); };
        // farthest depth (float bits) that 4 pixels of row r of 4x4 block
        // (bx, by) hold: +inf while one is empty; pixels outside the image
        // never hold a hit and do not bound the block
        auto row_zmax = [&](int bx, int by, int r) -> uint32_t {
            const int ly = by * 4 + r;
            uint32_t m = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int lx = bx * 4 + c;
                const unsigned long long kk = keys[ly * TS + lx];
                const uint32_t zb = (lx < tw && ly < th) ? (kk == ~0ull ? 0x7F800000u : (uint32_t)(kk >> 32)) : 0u;
                m = max(m, zb);
            }
            return m;
        };
        // refresh every block depth from the tile's depth buffer (the whole
        // workgroup, after its writes): four lanes per block, one row each
        auto hz_refresh = [&]() {
            for (int u = tid; u < kHzBlocks * 4; u += kBlock) {
                const int b = u >> 2;
                uint32_t m = row_zmax(b % (TS / 4), b / (TS / 4), u & 3);
                m = max(m, (uint32_t)__shfl_xor((int)m, 1));
                m = max(m, (uint32_t)__shfl_xor((int)m, 2));
                if ((u & 3) == 0) hz[b] = m;
            }
            __syncthreads();
        };
        // exclusive prefix of per-thread fragment counts `a` over the
        // workgroup into pref[0..kChunk]; the high bits of `a` may carry a
        // second count (kept records), summed alongside: returns the packed total
        auto block_scan = [&](uint32_t a) -> uint32_t {
            const uint32_t incl = wave_incl_scan(a);
            if (lane == 63) wsum[wave] = incl;
            __syncthreads();
            uint32_t wb = 0, tot = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                wb += w < wave ? wsum[w] : 0u;
                tot += wsum[w];
            }
            pref[tid] = (wb + incl - a) & kAreaMask;
            if (tid == kBlock - 1) pref[kChunk] = tot & kAreaMask;
            __syncthreads();
            return tot;
        };
        // fragments f of the chunk's records recs[j] with prefix pref.
        // Each wave takes an equal contiguous share and resolves it 64
        // consecutive fragments at a time (neighbouring pixels of a few
        // adjacent records, so early-out decisions agree across the wave).
        // The owner of a fragment is the last record starting at or before
        // it: one search finds it for the share's first fragment; after
        // that the records starting within each step mark their first
        // fragment in the wave's slots, and a max-scan over the lanes,
        // seeded with the previous owner, gives every lane its record.
        auto resolve_fragments = [&]() {
            constexpr int span = kChunk;
            const uint32_t total = pref[kChunk];
            const uint32_t share = (total + kBlock - 1) / kBlock * 64;
            const uint32_t q0 = min(total, (uint32_t)wave * share), q1 = min(total, q0 + share);
            if (q0 < q1) {
                int lo = 0, hi = span;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (pref[mid] <= q0) lo = mid;
                    else hi = mid;
                }
                uint32_t own = (uint32_t)__builtin_amdgcn_readfirstlane(lo);
                uint8_t* const st = ord + wave * 64;
                for (uint32_t f0 = q0; f0 < q1; f0 += 64) {
                    // records after `own` start at or after f0, in order: mark
                    // those with fragments that start before f0 + 64
                    for (uint32_t j0 = own + 1;; j0 += 64) {
                        const uint32_t j = j0 + (uint32_t)lane;
                        uint32_t e = ~0u;
                        bool some = false;
                        if (j < (uint32_t)span) {
                            e = pref[j];
                            some = pref[j + 1] > e;
                        }
                        const bool in = e < f0 + 64;
                        if (in && some) st[e - f0] = (uint8_t)j;
                        if (!__all(in)) break;
                    }
                    // the wave's own LDS writes are seen by its later reads
                    __builtin_amdgcn_wave_barrier();
                    uint32_t m = st[lane];
                    if (m) st[lane] = 0;
                    m = max(wave_incl_max(m), own);
                    own = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
                    const uint32_t f = f0 + (uint32_t)lane;
                    if (f < q1) {
                        const Rec& rr = rec_at(m);
                        const uint32_t local = f - pref[m];
                        const uint32_t rw = (rr.rect >> 16) & 0xFF;
                        // exact: local < 4096 and rw <= 64, so the rounding error of
                        // (local + 1/2) / rw is far below its distance to an integer
                        const uint32_t dy = (uint32_t)(((float)local + 0.5f) * rr.inv_w);
                        const uint32_t dx = local - __umul24(dy, rw);
                        test_pixel(rr, (int)(rr.rect & 0xFF) + (int)dx, (int)((rr.rect >> 8) & 0xFF) + (int)dy);
                    }
                }
            }
            __syncthreads();
        };
        // The kept records of a chunk in depth order (ord), resolved `sub`
        // at a time, front to back.  Every wave culls the sub-chunk against
        // the block depths (2 or 4 lanes per record; all waves read the same
        // depths, so they agree) and takes the prefix of the survivors'
        // footprints in its own slots; the workgroup resolves their
        // fragments, then refreshes the blocks under them before the next
        // sub-chunk is culled.
        // zlo, bstep: the depth buckets' origin and width (bucket b holds cull
        // depths from zlo + b * bstep on; bstep 0: one bucket)
        auto resolve_sorted = [&](uint32_t nk, int sub0, bool more, float zlo, float bstep) {
            // All waves compute the same prefix (from the same block depths),
            // so they share one array, the chunk's prefix, which is no longer
            // needed: every wave writes it whole before reading it.
            uint32_t* const wp = pref;
            uint32_t rbase = 0;
            for (uint32_t sc = 0; rbase < nk; ++sc) {
                if (sc > 0) {
                    // every record from rbase on lies in rbase's bucket or a later
                    // one: once that bucket's start (less a rounding margin) is
                    // behind every block depth of the tile, all of them would be
                    // culled.  Every wave reads the same LDS: a uniform decision.
                    const unsigned long long in = __ballot(lane < kBuckets && bbase[lane] <= rbase);
                    const float zb = fmaf((float)(63 - __clzll((long long)in)), bstep, zlo);
                    const float bound = zb - 1e-5f * (fabsf(zlo) + fabsf(zb));
                    uint32_t mt = 0;
                    for (int b = lane; b < kHzBlocks; b += 64) mt = max(mt, hz[b]);
                    mt = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(mt), 63);
                    if (bound > 0.0f && __float_as_uint(bound) > mt) {
                        if (counting && tid == 0) ++n_chunk_stop;
                        break;
                    }
                }
                // later sub-chunks stay small too: the finer the steps, the
                // sooner the bucket bound above ends the chunk
                const int sub = sc == 0 ? sub0 : kLaterSub;
                const int lg = sub == 4 ? 4 : sub == 8 ? 3 : sub == 16 ? 2 : sub == 32 ? 1 : 0;   // log2 of the lanes per record
                const uint32_t i = (uint32_t)lane >> lg;
                const bool real = rbase + i < nk;
                uint32_t rect = 0;
                float zcull = 0.0f;
                if (real) {
                    const Rec& r = recs[ord[rbase + i]];
                    rect = r.rect;
                    zcull = r.zcull;
                }
                const int bx0 = (int)(rect & 0xFF) >> 2, by0 = (int)((rect >> 8) & 0xFF) >> 2;
                const int bx1 = ((int)(rect & 0xFF) + (int)((rect >> 16) & 0xFF) - 1) >> 2;
                const int by1 = ((int)((rect >> 8) & 0xFF) + (int)(rect >> 24) - 1) >> 2;
                // the first sub-chunk was culled with the chunk, against the
                // same block depths
                uint32_t m = 0;
                if (real && sc > 0)
                    for (int by = by0 + (lane & ((1 << lg) - 1)); by <= by1; by += 1 << lg)
                        for (int bx = bx0; bx <= bx1; ++bx) m = max(m, hz[by * (TS / 4) + bx]);
                if (lg >= 1) m = max(m, (uint32_t)__shfl_xor((int)m, 1));
                if (lg >= 2) m = max(m, (uint32_t)__shfl_xor((int)m, 2));
                if (lg >= 3) m = max(m, (uint32_t)__shfl_xor((int)m, 4));
                if (lg >= 4) m = max(m, (uint32_t)__shfl_xor((int)m, 8));
                const bool live = real && !(sc > 0 && __float_as_uint(zcull) > m && zcull > 0.0f);
                // every wave takes the same decisions: wave 0 counts them, one lane per record
                if (counting && wave == 0 && real && !live && (lane & ((1 << lg) - 1)) == 0) n_culled += 1;
                // blocks under the live records (their union rectangle)
                const uint32_t ux0 = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(live ? 255u - bx0 : 0u), 63);
                const uint32_t uy0 = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(live ? 255u - by0 : 0u), 63);
                const uint32_t ux1 = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(live ? bx1 + 1u : 0u), 63);
                const uint32_t uy1 = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(live ? by1 + 1u : 0u), 63);
                // record i's footprint to lane i, then its prefix
                const uint32_t ag = (uint32_t)__shfl((int)(live ? rect_area(rect) : 0u), (lane << lg) & 63);
                const uint32_t incl = wave_incl_scan(lane < sub ? ag : 0u);
                if (lane < sub) wp[lane + 1] = incl;
                if (lane == 0) wp[0] = 0u;
                const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, sub - 1);
                __builtin_amdgcn_wave_barrier();
                for (uint32_t f = (uint32_t)tid; f < total; f += kBlock) {
                    int lo = 0, hi = sub;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (wp[mid] <= f) lo = mid;
                        else hi = mid;
                    }
                    const Rec& rr = rec_at(ord[rbase + (uint32_t)lo]);
                    const uint32_t local = f - wp[lo];
                    const uint32_t rw = (rr.rect >> 16) & 0xFF;
                    const uint32_t dy = (uint32_t)(((float)local + 0.5f) * rr.inv_w);
                    const uint32_t dx = local - __umul24(dy, rw);
                    test_pixel(rr, (int)(rr.rect & 0xFF) + (int)dx, (int)((rr.rect >> 8) & 0xFF) + (int)dy);
                }
                rbase += (uint32_t)sub;
                if (rbase >= nk && !more) break;
                __syncthreads();   // the sub-chunk's hits are in the depth buffer
                if (ux1 > 0) {
                    const int cx0 = 255 - (int)ux0, cy0 = 255 - (int)uy0;
                    const int bw = (int)ux1 - cx0, nb = bw * ((int)uy1 - cy0);
                    for (int k = tid; k < 4 * nb; k += kBlock) {
                        const int b = k >> 2, by = cy0 + b / bw, bx = cx0 + b % bw;
                        uint32_t z = row_zmax(bx, by, k & 3);
                        z = max(z, (uint32_t)__shfl_xor((int)z, 1));
                        z = max(z, (uint32_t)__shfl_xor((int)z, 2));
                        if ((k & 3) == 0) hz[by * (TS / 4) + bx] = z;
                    }
                }
                __syncthreads();   // refreshed block depths are in LDS
            }
        };
        // Layered lists (resident scenes) run front to back by layer: once
        // every record from a layer on lies behind all block depths of the
        // tile, the rest of the list is culled whole, unread.
        const uint32_t L = kTail || stats || n <= (uint32_t)kChunk ? 1u : J.bb.layers;   // one chunk: nothing to stop
        if (L > 1 && wave == 0) {
            uint32_t zr = lane < (int)L ? ctr->layer_zlo[phase == kPhaseRest ? 1 : 0][lane] : 0x7F800000u;
#pragma unroll
            for (int o2 = 1; o2 < 32; o2 <<= 1) {
                const uint32_t u = (uint32_t)__shfl_down((int)zr, o2);
                if (lane + o2 < 64) zr = min(zr, u);
            }
            if (lane < (int)L) {
                lay_zrest[lane] = zr;
                lay_start[lane] = J.bb.layer_off[(size_t)lane * F.tiles_x * F.tiles_y + t];
            }
        }
        bool hz_set = false;   // the block depths hold a refresh (uniform)
        if (phase == kPhaseRest) {
            hz_refresh();   // the front pass's depths bound the blocks from the start
            hz_set = true;
        }
        for (uint64_t base = 0; base < nsrc; base += kChunk) {
            if (L > 1 && hz_set) {
                // every wave reads the same LDS after the last barrier: a uniform decision
                uint32_t m = 0;
                for (int i = lane; i < kHzBlocks; i += 64) m = max(m, hz[i]);
                m = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(m), 63);
                const unsigned long long started = __ballot(lane < (int)L && lay_start[lane] <= (uint32_t)base);
                const uint32_t zr = lay_zrest[63 - __clzll((long long)started)];
                if (zr > m && zr != 0u) {
                    if (counting && tid == 0) ++n_list_stop;
                    break;
                }
            }
            PrimRec pr;
            bool have;
            if constexpr (kTail) {
                have = base + tid < nsrc && fetch_overflow(base + tid, pr);
            } else {
                const uint2 e = nxt;
                have = nxt_ok && source_record(J, e.x, pr);
                pr.g1.w = e.y;
                nxt_ok = base + kChunk + tid < nsrc;
                if (nxt_ok) nxt = list[o + base + kChunk + tid];
            }
            bool keep = false;
            uint32_t area = 0;
            float zc = INFINITY;
            if (have) {
                const Rec rc = make_rec(F, pr);
                // until a refresh has stored depths every block is +inf: nothing to test
                keep = stats || !hz_set || !hz_culled(rc);
                if (counting && !keep) n_culled += 1;
                if (keep) {
                    area = rect_area(rc.rect);
                    zc = rc.zcull;
                    recs[tid] = rc;
                }
            }
            const bool more = base + kChunk < nsrc;
            // prefix of the footprint areas, with the kept records counted in
            // the high bits
            const uint32_t packed = block_scan(area | (keep ? 1u << kKeptShift : 0u));
            const uint32_t atot = packed & kAreaMask, nk = packed >> kKeptShift;
            // Large footprints (many records cover each pixel): order the
            // kept records front to back by a counting sort over depth
            // buckets and resolve them in sub-chunks, refreshing the block
            // depths in between, so records behind the first layers are
            // culled whole before any of their pixels is tested.  Sub-chunks
            // are small (8 records): the block depths are refreshed, and the
            // bucket bound can end the chunk, after every few records.
            const int sub = atot >= 64u * nk ? 8 : 32;
            const bool sorted = !stats && nk > (uint32_t)sub && atot > (uint32_t)kSortArea * nk;
            if (!sorted) {
                resolve_fragments();
                if (!stats && more) {
                    hz_refresh();
                    hz_set = true;
                }
                continue;
            }
            // depth range of the kept records
            float zlo = zc, zhi = keep ? zc : -INFINITY;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                zlo = fminf(zlo, __shfl_xor(zlo, o));
                zhi = fmaxf(zhi, __shfl_xor(zhi, o));
            }
            if (lane == 0) {
                red_lo[wave] = zlo;
                red_hi[wave] = zhi;
            }
            if (tid < kBuckets) bcnt[tid] = 0u;
            __syncthreads();
            zlo = fminf(fminf(red_lo[0], red_lo[1]), fminf(red_lo[2], red_lo[3]));
            zhi = fmaxf(fmaxf(red_hi[0], red_hi[1]), fmaxf(red_hi[2], red_hi[3]));
            const float span = zhi - zlo;
            const float scale = span > 0.0f ? (float)kBuckets / span : 0.0f;
            const int bk = keep ? min(kBuckets - 1, (int)((zc - zlo) * scale)) : 0;
            if (keep) atomicAdd(&bcnt[bk], 1u);
            __syncthreads();
            if (wave == 0) {
                const uint32_t c = lane < kBuckets ? bcnt[lane] : 0u;
                const uint32_t inc = wave_incl_scan(c);
                if (lane < kBuckets) {
                    bbase[lane] = inc - c;
                    bcnt[lane] = 0u;
                }
            }
            __syncthreads();
            if (keep) ord[bbase[bk] + atomicAdd(&bcnt[bk], 1u)] = (uint8_t)tid;
            __syncthreads();   // the order is in LDS
            resolve_sorted(nk, sub, more, zlo, span > 0.0f ? span * (1.0f / (float)kBuckets) : 0.0f);
            hz_set = true;
            __syncthreads();   // every wave is done with this chunk's records
            if (tid < kChunk / 4) reinterpret_cast<uint32_t*>(ord)[tid] = 0u;
        }
        __syncthreads();
        if constexpr (TS >= kHzCell) {
            if (phase == kPhaseFront) {
                // farthest depth of each 16x16 cell of the tile, for the rest
                // pass's cluster test (cells past the image edge are not stored)
                hz_refresh();
                constexpr int kCells = TS / kHzCell, kSub = kHzCell / 4;
                if (tid < kCells * kCells) {
                    const int cy = tid / kCells, cx = tid - cy * kCells;
                    const int gx = tx * kCells + cx, gy = ty * kCells + cy;
                    if (gx < J.bb.hz16_w && gy < (F.H + kHzCell - 1) / kHzCell) {
                        uint32_t m = 0;
                        for (int by = 0; by < kSub; ++by)
                            for (int bx = 0; bx < kSub; ++bx) m = max(m, hz[(cy * kSub + by) * (TS / 4) + cx * kSub + bx]);
                        J.bb.hz16[(size_t)gy * J.bb.hz16_w + gx] = m;
                    }
                }
            }
        }

        // The G-buffer: the winner of each pixel.  Inline, the last pass
        // writes the marked winners' depths recomputed in FP64 and plain ids;
        // otherwise (and in the front pass of a two-pass frame, which the
        // rest pass continues from) the FP32 depth and the id with its refine
        // mark, for the refine pass.
        const bool finish = kInline && phase != kPhaseFront;
#pragma unroll 1
        for (int i = tid; i < TS * TS; i += kBlock) {
            const int ly = i / TS, lx = i - ly * TS;
            if (lx < tw && ly < th) {
                const unsigned long long kk = keys[i];
                const size_t p = (size_t)(py0 + ly) * F.W + (px0 + lx);
                float zo = INFINITY;
                uint32_t io = kBackground;
                if (kk != ~0ull) {
                    io = (uint32_t)(kk & 0xFFFFFFFFull);
                    zo = __uint_as_float((uint32_t)(kk >> 32));
                    if (finish) {
                        const bool marked = !F.refine_flag || (io & kRefineBit);
                        io &= F.refine_flag ? ~kRefineBit : ~0u;
                        if (marked) zo = refine_depth(J, io, px0 + lx, py0 + ly, zo);
                    }
                }
                depth[p] = zo;
                out_id[p] = io;
            }
        }
    }
    if (counting) {
        unsigned long long a = n_tested, b = n_hit, c = n_hit_bond, d = n_tested_bond, e = n_skipped, g = n_culled;
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
            a += __shfl_xor(a, o2);
            b += __shfl_xor(b, o2);
            c += __shfl_xor(c, o2);
            d += __shfl_xor(d, o2);
            e += __shfl_xor(e, o2);
            g += __shfl_xor(g, o2);
        }
        if (lane == 0) {
            if (a) {
                atomicAdd(&ctr->frag_tested, a);
                atomicAdd(&ctr->frag_hit, b);
                atomicAdd(&ctr->frag_hit_bond, c);
                atomicAdd(&ctr->frag_tested_bond, d);
            }
            if (e) atomicAdd(&ctr->frag_skipped, e);
            if (g) atomicAdd(&ctr->rec_culled, g);
        }
        if (tid == 0 && n_list_stop) atomicAdd(&ctr->lists_stopped, (unsigned long long)n_list_stop);
        if (tid == 0 && n_chunk_stop) atomicAdd(&ctr->chunks_stopped, (unsigned long long)n_chunk_stop);
    }
}

// Main launch: work block t of a job is that job's tile t, so consecutive
// tiles go to different XCDs (the dispatcher deals blocks round-robin).  The
// costly tiles lie together, around the footprints of the nearest atoms:
// contiguous tile ranges per XCD left one XCD with most of them (20 % longer
// on the whole-cell frame).  A tile whose list overflowed the bins
// is left to the tail launch: it is appended to `ovf` (job << 32 | tile).
// kCount: the instantiation that can count fragments (jobs with
// VTX_FLAG_STATS); the other one carries no counters.
// kTwo: the instantiation for the passes of a two-pass frame.
template <int TS, class JS, bool kCount, bool kTwo>
__global__ void __launch_bounds__(kBlock, kCount ? 1 : 7) k_resolve(JS js, unsigned long long* ovf, uint32_t* ovf_n,
                                                                     int phase) {
    uint32_t tu;
    const int ji = js.find(blockIdx.x, tu);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const uint32_t n = J.bb.tile_cnt[tu];
    const uint64_t o = J.bb.tile_off[tu];
    if (o + n > J.bb.capacity) {
        if (threadIdx.x == 0) ovf[atomicAdd(ovf_n, 1u)] = ((unsigned long long)ji << 32) | tu;
        return;
    }
    resolve_tile<TS, kCount, false, kTwo, !JS::kMany>(J, (int)tu, n, o, phase);
}

// Tail launch (a fixed grid, queued right after the main one): resolves the
// overflowed tiles the main launch listed, then its last workgroup clears the
// list and publishes the fragment counters of every counting job.  Keeping the
// rare overflow path out of the main instantiation keeps its register budget.
template <int TS, class JS, bool kCount, bool kTwo>
__global__ void __launch_bounds__(kBlock) k_resolve_tail(JS js, const unsigned long long* ovf, uint32_t* ovf_n,
                                                          int phase) {
    const uint32_t total = *(volatile uint32_t*)ovf_n;
    for (uint32_t e = blockIdx.x; e < total; e += gridDim.x) {
        const unsigned long long v = ovf[e];
        const Job& J = js.job((int)(v >> 32));
        const int t = (int)(v & 0xFFFFFFFFull);
        resolve_tile<TS, kCount, true, kTwo, !JS::kMany>(J, t, J.bb.tile_cnt[t], J.bb.tile_off[t], phase);
        __syncthreads();   // the next tile reuses the LDS
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int ticket = atomicAdd(&ovf_n[1], 1u);
        if (ticket == gridDim.x - 1) {
            __threadfence();
            ovf_n[0] = 0;
            ovf_n[1] = 0;
            if (kCount) {
                for (uint32_t j = 0; j < js.count(); ++j) {
                    const Job& Jj = js.job((int)j);
                    if (!(Jj.F.flags & (1u | 16u)) || !Jj.bb.host_ctr) continue;
                    const volatile Counters* src = Jj.bb.ctr;
                    Jj.bb.host_ctr->frag_tested = src->frag_tested;
                    Jj.bb.host_ctr->frag_hit = src->frag_hit;
                    Jj.bb.host_ctr->frag_hit_bond = src->frag_hit_bond;
                    Jj.bb.host_ctr->frag_tested_bond = src->frag_tested_bond;
                    Jj.bb.host_ctr->frag_skipped = src->frag_skipped;
                    Jj.bb.host_ctr->rec_culled = src->rec_culled;
                    Jj.bb.host_ctr->lists_stopped = src->lists_stopped;
                    Jj.bb.host_ctr->chunks_stopped = src->chunks_stopped;
                }
            }
            __threadfence_system();
        }
    }
}


}  // namespace

template <int TS, class JS, bool kCount>
hipError_t resolve_launch(const JS& js, int phase, unsigned g, unsigned long long* ovf, uint32_t* ovf_n,
                          hipStream_t stream) {
    hipError_t e;
    if constexpr (!kCount && TS >= kHzCell) {
        if (phase != kPhaseAll) {
            if ((e = dispatch(k_resolve<TS, JS, false, true>, g, kBlock, 0, stream, js, ovf, ovf_n, phase)))
                return e;
            return dispatch(k_resolve_tail<TS, JS, false, true>, kTailBlocks, kBlock, 0, stream, js,
                            (const unsigned long long*)ovf, ovf_n, phase);
        }
    }
    if ((e = dispatch(k_resolve<TS, JS, kCount, false>, g, kBlock, 0, stream, js, ovf, ovf_n, phase))) return e;
    return dispatch(k_resolve_tail<TS, JS, kCount, false>, kTailBlocks, kBlock, 0, stream, js,
                    (const unsigned long long*)ovf, ovf_n, phase);
}

template <class JS, bool kCount>
hipError_t resolve_impl(const JS& js, int tile, int phase, uint32_t grid, unsigned long long* ovf, uint32_t* ovf_n,
                        hipStream_t stream) {
    if (grid == 0) return hipSuccess;
    if (phase != kPhaseAll && (kCount || tile < kHzCell)) return hipErrorInvalidValue;
    const unsigned g = (unsigned)xcd_grid((int)grid);
    switch (tile) {
        case 8: return resolve_launch<8, JS, kCount>(js, phase, g, ovf, ovf_n, stream);
        case 16: return resolve_launch<16, JS, kCount>(js, phase, g, ovf, ovf_n, stream);
        case 32: return resolve_launch<32, JS, kCount>(js, phase, g, ovf, ovf_n, stream);
        case 64: return resolve_launch<64, JS, kCount>(js, phase, g, ovf, ovf_n, stream);
        default: return hipErrorInvalidValue;
    }
}

// Depth refinement of a batch, over the shade's 16x16 blocks, kRefineBlocks
// of them per workgroup: a pixel whose winner the resolve marked (kRefineBit
// in the id, or every hit when the frame has too many primitives for the
// mark) gets its depth recomputed from the primitive's FP64 data
// (refine_depth) and its mark cleared; every other pixel keeps the resolve's
// FP32 depth, which is within the tolerance there (see kGrazeCos).
constexpr int kRefineBlocks = 16;   // 16x16 blocks per refine workgroup (pixels per thread in flight)

template <class JS>
__global__ void __launch_bounds__(kBlock, 6) k_refine(JS js, uint32_t nblocks) {
    __shared__ uint16_t todo[kRefineBlocks * kBlock];
    __shared__ uint32_t todo_id[kRefineBlocks * kBlock];   // the entry's id as loaded (mark included)
    __shared__ uint32_t wave_n[kBlock / 64];
    __shared__ int blk_job[kRefineBlocks];
    __shared__ uint32_t blk_tile[kRefineBlocks];
    const int tid = threadIdx.x, wave = tid >> 6;
    const uint32_t q = (uint32_t)xcd_contiguous(blockIdx.x, gridDim.x);
    // the id of this thread's pixel in each of the workgroup's blocks, all
    // loads issued before any is used
    // (one search for the first block; the others follow it)
    int ji[kRefineBlocks];
    uint32_t tu[kRefineBlocks], raw[kRefineBlocks];
    ji[0] = q * kRefineBlocks < nblocks ? js.find(q * kRefineBlocks, tu[0]) : -1;
#pragma unroll
    for (int s = 0; s < kRefineBlocks; ++s) {
        if (s > 0) {
            ji[s] = ji[s - 1];
            tu[s] = tu[s - 1];
            js.next(ji[s], tu[s]);
        }
        raw[s] = kBackground;
        if (ji[s] >= 0) {
            const Frame& F = js.job(ji[s]).F;
            const int tiles_x = (F.W + 15) / 16;
            const int x = ((int)tu[s] % tiles_x) * 16 + (tid & 15), y = ((int)tu[s] / tiles_x) * 16 + (tid >> 4);
            if (x < F.W && y < F.H) raw[s] = to_global(js.job(ji[s]).id)[(size_t)y * F.W + x];
        }
    }
    // the marked pixels, packed into a list so that only as many waves as
    // they fill run the FP64 recomputation
    uint32_t mine = 0, n_mine = 0;
#pragma unroll
    for (int s = 0; s < kRefineBlocks; ++s) {
        if (ji[s] < 0 || raw[s] == kBackground) continue;
        if (!js.job(ji[s]).F.refine_flag || (raw[s] & kRefineBit)) {
            mine |= 1u << s;
            ++n_mine;
        }
    }
    uint32_t incl = n_mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)incl, o);
        if ((int)__lane_id() >= o) incl += u;
    }
    if (__lane_id() == 63) wave_n[wave] = incl;
    if (tid < kRefineBlocks) {
        // each entry's job and block, for the threads that take it
#pragma unroll
        for (int s = 0; s < kRefineBlocks; ++s)
            if (tid == s) {
                blk_job[s] = ji[s];
                blk_tile[s] = tu[s];
            }
    }
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        before += w < wave ? wave_n[w] : 0u;
        total += wave_n[w];
    }
    uint32_t at = before + incl - n_mine;
#pragma unroll
    for (int s = 0; s < kRefineBlocks; ++s)
        if (mine & (1u << s)) {
            todo_id[at] = raw[s];
            todo[at++] = (uint16_t)(s * kBlock + tid);
        }
    __syncthreads();
    if (ji[0] >= 0 && ji[kRefineBlocks - 1] == ji[0]) {
        // all the workgroup's blocks are one job's (the usual case): block s
        // is that job's block tu[0] + s, and the job's frame is read once,
        // into scalar registers, rather than per entry
        const Job& J = js.job(__builtin_amdgcn_readfirstlane(ji[0]));
        const Frame& F = J.F;
        const global_t<const float>* __restrict__ const pos = to_global(J.pos);
        const global_t<const float>* __restrict__ const rad = to_global(J.rad);
        const global_t<const uint32_t>* __restrict__ const bonds = to_global(J.bonds);
        global_t<float>* __restrict__ const depth = to_global(J.depth);
        global_t<uint32_t>* __restrict__ const out_id = to_global(J.id);
        const int tiles_x = (F.W + 15) / 16, tb0 = __builtin_amdgcn_readfirstlane((int)tu[0]);
        for (uint32_t e = (uint32_t)tid; e < total; e += kBlock) {
            const int s = todo[e] / kBlock, t = todo[e] % kBlock;
            const int tb = tb0 + s;
            const int px = (tb % tiles_x) * 16 + (t & 15), py = (tb / tiles_x) * 16 + (t >> 4);
            const size_t p = (size_t)py * F.W + px;
            const uint32_t r0 = todo_id[e];
            const uint32_t id = F.refine_flag ? r0 & ~kRefineBit : r0;
            depth[p] = refine_depth_at(F, pos, rad, bonds, id, px, py, depth[p]);
            if (F.refine_flag) out_id[p] = id;
        }
        return;
    }
    for (uint32_t e = (uint32_t)tid; e < total; e += kBlock) {
        const int s = todo[e] / kBlock, t = todo[e] % kBlock;
        // the entry's block, one of the workgroup's (no second search)
        const int j = blk_job[s];
        const uint32_t tb = blk_tile[s];
        const Job& J = js.job(j);
        const Frame& F = J.F;
        const int tiles_x = (F.W + 15) / 16;
        const int px = ((int)tb % tiles_x) * 16 + (t & 15), py = ((int)tb / tiles_x) * 16 + (t >> 4);
        const size_t p = (size_t)py * F.W + px;
        const uint32_t r0 = todo_id[e];
        const uint32_t id = F.refine_flag ? r0 & ~kRefineBit : r0;
        global_t<float>* const depth = to_global(J.depth);
        depth[p] = refine_depth(J, id, px, py, depth[p]);
        if (F.refine_flag) to_global(J.id)[p] = id;
    }
}

// One workgroup per kRefineBlocks of the 16x16 blocks, the grid rounded up
// to whole XCD rounds as xcd_contiguous needs.
template <class JS>
hipError_t refine_impl(const JS& js, uint32_t blocks, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    const int grid = xcd_grid((int)((blocks + kRefineBlocks - 1) / kRefineBlocks));
    return dispatch(k_refine<JS>, (unsigned)grid, kBlock, 0, stream, js, blocks);
}
hipError_t launch_refine(const OneJob& js, uint32_t grid, hipStream_t stream) { return refine_impl(js, grid, stream); }
hipError_t launch_refine(const JobList& js, uint32_t grid, hipStream_t stream) { return refine_impl(js, grid, stream); }

hipError_t launch_resolve(const OneJob& js, int tile, int phase, uint32_t grid, bool count, unsigned long long* ovf,
                          uint32_t* ovf_n, hipStream_t stream) {
    return count ? resolve_impl<OneJob, true>(js, tile, phase, grid, ovf, ovf_n, stream)
                 : resolve_impl<OneJob, false>(js, tile, phase, grid, ovf, ovf_n, stream);
}
hipError_t launch_resolve(const JobList& js, int tile, int phase, uint32_t grid, bool count, unsigned long long* ovf,
                          uint32_t* ovf_n, hipStream_t stream) {
    return count ? resolve_impl<JobList, true>(js, tile, phase, grid, ovf, ovf_n, stream)
                 : resolve_impl<JobList, false>(js, tile, phase, grid, ovf, ovf_n, stream);
}

}  // namespace vtx
