// Screen-tile binning of atoms and bonds: a counting sort by tile.
//
// The paper rasterizes one screen quad per primitive and lets the fixed
// function rasterizer find the pixels it covers (Methods, "Meshless
// Representations").  Here the quad's role, a conservative footprint, becomes
// an exact tile rectangle per primitive, and the rasterizer becomes a
// counting sort of (tile, primitive) pairs:
//   count    G workgroups each own a contiguous run of primitives (resident
//            scenes: of the visible clusters in depth-class order, so the
//            workgroups run front to back): view transform (FP64), culling,
//            footprint rectangle, a compacted per-workgroup list of the
//            visible ones, and a tile histogram in LDS; the histogram row is
//            stored and its non-zero entries are added to the tile totals
//            (resident scenes: to the totals of the workgroup's layer, 1/32
//            of the workgroups), one atomic per touched tile;
//   layers   resident scenes: the per-layer totals become the start of each
//            layer's run in every tile list, and the tile totals;
//   offsets  one exclusive scan of the tile totals per job: the list offsets;
//   scatter  each workgroup reserves, per touched tile, one run of the tile's
//            list inside its layer's run (one atomic), then places its
//            primitives with LDS atomics (one per run of lanes with the same
//            tile): 8 bytes per (primitive, tile), the source index and the
//            footprint clipped to the tile.  The resolve rebuilds each record
//            from its source, so the view-space record is never written out.
// So the global atomics scale with (workgroup, touched tile) pairs rather
// than with (primitive, tile) pairs, and a resident scene's tile lists run
// roughly front to back.  Lists that would not fit the bin
// capacity are left empty; the resolve pass then finds those tiles' primitives
// in the per-workgroup visible lists, so every frame is exact whatever the
// capacity.
#include "prims.h"

namespace vtx {

namespace {

// Zeroes n words (allocation time only: afterwards every frame leaves the
// tile counts and the frame counters at zero for the next one).
__global__ void __launch_bounds__(kBlock) k_zero(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Footprint of a visible item (its view coordinates from item_view).
__device__ inline bool item_rect(const Frame& F, const Item& it, const double* v, double r, int& x0, int& y0,
                                 int& x1, int& y1) {
    if (it.kind == kAtom) return sphere_rect_fast(F, v[0], v[1], v[2], r, x0, y0, x1, y1);
    return bond_rect_fast(F, v, v + 3, r, x0, y0, x1, y1);
}

// Primitive sources of the count kernel.  Workgroup b owns items
// [0, items()) (after begin(b)) and the visible-list region
// [b * chunk, (b + 1) * chunk).
struct PlainSource {     // the caller's arrays, primitives in their given order
    const float* pos;
    const float* rad;
    const uint32_t* bonds;
    uint64_t total;
    uint32_t chunk;
    uint32_t n_atoms;
    uint64_t first, count;
    __device__ void begin(uint32_t b) {
        first = (uint64_t)b * chunk;
        count = first < total ? min((uint64_t)chunk, total - first) : 0;
    }
    __device__ uint64_t items() const { return count; }
    __device__ Item fetch(uint64_t k) const {
        return fetch_plain(to_global(pos), to_global(rad), to_global(bonds), n_atoms, first + k);
    }
};

struct SceneSource {     // a resident scene: the clusters that passed the frustum test, by depth class
    SceneDev S;
    uint32_t groups;
};

template <bool kScene>
struct SourceOf;
template <>
struct SourceOf<false> {
    __device__ static PlainSource make(const Job& J) {
        PlainSource s;
        s.pos = J.pos;
        s.rad = J.rad;
        s.bonds = J.bonds;
        s.total = (uint64_t)J.F.n_atoms + J.F.n_bonds;
        s.chunk = J.bb.chunk;
        s.n_atoms = J.F.n_atoms;
        return s;
    }
};
template <>
struct SourceOf<true> {
    __device__ static SceneSource make(const Job& J) {
        SceneSource s;
        s.S = J.S;
        s.groups = J.bb.groups;
        return s;
    }
};

// Runs of consecutive lanes whose primitives lie in the same single tile t
// (t < 0: none); Morton-ordered primitives keep them long.  For such a lane
// `head` is its run's first lane, and for a head `len` is the run's length
// (other lanes: head = the lane itself).  Branch-free: one DPP shift, one
// ballot and a few mask operations.  Every lane of the wave calls it.
__device__ inline void lane_run(int t, int& head, uint32_t& len) {
    const int lane = __lane_id();
    const int tp = __builtin_amdgcn_update_dpp(-1, t, 0x138, 0xf, 0xf, false);   // wave_shr:1: lane - 1's t
    const unsigned long long cm = __ballot(t >= 0 && lane > 0 && t == tp);     // lanes continuing a run
    head = 63 - __clzll((long long)(~cm & ((2ull << lane) - 1ull)));            // nearest non-continuing lane <= lane
    len = (uint32_t)__builtin_ctzll(~((cm >> lane) >> 1)) + 1u;                  // continuing lanes after it, + 1
}

// Adds one to the LDS counter of each lane's tile t (t < 0: nothing): one
// atomic per run of lanes with the same tile.
__device__ inline void wave_count(uint32_t* hist, int t) {
    int head;
    uint32_t len;
    lane_run(t, head, len);
    if (t >= 0 && head == (int)__lane_id()) atomicAdd(&hist[t], len);
}

// Inclusive sum over the 64 lanes of a wave by DPP row shifts and row
// broadcasts (lanes shifted in from outside a row read 0).
__device__ inline uint32_t wave_scan_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// Tile of entry i of a workgroup's histogram row: the row covers the box of
// tiles [bx0, bx0 + bw) x [by0, ...) its primitives touch, row-major.
__device__ inline int box_tile(const Frame& F, uint32_t bx0, uint32_t by0, int bw, int i) {
    const int q = i / bw;
    return ((int)by0 + q) * F.tiles_x + (int)bx0 + (i - q * bw);
}

// Rest pass of a two-pass frame: true when cluster c cannot win a pixel.
// The lower bound of the cull depth of its primitives (the bounding sphere
// of its box, widened as in the frustum test, with the margin of the
// per-primitive bound) lies behind the front pass's depth of every 16x16
// cell under the sphere's footprint; those depths only decrease later.
// Called by whole waves with a wave-uniform c: the lanes share the cells.
__device__ inline bool cluster_hidden(const Frame& F, const SceneDev& S, const BinBuffers& bb, uint32_t c) {
    const float4 lo = S.cluster_box[2 * (size_t)c], hi = S.cluster_box[2 * (size_t)c + 1];
    const float pad = c < S.atom_clusters ? (F.rep == 2 ? F.bond_radius : F.rep == 3 ? F.probe : 0.0f) : F.bond_radius;
    const double hx = 0.5 * ((double)hi.x - lo.x), hy = 0.5 * ((double)hi.y - lo.y), hz = 0.5 * ((double)hi.z - lo.z);
    double vx, vy, vz;
    to_view(F, (float)(lo.x + hx), (float)(lo.y + hy), (float)(lo.z + hz), vx, vy, vz);
    const double r = sqrt(hx * hx + hy * hy + hz * hz) + pad +
                     1e-6 * (fabs((double)lo.x) + fabs((double)lo.y) + fabs((double)lo.z) + 1.0);
    const float zlo = __double2float_rd(vz - r - 2e-5 * (fabs(vz) + r) - 2e-6);
    if (!(zlo > 0.0f)) return false;
    int x0, y0, x1, y1;
    if (!sphere_rect_fast(F, vx, vy, vz, r, x0, y0, x1, y1)) return true;   // covers no pixel of the image
    const int cx0 = x0 / kHzCell, cy0 = y0 / kHzCell, cw = x1 / kHzCell - cx0 + 1;
    const int n = cw * (y1 / kHzCell - cy0 + 1);
    if (n > 16 * 64) return false;   // a footprint this large is rarely hidden: not worth the reads
    uint32_t m = 0;
    for (int k = (int)__lane_id(); k < n; k += 64) {
        const int q = k / cw;
        m = max(m, bb.hz16[(size_t)(cy0 + q) * bb.hz16_w + (cx0 + k - q * cw)]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
    return __float_as_uint(zlo) > m;
}

// Count.  Work block b of a job is that job's binning workgroup b.
// kRest: the rest pass of a two-pass frame (a separate instantiation keeps
// the cluster test out of the others' registers).  kAtoms: a scene without
// bonds (no bond path in the loop: fewer live registers).
template <class JS, bool kScene, bool kRest, bool kAtoms = false>
__global__ void __launch_bounds__(kBinThreads, 8) k_count(JS js, int phase) {
    extern __shared__ uint32_t hist[];
    __shared__ uint32_t local_n, bx0, by0, bx1, by1;
    __shared__ unsigned long long local_pairs;
    __shared__ uint32_t cls_end[kDepthBuckets];
    __shared__ uint32_t wg_zlo;
    uint32_t blk;
    const int ji = js.find(blockIdx.x, blk);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const Frame F = J.F;
    const auto src0 = SourceOf<kScene>::make(J);
    const uint32_t chunk = J.bb.chunk;
    global_t<uint32_t>* __restrict__ const vis_src = to_global(J.bb.vis_src);
    global_t<uint2>* __restrict__ const vis_rect = to_global(J.bb.vis_rect);
    global_t<uint32_t>* __restrict__ const vis_cnt = to_global(J.bb.vis_cnt);
    global_t<uint2>* __restrict__ const vis_box = to_global(J.bb.vis_box);
    global_t<uint32_t>* __restrict__ const hist_out = to_global(J.bb.hist);
    uint32_t* __restrict__ const tile_cnt = J.bb.tile_cnt;
    Counters* const ctr = J.bb.ctr;
    const int T = F.tiles_x * F.tiles_y;
    const int tid = threadIdx.x;
    for (int t = tid; t < T; t += kBinThreads) hist[t] = 0;
    if constexpr (kScene) {
        // end of each depth class in the front-to-back order of the visible clusters
        if (tid < 64) {
            uint32_t v = tid < kDepthBuckets ? ctr->vis_bucket[tid] : 0u;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t u = __shfl_up(v, o);
                if (tid >= o) v += u;
            }
            if (tid < kDepthBuckets) cls_end[tid] = v;
        }
    }
    if (tid == 0) {
        local_n = 0;
        wg_zlo = 0x7F800000u;
        local_pairs = 0;
        bx0 = 0xFFFF;
        by0 = 0xFFFF;
        bx1 = 0;
        by1 = 0;
    }
    __syncthreads();
    // resident scenes: the least cull depth of this lane's visible primitives
    // (float bits), a bound the resolve may stop a tile's list at.  The
    // resolve culls a record by (z - r)(1 - 1e-5) from FP32 coordinates
    // (bonds: the nearer end's z less the radius, and 1e-6 less); the FP64
    // value here, 2e-5 of the magnitudes and 2e-6 lower and rounded down,
    // stays below it.
    uint32_t my_zlo = 0x7F800000u;
    auto note_z = [&](double zmin, double mag) {
        const float lb = __double2float_rd(zmin - 2e-5 * mag - 2e-6);
        my_zlo = min(my_zlo, lb > 0.0f ? __float_as_uint(lb) : 0u);
    };

    const uint64_t start = (uint64_t)blk * chunk;
    auto src = src0;
    if constexpr (!kScene) src.begin(blk);
    const int tsh = F.tile_shift;
    uint32_t bad_count = 0;
    global_t<uint32_t>* __restrict__ const my_src = vis_src + start;   // this workgroup's visible list
    global_t<uint2>* __restrict__ const my_rect = vis_rect + start;
    // One visible-or-not primitive per lane (every lane of the wave calls
    // it): its slot in the workgroup's visible list, its tile counts.
    auto emit = [&](bool vis, uint32_t sidx, int x0, int y0, int x1, int y1) {
        const unsigned long long vmask = __ballot(vis);
        uint32_t slot_base = 0;
        const int leader = __ffsll((long long)(vmask | 1ull)) - 1;
        if (vmask && (int)__lane_id() == leader) slot_base = atomicAdd(&local_n, (uint32_t)__popcll(vmask));
        slot_base = __shfl(slot_base, leader);
        const int tx0 = x0 >> tsh, tx1 = x1 >> tsh, ty0 = y0 >> tsh, ty1 = y1 >> tsh;
        const bool single = vis && tx0 == tx1 && ty0 == ty1;
        wave_count(hist, single ? ty0 * F.tiles_x + tx0 : -1);
        if (vis) {
            const uint32_t slot = slot_base + (uint32_t)__popcll(vmask & __lanemask_lt());
            my_src[slot] = sidx;
            my_rect[slot] = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
            if (!single)
                for (int ty = ty0; ty <= ty1; ++ty)
                    for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&hist[ty * F.tiles_x + tx], 1u);
        }
    };
    // any primitive (the generic path)
    auto emit_item = [&](const Item& it) {
        int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
        PrimRec rec;
        double v[6], r = 0.0;
        const bool vis = item_view(F, it, rec, v, r) && item_rect(F, it, v, r, x0, y0, x1, y1);
        bad_count += it.kind == kBadBond ? 1u : 0u;
        if (kScene && vis) {
            if (it.kind == kAtom) note_z(v[2] - r, fabs(v[2]) + r);
            else note_z(fmin(v[2], v[5]) - r, fabs(v[2]) + fabs(v[5]) + r);
        }
        emit(vis, it.src, x0, y0, x1, y1);
    };
    if constexpr (kScene) {
        // Resident scene: each wave takes whole clusters (256 primitives of
        // one kind, so the kind is the same across the wave).  An atom
        // cluster's 64-atom quarters take the sphere-only path.
        // Workgroup b takes positions [c0, c1) of the visible clusters in
        // depth-class order, so the workgroups run front to back.  A
        // two-pass frame splits the positions at the first 1 / kFrontShare.
        const SceneDev& S = src.S;
        const uint32_t stride = S.atom_clusters + S.bond_clusters;
        const uint32_t nvc = cls_end[kDepthBuckets - 1];
        // the front pass ends at a depth-class boundary (the order inside a
        // class is arbitrary), unless that would take more than half
        uint32_t front = (nvc + kFrontShare - 1) / kFrontShare;
        for (int k = 0; k < kDepthBuckets; ++k) {
            if (cls_end[k] < front) continue;
            if (cls_end[k] <= nvc / 2) front = cls_end[k];
            break;
        }
        const uint32_t lo = phase == kPhaseRest ? front : 0u, hi = phase == kPhaseFront ? front : nvc;
        const uint32_t cpw = (hi - lo + src.groups - 1) / src.groups;
        const uint32_t c0 = min(hi, lo + blk * cpw), c1 = min(hi, c0 + cpw);
        int cls = 0;   // class of the positions this wave reads next (they increase)
        auto cluster_at = [&](uint32_t q) -> uint32_t {
            while (cls_end[cls] <= q) ++cls;
            return S.vis_clusters[(size_t)cls * stride + (q - (cls ? cls_end[cls - 1] : 0u))];
        };
        const uint32_t nw = kBinThreads / 64;
        const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6);
        const uint32_t lane = __lane_id();
        uint32_t cn = c0 + wave < c1 ? cluster_at(c0 + wave) : 0u;
        for (uint32_t ci = c0 + wave; ci < c1; ci += nw) {
            const uint32_t ce = (uint32_t)__builtin_amdgcn_readfirstlane((int)cn);
            const uint32_t c = ce & ~kClusterInside;
            const bool inside = (ce & kClusterInside) != 0u;   // its atoms need no frustum test
            if (ci + nw < c1) cn = cluster_at(ci + nw);   // the next cluster's id, ahead of its use
            if constexpr (kRest) {
                if (cluster_hidden(F, S, J.bb, c)) continue;
            }
            if (kAtoms || c < S.atom_clusters) {
                // one quarter at a time: holding more quarters' atoms spills
                // registers, which costs more than the load latency it hides
                for (int q = 0; q < 4; ++q) {
                    const uint32_t i = c * kCluster + (uint32_t)q * 64u + lane;
                    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (i < S.n_atoms) a = to_global(S.xyzr)[i];
                    int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
                    double vx, vy, vz;
                    to_view(F, a.x, a.y, a.z, vx, vy, vz);
                    const double r = (double)atom_radius(F, a.w);
                    const bool vis = i < S.n_atoms && r > 0.0 && (inside || sphere_in_frustum(F, vx, vy, vz, r)) &&
                                     sphere_rect_fast(F, vx, vy, vz, r, x0, y0, x1, y1);
                    if (vis) {
                        // in FP32: the resolve takes (z - r)(1 - 1e-5) from
                        // these same rounded z and r; 3e-5 of the magnitudes
                        // covers that and the few roundings here
                        const float zf = (float)vz, rf = (float)r;
                        const float lb = (zf - rf) - 3e-5f * (fabsf(zf) + rf) - 2e-6f;
                        my_zlo = min(my_zlo, lb > 0.0f ? __float_as_uint(lb) : 0u);
                    }
                    emit(vis, i, x0, y0, x1, y1);
                }
            } else if constexpr (!kAtoms) {
                for (int q = 0; q < 4; ++q) {
                    const uint32_t j = (c - S.atom_clusters) * kCluster + (uint32_t)q * 64u + lane;
                    emit_item(j < S.n_bonds ? fetch_scene(S, S.n_atoms + j) : empty_item());
                }
            }
        }
    } else {
        const uint64_t nitems = src.items();
        Item cur = empty_item();
        if ((uint64_t)tid < nitems) cur = src.fetch(tid);
        for (uint64_t base = 0; base < nitems; base += kBinThreads) {
            // the next iteration's inputs are loaded while this one is processed
            Item nxt = empty_item();
            if (base + kBinThreads + tid < nitems) nxt = src.fetch(base + kBinThreads + tid);
            emit_item(cur);
            cur = nxt;
        }
    }
    if (bad_count) atomicAdd(&ctr->bad_bonds, bad_count);
    if (kScene && my_zlo != 0x7F800000u) atomicMin(&wg_zlo, my_zlo);
    __syncthreads();   // the histogram is complete
    {
        // the workgroup's box of touched tiles and its pair count, read from
        // the histogram once rather than tracked per primitive
        uint32_t mx0 = 0xFFFF, my0 = 0xFFFF, mx1 = 0, my1 = 0;
        unsigned long long my_pairs = 0;
        for (int t = tid; t < T; t += kBinThreads) {
            const uint32_t h = hist[t];
            if (h) {
                const uint32_t ty = (uint32_t)(t / F.tiles_x), tx = (uint32_t)t - ty * (uint32_t)F.tiles_x;
                mx0 = min(mx0, tx);
                my0 = min(my0, ty);
                mx1 = max(mx1, tx);
                my1 = max(my1, ty);
                my_pairs += h;
            }
        }
        if (my_pairs) {
            atomicMin(&bx0, mx0);
            atomicMin(&by0, my0);
            atomicMax(&bx1, mx1);
            atomicMax(&by1, my1);
            atomicAdd(&local_pairs, my_pairs);
        }
    }
    __syncthreads();
    global_t<uint32_t>* const row = hist_out + (size_t)blk * T;
    // layered lists: per-layer totals (the layer kernel turns them into list
    // starts and tile totals); otherwise the tile totals directly
    uint32_t* const tot = kScene && J.bb.layers > 1
                              ? J.bb.layer_sum + (size_t)layer_of(blk, J.bb.groups, J.bb.layers) * T
                              : tile_cnt;
    // the histogram row holds the tiles of the workgroup's box only (see
    // box_tile), row-major within the box
    const int bw = bx0 <= bx1 ? (int)(bx1 - bx0) + 1 : 0, nb = bw * (bw ? (int)(by1 - by0) + 1 : 0);
    for (int i = tid; i < nb; i += kBinThreads) {
        const int t = box_tile(F, bx0, by0, bw, i);
        const uint32_t h = hist[t];
        row[i] = h;
        if (h) atomicAdd(&tot[t], h);
    }
    if (tid == 0) {
        if (kScene && J.bb.layers > 1 && wg_zlo != 0x7F800000u)
            atomicMin(&ctr->layer_zlo[phase == kPhaseRest ? 1 : 0][layer_of(blk, J.bb.groups, J.bb.layers)], wg_zlo);
        vis_cnt[blk] = local_n;
        vis_box[blk] = make_uint2(bx0 | (by0 << 16), bx1 | (by1 << 16));
        atomicAdd(&ctr->vis_count, local_n);
        if (local_pairs) atomicAdd(&ctr->pairs_counted, local_pairs);
    }
}

// Layer starts of the tile lists (jobs with layers > 1).  For tile t,
// layer_off[g][t] is the number of t's entries in the layers before g (the
// exclusive prefix over g of the count kernel's per-layer totals), and
// tile_cnt[t] the list's length; the totals are re-zeroed for the next frame.
// With P the power of two >= layers, work block b takes the (1024 / P)-tile
// blocks b, b + groups, ...; thread (g, i) = (tid / W, tid % W) holds layer
// g's total of tile i (loads coalesced along i), and the prefix over g goes
// through LDS.
template <class JS>
__global__ void __launch_bounds__(kBinThreads) k_layers(JS js) {
    static_assert(kBinThreads == 1024 && kLayers <= 32, "tile blocks of 1024 / P tiles, P <= 32");
    __shared__ uint32_t part[kBinThreads + kLayers];
    uint32_t blk;
    const int ji = js.find(blockIdx.x, blk);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const uint32_t L = J.bb.layers, groups = J.bb.groups;
    if (L <= 1) return;
    const uint32_t T = (uint32_t)(J.F.tiles_x * J.F.tiles_y);
    uint32_t* __restrict__ const sum = J.bb.layer_sum;
    uint32_t* __restrict__ const loff = J.bb.layer_off;
    const uint32_t lsh = 32u - (uint32_t)__builtin_clz(L - 1u);   // P = 1 << lsh >= L (L <= kLayers)
    const uint32_t wsh = 10u - lsh, W = 1u << wsh;                  // tiles per block: kBinThreads / P
    const uint32_t g = threadIdx.x >> wsh, i = threadIdx.x & (W - 1u);
    for (uint32_t tb = blk; tb * W < T; tb += groups) {   // trip count uniform over the workgroup
        const uint32_t t = tb * W + i;
        const bool mine = t < T && g < L;
        uint32_t v = 0;
        if (mine) {
            v = sum[(size_t)g * T + t];
            sum[(size_t)g * T + t] = 0u;
        }
        part[g * (W + 1u) + i] = v;
        __syncthreads();
        uint32_t pre = 0;
        for (uint32_t h = 0; h < g; ++h) pre += part[h * (W + 1u) + i];
        if (mine) {
            loff[(size_t)g * T + t] = pre;
            if (g == L - 1u) J.bb.tile_cnt[t] = pre + v;
        }
        __syncthreads();   // part is rewritten by the next tile block
    }
}

// Scatter cursor of a tile this workgroup has no run in (its list did not
// fit, or it has no primitive there).  Slots are below kMaxCapacity <=
// 2^28, and adding at most a workgroup's pairs keeps the flag bit set.
constexpr uint32_t kNoRun = 0x80000000u;

// List offsets: the exclusive prefix sum of the tile counts, once per job
// (work block j of the launch scans job j's counts), with the list total and
// the overflow flag in the frame counters.  The counts are read as up to
// kMaxLdsTiles / 1024 rows of 1024 consecutive tiles, every load issued
// before the first is used (coalesced, all in flight); each wave scans its
// 64 lanes of every row with DPP steps, and one wave scans the (row, wave)
// totals, which gives every (row, wave) its start.
template <class JS>
__global__ void __launch_bounds__(kBinThreads) k_tile_offsets(JS js) {
    constexpr int kRows = (kMaxLdsTiles + kBinThreads - 1) / kBinThreads;
    constexpr int kWaves = kBinThreads / 64;
    constexpr int kPre = (kRows * kWaves + 63) / 64;
    __shared__ uint32_t wsum[kRows][kWaves];
    __shared__ unsigned long long wpre[kRows * kWaves + 1];
    __shared__ uint32_t over_sum;
    if (blockIdx.x >= js.count()) return;
    const Job& J = js.job((int)blockIdx.x);
    const int T = J.F.tiles_x * J.F.tiles_y;
    const uint32_t* __restrict__ const cnt = J.bb.tile_cnt;
    uint64_t* __restrict__ const off = J.bb.tile_off;
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const int rows = (T + kBinThreads - 1) / kBinThreads;
    uint32_t v[kRows], incl[kRows];
    uint32_t n_over = 0;
    if (tid == 0) over_sum = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int t = r * kBinThreads + tid;
        v[r] = r < rows && t < T ? cnt[t] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        incl[r] = wave_scan_u32(v[r]);
        if (lane == 63) wsum[r][wave] = incl[r];
    }
    __syncthreads();
    // wave 0: the exclusive prefix of the (row, wave) totals in row-major
    // order, kPre per lane, and the list total after them
    if (wave == 0) {
        unsigned long long part[kPre], s = 0;
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int i = lane * kPre + k;
            part[k] = s;
            s += i < rows * kWaves ? wsum[i / kWaves][i % kWaves] : 0u;
        }
        unsigned long long pre = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long u = __shfl_up(pre, o);
            if (lane >= o) pre += u;
        }
        pre -= s;
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int i = lane * kPre + k;
            if (i < kRows * kWaves) wpre[i] = pre + part[k];
        }
        if (lane == 63) wpre[kRows * kWaves] = pre + s;
    }
    __syncthreads();
    // start of this thread's tile in each row: the (row, wave) start, then
    // the lanes before it
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        if (r >= rows) break;
        const int t = r * kBinThreads + tid;
        if (t < T) {
            const uint64_t o = wpre[r * kWaves + wave] + (incl[r] - v[r]);
            off[t] = o;
            n_over += o + v[r] > J.bb.capacity ? 1u : 0u;   // lists the scatter leaves to the resolve's tail
        }
    }
    const unsigned long long base = wpre[kRows * kWaves];
    for (int o = 32; o > 0; o >>= 1) n_over += (uint32_t)__shfl_xor((int)n_over, o);
    if (lane == 0 && n_over) atomicAdd(&over_sum, n_over);
    __syncthreads();
    if (tid == 0) {
        J.bb.ctr->pairs = base;
        J.bb.ctr->overflow = base > J.bb.capacity ? 1u : 0u;
        J.bb.ctr->overflow_tiles = over_sum;
    }
}

// Scatter.  Every workgroup reserves, for each tile its primitives touch,
// one run of that tile's list (one global atomic), then places its visible
// primitives kScatterPer per thread at a time, all their loads issued
// before any is used.  Lanes of a wave whose primitive lies in one tile take
// their slots by runs of consecutive lanes with the same tile (one LDS
// atomic per run, in one instruction for the wave).  Primitives spanning
// several tiles take one LDS atomic per tile.  Workgroup 0 also publishes
// the frame counters.
constexpr int kScatterPer = 4;

template <class JS>
__global__ void __launch_bounds__(kBinThreads, 8) k_scatter(JS js, int phase) {
    constexpr int kTileRows = (kMaxLdsTiles + kBinThreads - 1) / kBinThreads;
    extern __shared__ uint32_t cur[];
    uint32_t blk;
    const int ji = js.find(blockIdx.x, blk);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const Frame F = J.F;
    const uint32_t chunk = J.bb.chunk;
    const global_t<const uint32_t>* __restrict__ const vis_src = to_global(J.bb.vis_src);
    const global_t<const uint2>* __restrict__ const vis_rect = to_global(J.bb.vis_rect);
    const global_t<const uint32_t>* __restrict__ const vis_cnt = to_global(J.bb.vis_cnt);
    const global_t<const uint32_t>* __restrict__ const hist_in = to_global(J.bb.hist);
    const global_t<const uint32_t>* __restrict__ const cnt = to_global(J.bb.tile_cnt);
    const global_t<const uint64_t>* __restrict__ const off = to_global(J.bb.tile_off);
    global_t<uint2>* __restrict__ const list = to_global(J.bb.list);
    const uint64_t capacity = J.bb.capacity;
    Counters* const ctr = J.bb.ctr;
    Counters* const host_ctr = J.bb.host_ctr;
    const int T = F.tiles_x * F.tiles_y;
    // this workgroup's layer: its runs go after those of the layers before it
    const uint32_t lay = J.bb.layers > 1 ? layer_of(blk, J.bb.groups, J.bb.layers) : 0u;
    uint32_t* const fill = J.bb.tile_fill + (size_t)lay * T;
    const global_t<const uint32_t>* __restrict__ const loff =
        J.bb.layers > 1 ? to_global(J.bb.layer_off + (size_t)lay * T) : nullptr;
    const int tid = threadIdx.x;
    const bool lead = blk == 0;
    const global_t<const uint32_t>* const row = hist_in + (size_t)blk * T;
    {
        // the workgroup's tile box (its primitives touch no tile outside it,
        // whose cursors are never read); the box's counts first, then the
        // reservations of the touched tiles, so the loads and atomics overlap
        const uint2 box = to_global(J.bb.vis_box)[blk];
        const uint32_t bx0 = box.x & 0xFFFFu, by0 = box.x >> 16, bx1 = box.y & 0xFFFFu, by1 = box.y >> 16;
        const int bw = bx0 <= bx1 ? (int)(bx1 - bx0) + 1 : 0, nb = bw * (bw ? (int)(by1 - by0) + 1 : 0);
        uint32_t h[kTileRows], r[kTileRows];
#pragma unroll
        for (int q = 0; q < kTileRows; ++q) {
            const int i = q * kBinThreads + tid;
            h[q] = i < nb ? row[i] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kTileRows; ++q) {
            const int i = q * kBinThreads + tid;
            r[q] = h[q] ? atomicAdd(&fill[box_tile(F, bx0, by0, bw, i)], h[q]) : 0u;
        }
#pragma unroll
        for (int q = 0; q < kTileRows; ++q) {
            const int i = q * kBinThreads + tid;
            if (i >= nb) break;
            const int t = box_tile(F, bx0, by0, bw, i);
            const uint64_t run = off[t];
            const bool fits = run + cnt[t] <= capacity;   // else the resolve rebuilds this tile from the visible lists
            cur[t] = h[q] && fits ? (uint32_t)(run + (loff ? loff[t] : 0u) + r[q]) : kNoRun;
        }
    }
    if (lead) {
        if (tid == 0) {
            const unsigned int vis = ctr->vis_count, bad = ctr->bad_bonds;
            const unsigned long long total = ctr->pairs;
            const unsigned int n_over = ctr->overflow_tiles;   // from k_tile_offsets
            ctr->vis_count = 0;            // the next frame's count kernel adds to these
            ctr->bad_bonds = 0;
            ctr->frag_tested = 0;          // this frame's resolve adds to these
            ctr->frag_hit = 0;
            ctr->frag_hit_bond = 0;
            ctr->frag_tested_bond = 0;
            ctr->frag_skipped = 0;
            ctr->rec_culled = 0;
            ctr->lists_stopped = 0;
            ctr->chunks_stopped = 0;
            ctr->done_blocks = 0;
            ctr->pairs_counted = 0;
            // the next frame's cluster test adds to these (the rest pass reads them)
            if (phase != kPhaseFront)
                for (int k = 0; k < kDepthBuckets; ++k) ctr->vis_bucket[k] = 0;
            if (host_ctr && phase == kPhaseRest) {
                // a two-pass frame: visible primitives and overflowed tiles of
                // both passes, the larger list total
                host_ctr->vis_count += vis;
                host_ctr->bad_bonds += bad;
                if (total > host_ctr->pairs) host_ctr->pairs = total;
                host_ctr->overflow |= total > capacity ? 1u : 0u;
                host_ctr->overflow_tiles += n_over;
                __threadfence_system();
            } else if (host_ctr) {
                host_ctr->vis_count = vis;
                host_ctr->bad_bonds = bad;
                host_ctr->pairs = total;
                host_ctr->overflow = total > capacity ? 1u : 0u;
                host_ctr->overflow_tiles = n_over;
                host_ctr->frag_tested = 0;
                host_ctr->frag_hit = 0;
                host_ctr->frag_hit_bond = 0;
                host_ctr->frag_tested_bond = 0;
                host_ctr->frag_skipped = 0;
                host_ctr->rec_culled = 0;
                host_ctr->lists_stopped = 0;
                host_ctr->chunks_stopped = 0;
                __threadfence_system();
            }
        }
    }
    __syncthreads();
    const uint32_t n = vis_cnt[blk];
    if (n == 0) return;
    const global_t<const uint32_t>* __restrict__ const my_src = vis_src + (size_t)blk * chunk;
    const global_t<const uint2>* __restrict__ const my_rect = vis_rect + (size_t)blk * chunk;
    const int ts = F.tile, tsh = F.tile_shift;
    // the footprint clipped to tile (tx, ty), in tile-local pixels
    auto local_fp = [&](int x0, int y0, int x1, int y1, int tx, int ty) -> uint32_t {
        const int lx0 = max(x0 - tx * ts, 0), ly0 = max(y0 - ty * ts, 0);
        const int lx1 = min(x1 - tx * ts, ts - 1), ly1 = min(y1 - ty * ts, ts - 1);
        return (uint32_t)lx0 | ((uint32_t)ly0 << 8) | ((uint32_t)(lx1 - lx0 + 1) << 16) |
               ((uint32_t)(ly1 - ly0 + 1) << 24);
    };
    const int lane = __lane_id();
    constexpr uint32_t kSpan = (uint32_t)kBinThreads * kScatterPer;
    for (uint32_t base = 0; base < n; base += kSpan) {   // uniform trip count (wave ops inside)
        uint32_t src[kScatterPer];
        uint2 rc[kScatterPer];
#pragma unroll
        for (int p = 0; p < kScatterPer; ++p) {
            // past the end: a copy of the last entry, dropped below (loads stay in bounds)
            const uint32_t k = min(base + (uint32_t)(p * kBinThreads + tid), n - 1u);
            src[p] = my_src[k];
            rc[p] = my_rect[k];
        }
        // the single-tile primitives of all kScatterPer batches take their
        // slots first (their atomics and slot exchanges overlap), then write
        // their entries; the primitives spanning several tiles follow
        uint32_t slot[kScatterPer];
        bool single[kScatterPer];
#pragma unroll
        for (int p = 0; p < kScatterPer; ++p) {
            const bool have = base + (uint32_t)(p * kBinThreads + tid) < n;
            const int x0 = rc[p].x & 0xFFFF, y0 = rc[p].x >> 16, x1 = rc[p].y & 0xFFFF, y1 = rc[p].y >> 16;
            single[p] = have && (x0 >> tsh) == (x1 >> tsh) && (y0 >> tsh) == (y1 >> tsh);
            const int t1 = single[p] ? (y0 >> tsh) * F.tiles_x + (x0 >> tsh) : -1;
            // one LDS atomic per run of lanes with the same tile; the run's
            // lanes take consecutive slots after its head's
            int head;
            uint32_t len;
            lane_run(t1, head, len);
            const uint32_t first = single[p] && head == lane ? atomicAdd(&cur[t1], len) : 0u;
            slot[p] = (uint32_t)__shfl((int)first, head) + (uint32_t)(lane - head);
        }
#pragma unroll
        for (int p = 0; p < kScatterPer; ++p) {
            if (single[p] && !(slot[p] & kNoRun)) {
                // inside its one tile: the rectangle in tile-local pixels, unclipped
                const uint32_t x0 = rc[p].x & 0xFFFFu, y0 = rc[p].x >> 16, x1 = rc[p].y & 0xFFFFu, y1 = rc[p].y >> 16;
                const uint32_t m = (uint32_t)ts - 1u;
                list[slot[p]] = make_uint2(src[p], (x0 & m) | ((y0 & m) << 8) | ((x1 - x0 + 1u) << 16) |
                                                       ((y1 - y0 + 1u) << 24));
            }
        }
#pragma unroll
        for (int p = 0; p < kScatterPer; ++p) {
            const bool have = base + (uint32_t)(p * kBinThreads + tid) < n;
            if (have && !single[p]) {
                const int x0 = rc[p].x & 0xFFFF, y0 = rc[p].x >> 16, x1 = rc[p].y & 0xFFFF, y1 = rc[p].y >> 16;
                for (int ty = y0 >> tsh; ty <= (y1 >> tsh); ++ty)
                    for (int tx = x0 >> tsh; tx <= (x1 >> tsh); ++tx) {
                        const uint32_t sl = atomicAdd(&cur[ty * F.tiles_x + tx], 1u);
                        if (!(sl & kNoRun)) list[sl] = make_uint2(src[p], local_fp(x0, y0, x1, y1, tx, ty));
                    }
            }
        }
    }
}

}  // namespace

void bin_grid(uint64_t nprim, uint32_t* groups, uint32_t* chunk) {
    uint64_t g = (nprim + 4095) / 4096;
    if (g < 1) g = 1;
    if (g > kMaxBinGroups) g = kMaxBinGroups;
    uint64_t c = (nprim + g - 1) / g;
    if (c < 1) c = 1;
    *groups = (uint32_t)g;
    *chunk = (uint32_t)c;
}

hipError_t launch_zero(uint32_t* p, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    k_zero<<<(unsigned)blocks, kBlock, 0, stream>>>(p, n);
    return hipGetLastError();
}

// A render, or a batch, of scenes without bonds takes the atom-only count.
inline bool atoms_only(const OneJob& js) { return js.j.S.bond_clusters == 0; }
inline bool atoms_only(const JobList& js) { return js.no_bonds != 0; }

template <class JS>
hipError_t count_impl(const JS& js, bool scene, int phase, uint32_t grid, int max_tiles, hipStream_t stream) {
    if (max_tiles > kMaxLdsTiles) return hipErrorInvalidValue;
    if (phase != kPhaseAll && !scene) return hipErrorInvalidValue;
    if (grid == 0) return hipSuccess;
    const size_t lds = (size_t)max_tiles * sizeof(uint32_t);
    if (scene && phase == kPhaseRest) return dispatch(k_count<JS, true, true>, grid, kBinThreads, lds, stream, js, phase);
    if (scene && atoms_only(js)) return dispatch(k_count<JS, true, false, true>, grid, kBinThreads, lds, stream, js, phase);
    if (scene) return dispatch(k_count<JS, true, false>, grid, kBinThreads, lds, stream, js, phase);
    return dispatch(k_count<JS, false, false>, grid, kBinThreads, lds, stream, js, phase);
}

template <class JS>
hipError_t scatter_impl(const JS& js, int phase, uint32_t grid, int max_tiles, hipStream_t stream) {
    if (max_tiles > kMaxLdsTiles) return hipErrorInvalidValue;
    if (grid == 0) return hipSuccess;
    return dispatch(k_scatter<JS>, grid, kBinThreads, (uint32_t)(max_tiles * sizeof(uint32_t)), stream, js, phase);
}

hipError_t launch_count(const OneJob& js, bool scene, int phase, uint32_t grid, int max_tiles, hipStream_t stream) {
    return count_impl(js, scene, phase, grid, max_tiles, stream);
}
hipError_t launch_count(const JobList& js, bool scene, int phase, uint32_t grid, int max_tiles, hipStream_t stream) {
    return count_impl(js, scene, phase, grid, max_tiles, stream);
}
hipError_t launch_layers(const OneJob& js, uint32_t grid, hipStream_t stream) {
    return dispatch(k_layers<OneJob>, grid, kBinThreads, 0, stream, js);
}
hipError_t launch_layers(const JobList& js, uint32_t grid, hipStream_t stream) {
    return dispatch(k_layers<JobList>, grid, kBinThreads, 0, stream, js);
}
hipError_t launch_tile_offsets(const OneJob& js, hipStream_t stream) {
    return dispatch(k_tile_offsets<OneJob>, 1, kBinThreads, 0, stream, js);
}
hipError_t launch_tile_offsets(const JobList& js, hipStream_t stream) {
    return dispatch(k_tile_offsets<JobList>, js.n, kBinThreads, 0, stream, js);
}
hipError_t launch_scatter(const OneJob& js, int phase, uint32_t grid, int max_tiles, hipStream_t stream) {
    return scatter_impl(js, phase, grid, max_tiles, stream);
}
hipError_t launch_scatter(const JobList& js, int phase, uint32_t grid, int max_tiles, hipStream_t stream) {
    return scatter_impl(js, phase, grid, max_tiles, stream);
}

}  // namespace vtx
