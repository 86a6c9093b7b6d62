// Screen-tile binning of atoms and bonds: a counting sort by tile.
//
// The paper rasterizes one screen quad per primitive and lets the fixed
// function rasterizer find the pixels it covers (Methods, "Meshless
// Representations").  Here the quad's role, a conservative footprint, becomes
// an exact tile rectangle per primitive, and the rasterizer becomes a
// counting sort of (tile, primitive) pairs:
//   count    G workgroups each own a contiguous run of primitives: view
//            transform (FP64), culling, footprint rectangle, a compacted
//            per-workgroup list of the visible ones, and a tile histogram
//            in LDS; the histogram row is stored and its non-zero entries are
//            added to the global tile counts (one atomic per touched tile);
//   scatter  each workgroup rebuilds the exclusive prefix sum of the tile
//            counts (list offsets), reserves, per touched tile, one run of the
//            tile's list (one atomic), then places its primitives with LDS
//            atomics.
// So the global atomics scale with (workgroup, touched tile) pairs rather
// than with (primitive, tile) pairs.  Lists that would not fit the bin
// capacity are left empty; the resolve pass then finds those tiles' primitives
// in the per-workgroup visible lists, so every frame is exact whatever the
// capacity.
#include "vtx_internal.h"

namespace vtx {

namespace {

// Zeroes n words (allocation time only: afterwards every frame leaves the
// tile counts and the frame counters at zero for the next one).
__global__ void __launch_bounds__(kBlock) k_zero(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// View-space record and footprint of a sphere (id = primitive id); false if
// it cannot show.  The FP32 frustum test rejects most off-screen spheres
// before the exact FP64 footprint.
__device__ inline bool sphere_record(const Frame& F, double vx, double vy, double vz, double r, uint32_t id, int& x0,
                                     int& y0, int& x1, int& y1, PrimRec& rec) {
    if (!(r > 0.0) || !sphere_in_frustum(F, vx, vy, vz, r)) return false;
    rec.g0 = make_float4((float)vx, (float)vy, (float)vz, (float)r);
    rec.g1 = make_uint4(0u, 0u, id, 0u);
    return sphere_rect(F, vx, vy, vz, r, x0, y0, x1, y1);
}

// Same for a bond between view points A and B (the difference B - A is kept
// from FP64, so the axis is accurate however far the bond is).
__device__ inline bool bond_record(const Frame& F, const double* A, const double* B, uint32_t id, int& x0, int& y0,
                                   int& x1, int& y1, PrimRec& rec) {
    const double rho = F.bond_radius;
    const double dx = B[0] - A[0], dy = B[1] - A[1], dz = B[2] - A[2];
    const double half = 0.5 * sqrt(dx * dx + dy * dy + dz * dz);
    if (!sphere_in_frustum(F, A[0] + 0.5 * dx, A[1] + 0.5 * dy, A[2] + 0.5 * dz, half + rho)) return false;
    rec.g0 = make_float4((float)A[0], (float)A[1], (float)A[2], (float)dx);
    rec.g1 = make_uint4(__float_as_uint((float)dy), __float_as_uint((float)dz), id, 0u);
    return bond_rect(F, A, B, rho, x0, y0, x1, y1);
}

// Footprint and view-space record of primitive p; false if it cannot show.
__device__ inline bool primitive_record(const Frame& F, uint32_t p, const float* __restrict__ pos,
                                        const float* __restrict__ rad, const uint32_t* __restrict__ bonds,
                                        int& x0, int& y0, int& x1, int& y1, PrimRec& rec, bool& bad) {
    bad = false;
    if (p < F.n_atoms) {
        double vx, vy, vz;
        to_view(F, pos[3 * (size_t)p], pos[3 * (size_t)p + 1], pos[3 * (size_t)p + 2], vx, vy, vz);
        return sphere_record(F, vx, vy, vz, (double)rad[p], p, x0, y0, x1, y1, rec);
    }
    const size_t b = p - F.n_atoms;
    const uint32_t ia = bonds[2 * b], ib = bonds[2 * b + 1];
    if (ia >= F.n_atoms || ib >= F.n_atoms) {
        bad = true;
        return false;
    }
    if (ia == ib) return false;
    const float ax = pos[3 * (size_t)ia], ay = pos[3 * (size_t)ia + 1], az = pos[3 * (size_t)ia + 2];
    const float bx = pos[3 * (size_t)ib], by = pos[3 * (size_t)ib + 1], bz = pos[3 * (size_t)ib + 2];
    if (ax == bx && ay == by && az == bz) return false;
    double A[3], B[3];
    to_view(F, ax, ay, az, A[0], A[1], A[2]);
    to_view(F, bx, by, bz, B[0], B[1], B[2]);
    return bond_record(F, A, B, p, x0, y0, x1, y1, rec);
}

// Primitive sources of the count kernel.  Workgroup b owns items
// [0, items(b)) and the visible-list region [b * chunk, (b + 1) * chunk).
struct PlainSource {     // the caller's arrays, primitives in their given order
    const float* pos;
    const float* rad;
    const uint32_t* bonds;
    uint64_t total;
    uint32_t chunk;
    __device__ uint64_t items(uint32_t b) const {
        const uint64_t s = (uint64_t)b * chunk;
        return s < total ? min((uint64_t)chunk, total - s) : 0;
    }
    __device__ bool record(const Frame& F, uint32_t b, uint64_t k, int& x0, int& y0, int& x1, int& y1, PrimRec& rec,
                           bool& bad) const {
        return primitive_record(F, (uint32_t)((uint64_t)b * chunk + k), pos, rad, bonds, x0, y0, x1, y1, rec, bad);
    }
};

struct SceneSource {     // a resident scene: the clusters that passed the frustum test
    SceneDev S;
    const Counters* ctr;
    uint32_t groups;
    __device__ void range(uint32_t b, uint32_t& c0, uint32_t& c1) const {
        const uint32_t nvc = ctr->vis_clusters;
        const uint32_t cpw = (nvc + groups - 1) / groups;
        c0 = min(nvc, b * cpw);
        c1 = min(nvc, c0 + cpw);
    }
    __device__ uint64_t items(uint32_t b) const {
        uint32_t c0, c1;
        range(b, c0, c1);
        return (uint64_t)(c1 - c0) * kCluster;
    }
    __device__ bool record(const Frame& F, uint32_t b, uint64_t k, int& x0, int& y0, int& x1, int& y1, PrimRec& rec,
                           bool& bad) const {
        bad = false;
        uint32_t c0, c1;
        range(b, c0, c1);
        const uint32_t c = S.vis_clusters[c0 + (uint32_t)(k / kCluster)];
        const uint32_t slot = (uint32_t)(k % kCluster);
        if (c < S.atom_clusters) {
            const uint32_t i = c * kCluster + slot;
            if (i >= S.n_atoms) return false;
            const float4 a = S.xyzr[i];
            double vx, vy, vz;
            to_view(F, a.x, a.y, a.z, vx, vy, vz);
            return sphere_record(F, vx, vy, vz, (double)a.w, S.atom_id[i], x0, y0, x1, y1, rec);
        }
        const uint32_t j = (c - S.atom_clusters) * kCluster + slot;
        if (j >= S.n_bonds) return false;
        const uint4 br = S.bond_rec[j];
        if (br.x == br.y) return false;
        const float4 a = S.xyzr[br.x], bb = S.xyzr[br.y];
        if (a.x == bb.x && a.y == bb.y && a.z == bb.z) return false;
        double A[3], B[3];
        to_view(F, a.x, a.y, a.z, A[0], A[1], A[2]);
        to_view(F, bb.x, bb.y, bb.z, B[0], B[1], B[2]);
        return bond_record(F, A, B, F.n_atoms + br.z, x0, y0, x1, y1, rec);
    }
};

template <bool kScene>
struct SourceOf;
template <>
struct SourceOf<false> {
    __device__ static PlainSource make(const Job& J) {
        return PlainSource{J.pos, J.rad, J.bonds, (uint64_t)J.F.n_atoms + J.F.n_bonds, J.bb.chunk};
    }
};
template <>
struct SourceOf<true> {
    __device__ static SceneSource make(const Job& J) { return SceneSource{J.S, J.bb.ctr, J.bb.groups}; }
};

// Count.  Work block b of a job is that job's binning workgroup b.
template <class JS, bool kScene>
__global__ void __launch_bounds__(kBinThreads) k_count(JS js) {
    extern __shared__ uint32_t hist[];
    __shared__ uint32_t local_n, bx0, by0, bx1, by1;
    __shared__ unsigned long long local_pairs;
    uint32_t blk;
    const int ji = js.find(blockIdx.x, blk);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const Frame F = J.F;
    const auto src = SourceOf<kScene>::make(J);
    const uint32_t chunk = J.bb.chunk;
    PrimRec* __restrict__ const vis_rec = J.bb.vis_rec;
    uint2* __restrict__ const vis_rect = J.bb.vis_rect;
    uint32_t* __restrict__ const vis_cnt = J.bb.vis_cnt;
    uint2* __restrict__ const vis_box = J.bb.vis_box;
    uint32_t* __restrict__ const hist_out = J.bb.hist;
    uint32_t* __restrict__ const tile_cnt = J.bb.tile_cnt;
    Counters* const ctr = J.bb.ctr;
    const int T = F.tiles_x * F.tiles_y;
    const int tid = threadIdx.x;
    for (int t = tid; t < T; t += kBinThreads) hist[t] = 0;
    if (tid == 0) {
        local_n = 0;
        local_pairs = 0;
        bx0 = 0xFFFF;
        by0 = 0xFFFF;
        bx1 = 0;
        by1 = 0;
    }
    __syncthreads();
    uint32_t mx0 = 0xFFFF, my0 = 0xFFFF, mx1 = 0, my1 = 0, my_pairs = 0;

    const uint64_t start = (uint64_t)blk * chunk;
    const uint64_t nitems = src.items(blk);
    const int ts = F.tile;
    uint32_t bad_count = 0;
    for (uint64_t base = 0; base < nitems; base += kBinThreads) {
        const uint64_t k = base + tid;
        int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
        bool bad = false;
        PrimRec rec;
        const bool vis = k < nitems && src.record(F, blk, k, x0, y0, x1, y1, rec, bad);
        bad_count += bad ? 1u : 0u;
        const unsigned long long vmask = __ballot(vis);
        uint32_t slot_base = 0;
        const int leader = __ffsll((long long)(vmask | 1ull)) - 1;
        if (vmask && (int)__lane_id() == leader) slot_base = atomicAdd(&local_n, (uint32_t)__popcll(vmask));
        slot_base = __shfl(slot_base, leader);
        if (vis) {
            const uint64_t slot = start + slot_base + (uint32_t)__popcll(vmask & __lanemask_lt());
            const int tx0 = x0 / ts, tx1 = x1 / ts, ty0 = y0 / ts, ty1 = y1 / ts;
            vis_rec[slot] = rec;
            vis_rect[slot] = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&hist[ty * F.tiles_x + tx], 1u);
            mx0 = min(mx0, (uint32_t)tx0);
            my0 = min(my0, (uint32_t)ty0);
            mx1 = max(mx1, (uint32_t)tx1);
            my1 = max(my1, (uint32_t)ty1);
            my_pairs += (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
        }
    }
    if (bad_count) atomicAdd(&ctr->bad_bonds, bad_count);
    if (my_pairs) {
        atomicMin(&bx0, mx0);
        atomicMin(&by0, my0);
        atomicMax(&bx1, mx1);
        atomicMax(&by1, my1);
        atomicAdd(&local_pairs, (unsigned long long)my_pairs);
    }
    __syncthreads();
    uint32_t* row = hist_out + (size_t)blk * T;
    for (int t = tid; t < T; t += kBinThreads) {
        const uint32_t h = hist[t];
        row[t] = h;
        if (h) atomicAdd(&tile_cnt[t], h);
    }
    if (tid == 0) {
        vis_cnt[blk] = local_n;
        vis_box[blk] = make_uint2(bx0 | (by0 << 16), bx1 | (by1 << 16));
        atomicAdd(&ctr->vis_count, local_n);
        if (local_pairs) atomicAdd(&ctr->pairs_counted, local_pairs);
    }
}

constexpr uint32_t kNoRun = 0xFFFFFFFFu;

// Scatter.  Every workgroup first rebuilds the exclusive prefix sum of the
// tile counts for itself (one read of T counts from L2; lane j owns a
// contiguous run of tiles, the run totals are scanned with wave shuffles and
// one LDS exchange), and while walking its run reserves, for each tile its
// primitives touch, one run of that tile's list (one global atomic).  It then
// places its primitives with LDS atomics.  Workgroup 0 also stores the tile
// offsets for the resolve and publishes the frame counters.
template <class JS>
__global__ void __launch_bounds__(kBinThreads) k_scatter(JS js) {
    extern __shared__ uint32_t cur[];
    __shared__ unsigned long long wtot[kBinThreads / 64];
    __shared__ unsigned int n_over;
    uint32_t blk;
    const int ji = js.find(blockIdx.x, blk);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const Frame F = J.F;
    const uint32_t chunk = J.bb.chunk;
    const PrimRec* __restrict__ const vis_rec = J.bb.vis_rec;
    const uint2* __restrict__ const vis_rect = J.bb.vis_rect;
    const uint32_t* __restrict__ const vis_cnt = J.bb.vis_cnt;
    const uint32_t* __restrict__ const hist_in = J.bb.hist;
    const uint32_t* __restrict__ const cnt = J.bb.tile_cnt;
    uint64_t* __restrict__ const off = J.bb.tile_off;
    uint32_t* const fill = J.bb.tile_fill;
    PrimRec* __restrict__ const list = J.bb.list;
    const uint64_t capacity = J.bb.capacity;
    Counters* const ctr = J.bb.ctr;
    Counters* const host_ctr = J.bb.host_ctr;
    const int T = F.tiles_x * F.tiles_y;
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const bool lead = blk == 0;
    const int per = (T + kBinThreads - 1) / kBinThreads;
    const int b = min(T, tid * per), e = min(T, b + per);
    unsigned long long sum = 0;
    for (int t = b; t < e; ++t) sum += cnt[t];
    unsigned long long incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wtot[wave] = incl;
    if (tid == 0) n_over = 0;
    __syncthreads();
    unsigned long long run = incl - sum, total = 0;
    for (int w = 0; w < kBinThreads / 64; ++w) {
        const unsigned long long v = wtot[w];
        run += w < wave ? v : 0ull;
        total += v;
    }
    const uint32_t* row = hist_in + (size_t)blk * T;
    unsigned int over = 0;
    for (int t = b; t < e; ++t) {
        const uint32_t c = cnt[t];
        const bool fits = run + c <= capacity;      // else the resolve rebuilds this tile from the visible lists
        const uint32_t h = row[t];
        uint32_t r = kNoRun;
        if (h && fits) r = (uint32_t)(run + atomicAdd(&fill[t], h));
        cur[t] = r;
        if (lead) off[t] = run;
        over += fits ? 0u : 1u;
        run += c;
    }
    if (lead) {
        if (over) atomicAdd(&n_over, over);
        __syncthreads();
        if (tid == 0) {
            const unsigned int vis = ctr->vis_count, bad = ctr->bad_bonds;
            ctr->pairs = total;
            ctr->overflow = total > capacity ? 1u : 0u;
            ctr->overflow_tiles = n_over;
            ctr->vis_count = 0;            // the next frame's count kernel adds to these
            ctr->bad_bonds = 0;
            ctr->frag_tested = 0;          // this frame's resolve adds to these
            ctr->frag_hit = 0;
            ctr->frag_hit_bond = 0;
            ctr->done_blocks = 0;
            ctr->pairs_counted = 0;
            ctr->vis_clusters = 0;         // the next frame's cluster test adds to this
            if (host_ctr) {
                host_ctr->vis_count = vis;
                host_ctr->bad_bonds = bad;
                host_ctr->pairs = total;
                host_ctr->overflow = total > capacity ? 1u : 0u;
                host_ctr->overflow_tiles = n_over;
                host_ctr->frag_tested = 0;
                host_ctr->frag_hit = 0;
                host_ctr->frag_hit_bond = 0;
                __threadfence_system();
            }
        }
    }
    __syncthreads();
    const uint32_t n = vis_cnt[blk];
    const uint64_t start = (uint64_t)blk * chunk;
    const int ts = F.tile;
    for (uint32_t k = tid; k < n; k += kBinThreads) {
        const float4 g0 = vis_rec[start + k].g0;
        const uint4 g1 = vis_rec[start + k].g1;
        const uint2 r = vis_rect[start + k];
        const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16;
        for (int ty = y0 / ts; ty <= y1 / ts; ++ty)
            for (int tx = x0 / ts; tx <= x1 / ts; ++tx) {
                const int t = ty * F.tiles_x + tx;
                if (cur[t] == kNoRun) continue;
                // the footprint clipped to this tile, in tile-local pixels
                const int lx0 = max(x0 - tx * ts, 0), ly0 = max(y0 - ty * ts, 0);
                const int lx1 = min(x1 - tx * ts, ts - 1), ly1 = min(y1 - ty * ts, ts - 1);
                const uint32_t fp = (uint32_t)lx0 | ((uint32_t)ly0 << 8) | ((uint32_t)(lx1 - lx0 + 1) << 16) |
                                    ((uint32_t)(ly1 - ly0 + 1) << 24);
                PrimRec* dst = &list[atomicAdd(&cur[t], 1u)];
                dst->g0 = g0;
                dst->g1 = make_uint4(g1.x, g1.y, g1.z, fp);
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

template <class JS>
hipError_t count_impl(const JS& js, bool scene, uint32_t grid, int max_tiles, hipStream_t stream) {
    if (max_tiles > kMaxLdsTiles) return hipErrorInvalidValue;
    if (grid == 0) return hipSuccess;
    const size_t lds = (size_t)max_tiles * sizeof(uint32_t);
    if (scene) k_count<JS, true><<<grid, kBinThreads, lds, stream>>>(js);
    else k_count<JS, false><<<grid, kBinThreads, lds, stream>>>(js);
    return hipGetLastError();
}

template <class JS>
hipError_t scatter_impl(const JS& js, uint32_t grid, int max_tiles, hipStream_t stream) {
    if (max_tiles > kMaxLdsTiles) return hipErrorInvalidValue;
    if (grid == 0) return hipSuccess;
    k_scatter<JS><<<grid, kBinThreads, (size_t)max_tiles * sizeof(uint32_t), stream>>>(js);
    return hipGetLastError();
}

hipError_t launch_count(const OneJob& js, bool scene, uint32_t grid, int max_tiles, hipStream_t stream) {
    return count_impl(js, scene, grid, max_tiles, stream);
}
hipError_t launch_count(const JobList& js, bool scene, uint32_t grid, int max_tiles, hipStream_t stream) {
    return count_impl(js, scene, grid, max_tiles, stream);
}
hipError_t launch_scatter(const OneJob& js, uint32_t grid, int max_tiles, hipStream_t stream) {
    return scatter_impl(js, grid, max_tiles, stream);
}
hipError_t launch_scatter(const JobList& js, uint32_t grid, int max_tiles, hipStream_t stream) {
    return scatter_impl(js, grid, max_tiles, stream);
}

}  // namespace vtx
