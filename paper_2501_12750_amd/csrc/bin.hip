// Screen-tile binning of atoms and bonds (a prefix-sum binner).
//
// The paper rasterizes one screen quad per primitive and lets the fixed
// function rasterizer find the pixels it covers (Methods, "Meshless
// Representations").  Here the quad's role, a conservative footprint, becomes
// an exact tile rectangle computed per primitive, and the rasterizer becomes
// three compute passes:
//   project  each primitive -> view space (FP64), cull, footprint rectangle,
//            one count per covered tile, compacted list of visible primitives;
//   scan     exclusive prefix sum of the tile counts -> list offsets;
//   scatter  each visible primitive id into the lists of its tiles.
// Lists that would not fit the bin capacity are left empty; the resolve pass
// finds their tiles from the compacted visible list instead, so every frame
// is exact whatever the capacity.
#include "vtx_internal.h"

namespace vtx {

namespace {

__global__ void __launch_bounds__(kBlock) k_clear(uint32_t* tile_cnt, int T, Counters* ctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) tile_cnt[i] = 0;
    if (i < (int)(sizeof(Counters) / sizeof(unsigned int))) reinterpret_cast<unsigned int*>(ctr)[i] = 0;
}

__device__ inline bool primitive_rect(const Frame& F, uint32_t p, const float* __restrict__ pos,
                                      const float* __restrict__ rad, const uint32_t* __restrict__ bonds,
                                      int& x0, int& y0, int& x1, int& y1, bool& bad) {
    bad = false;
    if (p < F.n_atoms) {
        double vx, vy, vz;
        to_view(F, pos[3 * (size_t)p], pos[3 * (size_t)p + 1], pos[3 * (size_t)p + 2], vx, vy, vz);
        return sphere_rect(F, vx, vy, vz, (double)rad[p], x0, y0, x1, y1);
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
    return bond_rect(F, A, B, (double)F.bond_radius, x0, y0, x1, y1);
}

// One lane per primitive.  Visible primitives get a slot in the compacted
// list (one atomic per wave), and every tile of their rectangle one count.
__global__ void __launch_bounds__(kBlock) k_project(Frame F, const float* __restrict__ pos,
                                                    const float* __restrict__ rad,
                                                    const uint32_t* __restrict__ bonds, uint32_t* tile_cnt,
                                                    uint32_t* vis_id, uint2* vis_rect, Counters* ctr) {
    const uint64_t total = (uint64_t)F.n_atoms + F.n_bonds;
    const int ts = F.tile;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < total;
         base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = base + threadIdx.x;
        int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
        bool bad = false;
        const bool vis = p < total && primitive_rect(F, (uint32_t)p, pos, rad, bonds, x0, y0, x1, y1, bad);
        const unsigned long long vmask = __ballot(vis);
        const unsigned long long bmask = __ballot(bad);
        uint32_t slot_base = 0;
        const int leader = __ffsll((long long)(vmask | 1ull)) - 1;
        if (vmask && (int)__lane_id() == leader) slot_base = atomicAdd(&ctr->vis_count, (uint32_t)__popcll(vmask));
        if (bmask && __lane_id() == 0) atomicAdd(&ctr->bad_bonds, (uint32_t)__popcll(bmask));
        slot_base = __shfl(slot_base, leader);
        if (vis) {
            const uint32_t slot = slot_base + (uint32_t)__popcll(vmask & __lanemask_lt());
            const int tx0 = x0 / ts, tx1 = x1 / ts, ty0 = y0 / ts, ty1 = y1 / ts;
            vis_id[slot] = (uint32_t)p;
            vis_rect[slot] = make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16));
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&tile_cnt[ty * F.tiles_x + tx], 1u);
        }
    }
}

// Exclusive scan of the tile counts by one workgroup of 1024 lanes: each lane
// sums a contiguous run, the run totals are scanned in LDS, then each lane
// writes its run's offsets.  Also clears the scatter cursors.
constexpr int kScanThreads = 1024;

__global__ void __launch_bounds__(kScanThreads) k_scan(const uint32_t* __restrict__ cnt, uint64_t* off,
                                                       uint32_t* fill, int T, uint64_t capacity, Counters* ctr) {
    __shared__ unsigned long long part[kScanThreads];
    const int tid = threadIdx.x;
    const int per = (T + kScanThreads - 1) / kScanThreads;
    const int b = tid * per, e = min(T, b + per);
    unsigned long long s = 0;
    for (int i = b; i < e; ++i) s += cnt[i];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const unsigned long long v = tid >= d ? part[tid - d] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    unsigned long long run = part[tid] - s;   // exclusive prefix of this lane's run
    for (int i = b; i < e; ++i) {
        off[i] = run;
        fill[i] = 0;
        run += cnt[i];
    }
    if (tid == kScanThreads - 1) {
        ctr->pairs = part[tid];
        ctr->overflow = part[tid] > capacity ? 1u : 0u;
    }
}

__global__ void __launch_bounds__(kBlock) k_scatter(Frame F, const uint32_t* __restrict__ vis_id,
                                                    const uint2* __restrict__ vis_rect,
                                                    const uint32_t* __restrict__ cnt,
                                                    const uint64_t* __restrict__ off, uint32_t* fill,
                                                    uint32_t* list, uint64_t capacity, const Counters* ctr) {
    const uint32_t nvis = ctr->vis_count;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nvis; k += gridDim.x * blockDim.x) {
        const uint32_t id = vis_id[k];
        const uint2 r = vis_rect[k];
        const int tx0 = r.x & 0xFFFF, ty0 = r.x >> 16, tx1 = r.y & 0xFFFF, ty1 = r.y >> 16;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                const int t = ty * F.tiles_x + tx;
                const uint64_t o = off[t];
                if (o + cnt[t] <= capacity) {
                    const uint32_t slot = atomicAdd(&fill[t], 1u);
                    list[o + slot] = id;
                }
            }
    }
}

}  // namespace

hipError_t launch_bin(const Frame& F, const float* pos, const float* rad, const uint32_t* bonds,
                      const BinBuffers& bb, hipStream_t stream, hipEvent_t* marks) {
    const int T = F.tiles_x * F.tiles_y;
    const int nclear = T > 64 ? T : 64;
    if (marks) (void)hipEventRecord(marks[0], stream);
    k_clear<<<(nclear + kBlock - 1) / kBlock, kBlock, 0, stream>>>(bb.tile_cnt, T, bb.ctr);
    const uint64_t total = (uint64_t)F.n_atoms + F.n_bonds;
    if (marks) (void)hipEventRecord(marks[1], stream);
    if (total > 0) {
        const uint64_t want = (total + kBlock - 1) / kBlock;
        const int grid = (int)(want < 8192 ? want : 8192);
        k_project<<<grid, kBlock, 0, stream>>>(F, pos, rad, bonds, bb.tile_cnt, bb.vis_id, bb.vis_rect, bb.ctr);
    }
    if (marks) (void)hipEventRecord(marks[2], stream);
    k_scan<<<1, kScanThreads, 0, stream>>>(bb.tile_cnt, bb.tile_off, bb.tile_fill, T, bb.capacity, bb.ctr);
    if (marks) (void)hipEventRecord(marks[3], stream);
    if (total > 0) {
        const uint64_t want = (total + kBlock - 1) / kBlock;
        const int grid = (int)(want < 4096 ? want : 4096);
        k_scatter<<<grid, kBlock, 0, stream>>>(F, bb.vis_id, bb.vis_rect, bb.tile_cnt, bb.tile_off,
                                                bb.tile_fill, bb.list, bb.capacity, bb.ctr);
    }
    return hipGetLastError();
}

}  // namespace vtx
