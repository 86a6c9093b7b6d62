// Resident scenes: the molecule's arrays kept in device memory across frames
// in a layout made for the per-frame passes (paper, Methods, "Molecular
// Graphics Engine": adapted data structures for millions of atoms).
//
// At creation the atoms are reordered along a Morton curve of their
// positions and stored as one xyzr float4 stream, so that every run of 256
// stored atoms (a cluster) is compact in space: a cluster's bounding box is
// tested against the frustum once per frame (which also files it under a
// depth class, for front-to-back binning), and the atoms a binning
// workgroup handles fall on few screen tiles.  Each stored atom keeps its
// original index, which is the id the renderer reports, so a resident scene
// renders exactly what the same arrays render through vtx_render.  Bonds
// are re-indexed to stored positions and sorted by their first atom, in
// clusters of 256 as well.  Both orders come from the stable radix sort of
// sort.hip, so atoms with equal Morton keys keep their original order, and so
// do bonds with the same first atom.
#include "vtx_internal.h"

namespace vtx {

namespace {

// Order-preserving map of a float to an unsigned int (for atomic min/max).
__device__ inline uint32_t ordered_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float from_ordered(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// Bounding box of the atom positions: box[0..2] min, box[3..5] max (ordered bits).
__global__ void __launch_bounds__(kBlock) k_bbox(const float* __restrict__ pos, uint32_t n, uint32_t* box) {
    __shared__ uint32_t sb[6];
    if (threadIdx.x < 6) sb[threadIdx.x] = threadIdx.x < 3 ? 0xFFFFFFFFu : 0u;
    __syncthreads();
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int k = 0; k < 3; ++k) {
            const uint32_t v = ordered_bits(pos[3 * (size_t)i + k]);
            lo[k] = min(lo[k], v);
            hi[k] = max(hi[k], v);
        }
    for (int k = 0; k < 3; ++k) {
        atomicMin(&sb[k], lo[k]);
        atomicMax(&sb[3 + k], hi[k]);
    }
    __syncthreads();
    if (threadIdx.x < 3) atomicMin(&box[threadIdx.x], sb[threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&box[threadIdx.x], sb[threadIdx.x]);
}

__global__ void k_box_init(uint32_t* box) {
    if (threadIdx.x < 6) box[threadIdx.x] = threadIdx.x < 3 ? 0xFFFFFFFFu : 0u;
}

// 30-bit Morton key (10 bits per axis) of each atom, and the identity payload.
__device__ inline uint32_t spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void __launch_bounds__(kBlock) k_morton(const float* __restrict__ pos, uint32_t n,
                                                   const uint32_t* __restrict__ box, uint32_t* keys, uint32_t* idx) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t key = 0;
    for (int k = 0; k < 3; ++k) {
        const float lo = from_ordered(box[k]), hi = from_ordered(box[3 + k]);
        const float ext = hi - lo;
        float u = ext > 0.0f ? (pos[3 * (size_t)i + k] - lo) / ext : 0.0f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const uint32_t q = min((uint32_t)(u * 1024.0f), 1023u);
        key |= spread10(q) << k;
    }
    keys[i] = key;
    idx[i] = i;
}

// Stored atom i is original atom atom_id[i].
__global__ void __launch_bounds__(kBlock) k_gather_atoms(const float* __restrict__ pos, const float* __restrict__ rad,
                                                         const uint32_t* __restrict__ atom_id, uint32_t n,
                                                         float4* xyzr, uint32_t* inv) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t a = atom_id[i];
    xyzr[i] = make_float4(pos[3 * (size_t)a], pos[3 * (size_t)a + 1], pos[3 * (size_t)a + 2], rad[a]);
    if (inv) inv[a] = i;
}

// New positions for a trajectory frame (radii kept).
// New positions of the stored atoms; the radii come from the scene's own
// stream (`rsrc`, which may be `xyzr` itself).
__global__ void __launch_bounds__(kBlock) k_update_positions(const float* __restrict__ pos,
                                                             const uint32_t* __restrict__ atom_id, uint32_t n,
                                                             const float4* rsrc, float4* xyzr) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t a = atom_id[i];
    const float r = rsrc[i].w;
    xyzr[i] = make_float4(pos[3 * (size_t)a], pos[3 * (size_t)a + 1], pos[3 * (size_t)a + 2], r);
}

// Sort key of bond b: stored index of its first atom (bonds with an index out
// of range get the largest key and are dropped).
__global__ void __launch_bounds__(kBlock) k_bond_keys(const uint32_t* __restrict__ bonds, uint32_t m, uint32_t n,
                                                      const uint32_t* __restrict__ inv, uint32_t* keys, uint32_t* idx,
                                                      uint32_t* n_bad) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m) return;
    const uint32_t ia = bonds[2 * (size_t)b], ib = bonds[2 * (size_t)b + 1];
    const bool ok = ia < n && ib < n;
    keys[b] = ok ? min(inv[ia], inv[ib]) : 0xFFFFFFFFu;
    idx[b] = b;
    if (!ok) atomicAdd(n_bad, 1u);
}

__global__ void __launch_bounds__(kBlock) k_bond_records(const uint32_t* __restrict__ bonds,
                                                         const uint32_t* __restrict__ order, uint32_t m_valid,
                                                         const uint32_t* __restrict__ inv, uint4* rec) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_valid) return;
    const uint32_t b = order[j];
    rec[j] = make_uint4(inv[bonds[2 * (size_t)b]], inv[bonds[2 * (size_t)b + 1]], b, 0u);
}

// Bounding box of each cluster: atoms (centre +- radius), bonds (both
// endpoints; the bond radius is added per frame).  One wave per cluster.
__global__ void __launch_bounds__(kBlock) k_cluster_boxes(SceneDev S, float4* box) {
    const uint32_t c = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = __lane_id();
    const uint32_t nc = S.atom_clusters + S.bond_clusters;
    if (c >= nc) return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int s = lane; s < kCluster; s += 64) {
        if (c < S.atom_clusters) {
            const uint32_t i = c * kCluster + s;
            if (i >= S.n_atoms) continue;
            const float4 a = S.xyzr[i];
            const float p[3] = {a.x, a.y, a.z};
            for (int k = 0; k < 3; ++k) {
                lo[k] = fminf(lo[k], p[k] - a.w);
                hi[k] = fmaxf(hi[k], p[k] + a.w);
            }
        } else {
            const uint32_t j = (c - S.atom_clusters) * kCluster + s;
            if (j >= S.n_bonds) continue;
            const uint4 br = S.bond_rec[j];
            const float4 a = S.xyzr[br.x], b = S.xyzr[br.y];
            const float pa[3] = {a.x, a.y, a.z}, pb[3] = {b.x, b.y, b.z};
            for (int k = 0; k < 3; ++k) {
                lo[k] = fminf(lo[k], fminf(pa[k], pb[k]));
                hi[k] = fmaxf(hi[k], fmaxf(pa[k], pb[k]));
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], o));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o));
        }
    if (lane == 0) {
        box[2 * (size_t)c] = make_float4(lo[0], lo[1], lo[2], 0.0f);
        box[2 * (size_t)c + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    }
}

// Per frame: clusters whose bounding sphere meets the view volume, appended
// (with kClusterInside when the sphere lies wholly inside it) to the region
// of S.vis_clusters of their depth class: the front depth of
// the bounding sphere on a log scale (Frame::cls_z0, cls_k), kDepthBuckets
// classes.  A workgroup's clusters of one class (neighbours in Morton order)
// take one contiguous run of that class, so a range of the class stays
// compact in space.
template <class JS>
__global__ void __launch_bounds__(kBlock) k_cluster_cull(JS js) {
    __shared__ uint32_t wcnt[kDepthBuckets], wbase[kDepthBuckets];
    uint32_t blk;
    const int ji = js.find(blockIdx.x, blk);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const Frame F = J.F;
    const SceneDev S = J.S;
    Counters* const ctr = J.bb.ctr;
    const uint32_t stride = S.atom_clusters + S.bond_clusters;   // entries of one depth class
    const uint32_t nc = S.atom_clusters + (F.n_bonds ? S.bond_clusters : 0u);
    const uint32_t c = blk * kBlock + threadIdx.x;
    if (threadIdx.x < kDepthBuckets) wcnt[threadIdx.x] = 0;
    if (blk == 0 && threadIdx.x < 2 * kLayers)   // the count kernel lowers these
        ctr->layer_zlo[threadIdx.x / kLayers][threadIdx.x % kLayers] = 0x7F800000u;
    __syncthreads();
    int cls = -1;
    bool inside = false;
    if (c < nc) {
        const float4 lo = S.cluster_box[2 * (size_t)c], hi = S.cluster_box[2 * (size_t)c + 1];
        if (lo.x <= hi.x) {   // empty clusters have an inverted box
            // atom boxes hold the given radii: the representation may draw
            // larger spheres (sticks, solvent-accessible surface)
            const float pad = c < S.atom_clusters ? (F.rep == 2 ? F.bond_radius : F.rep == 3 ? F.probe : 0.0f)
                                                  : F.bond_radius;
            const double hx = 0.5 * ((double)hi.x - lo.x), hy = 0.5 * ((double)hi.y - lo.y),
                         hz = 0.5 * ((double)hi.z - lo.z);
            double vx, vy, vz;
            to_view(F, (float)(lo.x + hx), (float)(lo.y + hy), (float)(lo.z + hz), vx, vy, vz);
            // the centre was rounded to FP32: widen by its rounding error
            const double r = sqrt(hx * hx + hy * hy + hz * hz) + pad +
                             1e-6 * (fabs((double)lo.x) + fabs((double)lo.y) + fabs((double)lo.z) + 1.0);
            if (sphere_in_frustum(F, vx, vy, vz, r)) {
                // only the order of the lists depends on the class, never the image
                const float zf = fmaxf((float)(vz - r), F.cls_z0);
                const float q = __log2f(zf / F.cls_z0) * F.cls_k;
                cls = q >= 0.0f ? (int)fminf(q, (float)(kDepthBuckets - 1)) : 0;   // NaN: class 0
                inside = sphere_inside_frustum(F, vx, vy, vz, r);
            }
        }
    }
    // place within the workgroup's run of the class (lanes sharing a class
    // take one LDS atomic), then one global atomic per class
    uint32_t off = 0;
    unsigned long long pend = __ballot(cls >= 0);
    while (pend) {
        const int leader = __ffsll((long long)pend) - 1;
        const int cl = __shfl(cls, leader);
        const unsigned long long grp = __ballot(cls == cl) & pend;
        uint32_t base = 0;
        if ((int)__lane_id() == leader) base = atomicAdd(&wcnt[cl], (uint32_t)__popcll(grp));
        base = __shfl(base, leader);
        if ((grp >> __lane_id()) & 1ull) off = base + (uint32_t)__popcll(grp & __lanemask_lt());
        pend &= ~grp;
    }
    __syncthreads();
    if (threadIdx.x < kDepthBuckets && wcnt[threadIdx.x])
        wbase[threadIdx.x] = atomicAdd(&ctr->vis_bucket[threadIdx.x], wcnt[threadIdx.x]);
    __syncthreads();
    if (cls >= 0) S.vis_clusters[(size_t)cls * stride + wbase[cls] + off] = c | (inside ? kClusterInside : 0u);
}

inline unsigned grid_for(uint64_t n) {
    const uint64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

// Device-side construction of a resident scene; see the comment at the top.
// `tmp` needs scene_build_temp_bytes(n, m) bytes.  Returns the number of
// valid bonds in *m_valid (synchronizes the stream).
size_t scene_build_temp_bytes(uint64_t n, uint64_t m) {
    const uint64_t mx = n > m ? n : m;
    // keys in/out, payload in/out, inverse permutation, box and bad count,
    // sort scratch, plus the 256-byte alignment of each of those pieces
    return 4 * sizeof(uint32_t) * (size_t)(mx ? mx : 1) + sizeof(uint32_t) * (size_t)(n ? n : 1) + 64 +
           sizeof(uint32_t) * radix_sort_scratch_words((size_t)mx) + 8 * 256;
}

hipError_t scene_build(const float* pos, const float* rad, const uint32_t* bonds, uint64_t n, uint64_t m,
                       SceneDev& S, float4* xyzr, uint32_t* atom_id, uint4* bond_rec, float4* cluster_box,
                       void* tmp, size_t tmp_bytes, uint32_t* m_valid, uint32_t* n_bad, uint32_t* box_bits,
                       hipStream_t stream) {
    const uint64_t mx = n > m ? n : m;
    char* p = static_cast<char*>(tmp);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += (bytes + 255) & ~(size_t)255;
        return q;
    };
    uint32_t* kin = (uint32_t*)take(sizeof(uint32_t) * (mx ? mx : 1));
    uint32_t* kout = (uint32_t*)take(sizeof(uint32_t) * (mx ? mx : 1));
    uint32_t* vin = (uint32_t*)take(sizeof(uint32_t) * (mx ? mx : 1));
    uint32_t* vout = (uint32_t*)take(sizeof(uint32_t) * (mx ? mx : 1));
    uint32_t* inv = (uint32_t*)take(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* box = (uint32_t*)take(64);
    uint32_t* bad = box + 8;
    uint32_t* sort_tmp = (uint32_t*)take(sizeof(uint32_t) * radix_sort_scratch_words((size_t)mx));
    if ((size_t)(p - static_cast<char*>(tmp)) > tmp_bytes) return hipErrorOutOfMemory;
    hipError_t e;
    k_box_init<<<1, 64, 0, stream>>>(box);
    if ((e = launch_zero(bad, 1, stream)) != hipSuccess) return e;
    if (n) {
        k_bbox<<<grid_for(n) < 1024 ? grid_for(n) : 1024, kBlock, 0, stream>>>(pos, (uint32_t)n, box);
        k_morton<<<grid_for(n), kBlock, 0, stream>>>(pos, (uint32_t)n, box, kin, vin);
        if ((e = radix_sort_pairs(kin, kout, vin, vout, atom_id, (size_t)n, 30, sort_tmp, stream)) != hipSuccess)
            return e;
        k_gather_atoms<<<grid_for(n), kBlock, 0, stream>>>(pos, rad, atom_id, (uint32_t)n, xyzr, inv);
    }
    uint32_t mv = 0, nb = 0;
    if (m) {
        k_bond_keys<<<grid_for(m), kBlock, 0, stream>>>(bonds, (uint32_t)m, (uint32_t)n, inv, kin, vin, bad);
        // sorted bond indices land in vin
        if ((e = radix_sort_pairs(kin, kout, vin, vout, vin, (size_t)m, 32, sort_tmp, stream)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(&nb, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
        mv = (uint32_t)m - nb;
        if (mv) k_bond_records<<<grid_for(mv), kBlock, 0, stream>>>(bonds, vin, mv, inv, bond_rec);
    }
    S.n_bonds = mv;
    S.bond_clusters = (mv + kCluster - 1) / kCluster;
    S.atom_clusters = (uint32_t)((n + kCluster - 1) / kCluster);
    S.cluster_box = cluster_box;
    const uint32_t nc = S.atom_clusters + S.bond_clusters;
    if (nc) k_cluster_boxes<<<grid_for((uint64_t)nc * 64), kBlock, 0, stream>>>(S, cluster_box);
    *m_valid = mv;
    *n_bad = nb;
    // the atoms' bounding box (order-preserving bits, min xyz then max xyz),
    // host memory, valid once the stream has reached this point
    if ((e = hipMemcpyAsync(box_bits, box, 6 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
    return hipGetLastError();
}

// Original index of each stored bond.
__global__ void __launch_bounds__(kBlock) k_bond_order(const uint4* __restrict__ rec, uint32_t m, uint32_t* out) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) out[j] = rec[j].z;
}

hipError_t scene_order(const SceneDev& S, uint32_t* atom_order, uint32_t* bond_order, hipStream_t stream) {
    hipError_t e;
    if (atom_order && S.n_atoms &&
        (e = hipMemcpyAsync(atom_order, S.atom_id, sizeof(uint32_t) * S.n_atoms, hipMemcpyDeviceToDevice, stream)))
        return e;
    if (bond_order && S.n_bonds) k_bond_order<<<grid_for(S.n_bonds), kBlock, 0, stream>>>(S.bond_rec, S.n_bonds, bond_order);
    return hipGetLastError();
}

// Writes the atom stream `xyzr` and the cluster boxes of new positions `pos`
// (caller's order) in the scene's stored order; radii are read from S.xyzr.
// `xyzr` may be S.xyzr (in-place update) or another frame's stream.
hipError_t scene_update_positions(const float* pos, SceneDev& S, float4* xyzr, float4* cluster_box,
                                  hipStream_t stream) {
    if (S.n_atoms)
        k_update_positions<<<grid_for(S.n_atoms), kBlock, 0, stream>>>(pos, S.atom_id, S.n_atoms, S.xyzr, xyzr);
    const uint32_t nc = S.atom_clusters + S.bond_clusters;
    SceneDev Sf = S;
    Sf.xyzr = xyzr;
    if (nc) k_cluster_boxes<<<grid_for((uint64_t)nc * 64), kBlock, 0, stream>>>(Sf, cluster_box);
    return hipGetLastError();
}

template <class JS>
hipError_t cull_impl(const JS& js, uint32_t grid, hipStream_t stream) {
    if (grid == 0) return hipSuccess;
    return dispatch(k_cluster_cull<JS>, grid, kBlock, 0, stream, js);
}

hipError_t launch_cluster_cull(const OneJob& js, uint32_t grid, hipStream_t stream) { return cull_impl(js, grid, stream); }
hipError_t launch_cluster_cull(const JobList& js, uint32_t grid, hipStream_t stream) { return cull_impl(js, grid, stream); }

}  // namespace vtx
