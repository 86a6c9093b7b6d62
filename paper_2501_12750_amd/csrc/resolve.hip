// Per-tile visibility resolve: ray-cast every pixel of a tile against the
// primitives binned to it and keep the nearest hit (paper, Methods,
// "Meshless Representations": ray-casting evaluates the implicit equation of
// each primitive, which makes the display pixel-exact).
//
// One workgroup owns one tile.  The tile's list holds 32-byte view-space
// records with the footprint clipped to the tile, so it is read contiguously
// with no gathers.  Records are staged through LDS 256 at a time; their
// footprints' pixel counts are prefix-summed and the resulting (record,
// pixel) fragments are dealt to the 256 lanes round-robin, so the load is
// balanced whatever the mix of tiny and large primitives.  A hit is folded into the tile's depth
// buffer in LDS with one 64-bit atomicMin of the packed key
// (float bits of z) << 32 | id: positive floats order like their bit
// patterns, so the minimum key is the nearest hit and equal depths go to the
// smaller id, in any order of evaluation.  Depth early-outs skip a record
// whose nearest possible depth lies behind everything the tile already
// holds, and a fragment whose pixel already holds a nearer hit.
#include "vtx_internal.h"

namespace vtx {

namespace {

constexpr int kChunk = kBlock;

struct Rec {
    float4 a;          // sphere: centre (view), radius | cylinder: A (view), radius
    float4 b;          // cylinder: unit axis (view), length
    float zcull;       // lower bound of the depth of any hit of this record
    uint32_t id;
    uint32_t rect;     // tile-local x0 | y0 << 8 | w << 16 | h << 24
    uint32_t kind;     // 0 sphere, 1 cylinder
};

__device__ inline float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Sphere: front root of |o + t D - c| = r with D = (Dx, Dy, 1), so t is the
// view depth.  Stable form: b = (c-o).D / D.D, q = (c-o) - b D,
// t = b - sqrt((r^2 - q.q) / D.D).
__device__ inline float hit_sphere(const float4 s, float ox, float oy, float Dx, float Dy) {
    const float cx = s.x - ox, cy = s.y - oy, cz = s.z;
    const float dd = fmaf(Dx, Dx, fmaf(Dy, Dy, 1.0f));
    const float b = fmaf(cx, Dx, fmaf(cy, Dy, cz)) / dd;
    const float qx = fmaf(-b, Dx, cx), qy = fmaf(-b, Dy, cy), qz = cz - b;
    const float disc = fmaf(s.w, s.w, -fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
    if (disc < 0.0f) return INFINITY;
    return b - sqrtf(disc / dd);
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
        const float tc = -fmaf(qx, px, fmaf(qy, py, qz * pz)) / k;
        const float rx = fmaf(tc, px, qx), ry = fmaf(tc, py, qy), rz = fmaf(tc, pz, qz);
        const float disc = rho2 - fmaf(rx, rx, fmaf(ry, ry, rz * rz));
        if (disc >= 0.0f) {
            const float ts = tc - sqrtf(disc / k);
            const float s = fmaf(ts, da, wa);
            if (s >= 0.0f && s <= cb.w) t = ts;
        }
    }
    if (da != 0.0f) {
        const float tp = (da > 0.0f ? -wa : cb.w - wa) / da;
        const float off = da > 0.0f ? 0.0f : cb.w;
        const float ex = fmaf(tp, Dx, wx) - off * cb.x;
        const float ey = fmaf(tp, Dy, wy) - off * cb.y;
        const float ez = (tp + wz) - off * cb.z;
        if (fmaf(ex, ex, fmaf(ey, ey, ez * ez)) <= rho2) t = fminf(t, tp);
    }
    return t;
}

// Expand a list record into the LDS form.
__device__ inline Rec make_rec(const Frame& F, const PrimRec& p) {
    Rec r;
    r.id = p.g1.z;
    r.rect = p.g1.w;
    if (r.id < F.n_atoms) {
        r.a = p.g0;
        r.b = make_float4(0.f, 0.f, 0.f, 0.f);
        r.zcull = (p.g0.z - p.g0.w) * (1.0f - 1e-5f);
        r.kind = 0;
    } else {
        const float dx = p.g0.w, dy = __uint_as_float(p.g1.x), dz = __uint_as_float(p.g1.y);
        const float L = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        const float inv = 1.0f / L;
        const float rho = F.bond_radius;
        r.a = make_float4(p.g0.x, p.g0.y, p.g0.z, rho);
        r.b = make_float4(dx * inv, dy * inv, dz * inv, L);
        r.zcull = (fminf(p.g0.z, p.g0.z + dz) - rho) * (1.0f - 1e-5f) - 1e-6f;
        r.kind = 1;
    }
    return r;
}

template <int TS>
__global__ void __launch_bounds__(kBlock) k_resolve(Frame F, uint32_t* __restrict__ cnt,
                                                    const uint64_t* __restrict__ off,
                                                    const PrimRec* __restrict__ list, uint64_t capacity,
                                                    const PrimRec* __restrict__ vis_rec,
                                                    const uint2* __restrict__ vis_rect,
                                                    const uint32_t* __restrict__ vis_cnt, uint32_t chunk,
                                                    uint32_t groups, Counters* ctr, Counters* host_ctr,
                                                    float* __restrict__ depth, uint32_t* __restrict__ out_id) {
    __shared__ unsigned long long keys[TS * TS];
    __shared__ Rec recs[kChunk];
    __shared__ uint32_t pref[kChunk + 1];
    __shared__ uint32_t wsum[kBlock / 64];
    __shared__ float wmax[kBlock / 64];

    const int T = F.tiles_x * F.tiles_y;
    const int t = xcd_contiguous(blockIdx.x, T);
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const bool stats = (F.flags & 1u) != 0;
    unsigned long long n_tested = 0, n_hit = 0, n_hit_bond = 0;

    if (t < T) {
        const int tx = t % F.tiles_x, ty = t / F.tiles_x;
        const int px0 = tx * TS, py0 = ty * TS;
        const int tw = min(TS, F.W - px0), th = min(TS, F.H - py0);
        for (int i = tid; i < TS * TS; i += kBlock) keys[i] = ~0ull;

        const uint32_t n = cnt[t];
        const uint64_t o = off[t];
        if (tid == 0) cnt[t] = 0;   // re-armed for the next frame's count kernel (no later reader)
        // a tile whose list did not fit the bins scans every workgroup's visible list
        const bool overflow = o + n > capacity;
        const uint64_t nsrc = overflow ? (uint64_t)groups * chunk : n;
        const bool persp = F.proj == 0;
        float tile_zmax = INFINITY;
        __syncthreads();

        for (uint64_t base = 0; base < nsrc; base += kChunk) {
            const uint64_t k = base + tid;
            uint32_t area = 0;
            bool take = false;
            PrimRec pr;
            if (k < nsrc) {
                if (!overflow) {
                    pr = list[o + k];
                    take = true;
                } else {
                    const uint32_t g = (uint32_t)(k / chunk);
                    if ((uint32_t)(k - (uint64_t)g * chunk) < vis_cnt[g]) {
                        const uint2 r = vis_rect[k];
                        const int x0 = max((int)(r.x & 0xFFFF), px0) - px0, y0 = max((int)(r.x >> 16), py0) - py0;
                        const int x1 = min((int)(r.y & 0xFFFF), px0 + TS - 1) - px0;
                        const int y1 = min((int)(r.y >> 16), py0 + TS - 1) - py0;
                        if (x0 <= x1 && y0 <= y1) {
                            pr = vis_rec[k];
                            pr.g1.w = (uint32_t)x0 | ((uint32_t)y0 << 8) | ((uint32_t)(x1 - x0 + 1) << 16) |
                                      ((uint32_t)(y1 - y0 + 1) << 24);
                            take = true;
                        }
                    }
                }
            }
            if (take) {
                const Rec rec = make_rec(F, pr);
                if (stats || !(rec.zcull > tile_zmax)) {
                    area = ((rec.rect >> 16) & 0xFF) * (rec.rect >> 24);
                    recs[tid] = rec;
                }
            }
            // exclusive prefix of the fragment counts over the workgroup
            const uint32_t incl = wave_incl_scan(area);
            if (lane == 63) wsum[wave] = incl;
            __syncthreads();
            uint32_t wbase = 0;
            for (int w = 0; w < wave; ++w) wbase += wsum[w];
            pref[tid] = wbase + incl - area;
            if (tid == kBlock - 1) pref[kChunk] = wbase + incl;
            __syncthreads();
            const uint32_t total = pref[kChunk];

            // fragments are dealt round-robin: the 64 lanes of a wave take 64
            // consecutive fragments, i.e. neighbouring pixels of a few
            // adjacent records of the same kind
            for (uint32_t f = tid; f < total; f += kBlock) {
                int lo = 0, hi = kChunk;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (pref[mid] <= f) lo = mid;
                    else hi = mid;
                }
                const Rec& rc = recs[lo];
                const uint32_t local = f - pref[lo];
                const uint32_t rw = (rc.rect >> 16) & 0xFF;
                // exact: local < 4096 and rw <= 64, so the rounding error of
                // (local + 1/2) / rw is far below its distance to an integer
                const uint32_t dy = (uint32_t)(((float)local + 0.5f) * __builtin_amdgcn_rcpf((float)rw));
                const uint32_t dx = local - dy * rw;
                const int lx = (int)(rc.rect & 0xFF) + (int)dx, ly = (int)((rc.rect >> 8) & 0xFF) + (int)dy;
                const int slot = ly * TS + lx;
                if (!stats) {
                    const unsigned long long cur = keys[slot];
                    if (__uint_as_float((uint32_t)(cur >> 32)) < rc.zcull) continue;
                }
                const float ndx = fmaf((float)(px0 + lx) + 0.5f, F.inv_w2, -1.0f);
                const float ndy = fmaf(-((float)(py0 + ly) + 0.5f), F.inv_h2, 1.0f);
                float ox, oy, Dx, Dy;
                if (persp) {
                    ox = 0.f; oy = 0.f; Dx = ndx * F.txf; Dy = ndy * F.tyf;
                } else {
                    ox = ndx * F.hxf; oy = ndy * F.hyf; Dx = 0.f; Dy = 0.f;
                }
                const float z = rc.kind == 0 ? hit_sphere(rc.a, ox, oy, Dx, Dy)
                                             : hit_cylinder(rc.a, rc.b, ox, oy, Dx, Dy);
                const bool hit = z >= F.znear && z <= F.zfar;
                if (stats) {
                    n_tested += 1;
                    n_hit += hit ? 1 : 0;
                    n_hit_bond += (hit && rc.kind == 1) ? 1 : 0;
                }
                if (hit) {
                    const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | rc.id;
                    atomicMin(&keys[slot], key);
                }
            }
            __syncthreads();
            if (!stats && base + kChunk < nsrc) {
                float m = 0.0f;
                for (int i = tid; i < TS * TS; i += kBlock) {
                    const int ly = i / TS, lx = i - ly * TS;
                    if (lx < tw && ly < th) {
                        const unsigned long long kk = keys[i];
                        m = fmaxf(m, kk == ~0ull ? INFINITY : __uint_as_float((uint32_t)(kk >> 32)));
                    }
                }
                m = wave_max(m);
                if (lane == 0) wmax[wave] = m;
                __syncthreads();
                tile_zmax = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
                __syncthreads();
            }
        }

        for (int i = tid; i < TS * TS; i += kBlock) {
            const int ly = i / TS, lx = i - ly * TS;
            if (lx < tw && ly < th) {
                const unsigned long long kk = keys[i];
                const size_t p = (size_t)(py0 + ly) * F.W + (px0 + lx);
                depth[p] = kk == ~0ull ? INFINITY : __uint_as_float((uint32_t)(kk >> 32));
                out_id[p] = kk == ~0ull ? kBackground : (uint32_t)(kk & 0xFFFFFFFFull);
            }
        }
    }
    if (stats) {
        unsigned long long a = n_tested, b = n_hit, c = n_hit_bond;
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
            a += __shfl_xor(a, o2);
            b += __shfl_xor(b, o2);
            c += __shfl_xor(c, o2);
        }
        if (lane == 0 && a) {
            atomicAdd(&ctr->frag_tested, a);
            atomicAdd(&ctr->frag_hit, b);
            atomicAdd(&ctr->frag_hit_bond, c);
        }
    }
    // with exact fragment counting on, the last workgroup to finish publishes
    // the fragment counters to the host-mapped copy
    if (stats && host_ctr) {
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            const unsigned int ticket = atomicAdd(&ctr->done_blocks, 1u);
            if (ticket == gridDim.x - 1) {
                __threadfence();
                const volatile Counters* src = ctr;
                host_ctr->frag_tested = src->frag_tested;
                host_ctr->frag_hit = src->frag_hit;
                host_ctr->frag_hit_bond = src->frag_hit_bond;
                __threadfence_system();
            }
        }
    }
}

}  // namespace

hipError_t launch_resolve(const Frame& F, const float* pos, const float* rad, const uint32_t* bonds,
                          const BinBuffers& bb, float* depth, uint32_t* id, hipStream_t stream) {
    (void)pos;
    (void)rad;
    (void)bonds;
    const int T = F.tiles_x * F.tiles_y;
    const int grid = xcd_grid(T);
#define VTX_RESOLVE(TS)                                                                                      \
    k_resolve<TS><<<grid, kBlock, 0, stream>>>(F, bb.tile_cnt, bb.tile_off, bb.list, bb.capacity, bb.vis_rec, \
                                               bb.vis_rect, bb.vis_cnt, bb.chunk, bb.groups, bb.ctr,         \
                                               bb.host_ctr, depth, id)
    switch (F.tile) {
        case 8: VTX_RESOLVE(8); break;
        case 16: VTX_RESOLVE(16); break;
        case 32: VTX_RESOLVE(32); break;
        case 64: VTX_RESOLVE(64); break;
        default: return hipErrorInvalidValue;
    }
#undef VTX_RESOLVE
    return hipGetLastError();
}

}  // namespace vtx
