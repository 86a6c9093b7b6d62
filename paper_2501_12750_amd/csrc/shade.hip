// Deferred pass: screen-space ambient occlusion and shading over the G-buffer
// (paper, Methods, "High Quality Rendering": a deferred shading pipeline
// computes lighting on the surfaces and applies screen-space post-processes,
// with ambient occlusion recomputed every frame because dynamic data cannot
// be precomputed).
//
// The G-buffer is the (depth, id) pair the resolve writes.  Each pixel's view
// position is rebuilt from its ray and depth, and its normal and colour from
// the primitive named by id, so no normal or colour buffer is stored.  The
// occlusion test of each hemisphere sample reads the depth at the sample's
// pixel through the cache: the samples of neighbouring pixels land on
// neighbouring pixels, which the cache holds (staging a haloed tile in LDS
// measured slower than the cached reads it saves).
#include "vtx_internal.h"

namespace vtx {

namespace {

constexpr int kTile = 16;
constexpr int kBatch = 16;  // SSAO samples whose depth loads are issued together

constexpr float kKa = 0.2f, kKd = 0.8f, kKs = 0.25f;

// floor(x) as an integer in one instruction (the compiler emits a floor and
// a conversion): saturates at the int range, NaN gives 0.  An SSAO sample
// whose projection is not finite lies behind the near plane, which its own
// test rejects, so the value then does not matter.
__device__ inline int floor_to_int(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ inline float smooth01(float x) {
    x = fminf(fmaxf(x, 0.0f), 1.0f);
    return x * x * (3.0f - 2.0f * x);
}

__device__ inline uint32_t quantize(float c) {
    c = fminf(fmaxf(c, 0.0f), 1.0f);
    return (uint32_t)floorf(fmaf(255.0f, c, 0.5f));
}

// The surface a G-buffer pixel shows: its view position on the pixel's ray,
// the direction towards the eye, the unit normal and the albedo.
struct Surface {
    float Px, Py, Pz;
    float Vx, Vy, Vz;
    float nx, ny, nz;
    uint32_t alb;
    bool hit;
};

__device__ inline Surface surface_at(const Job& J, const Frame& F, int x, int y, uint32_t pid, float z) {
    const global_t<const float>* __restrict__ const pos = to_global(J.pos);
    const global_t<const uint32_t>* __restrict__ const col = to_global(J.col);
    const global_t<const uint32_t>* __restrict__ const bonds = to_global(J.bonds);
    Surface s;
    const float ndx = fmaf((float)x + 0.5f, F.inv_w2, -1.0f);
    const float ndy = fmaf(-((float)y + 0.5f), F.inv_h2, 1.0f);
    if (F.proj == 0) {
        const float Dx = ndx * F.txf, Dy = ndy * F.tyf;
        s.Px = z * Dx;
        s.Py = z * Dy;
        // hardware reciprocal square root: what rsqrtf reduces to for an
        // argument of at least the smallest normal float (here at least 1)
        const float inv = __builtin_amdgcn_rsqf(fmaf(Dx, Dx, fmaf(Dy, Dy, 1.0f)));
        s.Vx = -Dx * inv; s.Vy = -Dy * inv; s.Vz = -inv;
    } else {
        s.Px = ndx * F.hxf;
        s.Py = ndy * F.hyf;
        s.Vx = 0.f; s.Vy = 0.f; s.Vz = -1.f;
    }
    s.Pz = z;
    s.hit = pid < F.n_atoms + F.n_bonds && z < INFINITY;
    float nx = 0.f, ny = 0.f, nz = 0.f;
    s.alb = 0;
    if (s.hit) {
        // The surface point relative to the primitive, in FP64: P = z D on the
        // pixel's ray (D = (ndx tx, ndy ty, 1), or the orthographic origin
        // plus z f), less the primitive's FP64 view coordinates.  Its error is
        // the rounding of the stored depth, u z |D|, so the normal is good to
        // u z |D| / r radians with no loss towards the silhouette.
        const double ndxd = fma((double)x + 0.5, F.inv_w2d, -1.0);
        const double ndyd = fma(-((double)y + 0.5), F.inv_h2d, 1.0);
        const double zd = (double)z;
        const double Qx = F.proj == 0 ? zd * (ndxd * F.tx) : ndxd * F.hx;
        const double Qy = F.proj == 0 ? zd * (ndyd * F.ty) : ndyd * F.hy;
        if (pid < F.n_atoms) {
            double cx, cy, cz;
            to_view(F, pos[3 * (size_t)pid], pos[3 * (size_t)pid + 1], pos[3 * (size_t)pid + 2], cx, cy, cz);
            nx = (float)(Qx - cx);
            ny = (float)(Qy - cy);
            nz = (float)(zd - cz);
            s.alb = col[pid];
        } else {
            const size_t b = pid - F.n_atoms;
            const uint32_t ia = bonds[2 * b], ib = bonds[2 * b + 1];
            if (ia >= F.n_atoms || ib >= F.n_atoms) {
                s.hit = false;
            } else {
                double A[3], B[3];
                to_view(F, pos[3 * (size_t)ia], pos[3 * (size_t)ia + 1], pos[3 * (size_t)ia + 2], A[0], A[1], A[2]);
                to_view(F, pos[3 * (size_t)ib], pos[3 * (size_t)ib + 1], pos[3 * (size_t)ib + 2], B[0], B[1], B[2]);
                double ax = B[0] - A[0], ay = B[1] - A[1], az = B[2] - A[2];
                const double L = sqrt(fma(ax, ax, fma(ay, ay, az * az)));
                const double il = 1.0 / L;
                ax *= il;
                ay *= il;
                az *= il;
                const double rx = Qx - A[0], ry = Qy - A[1], rz = zd - A[2];
                const double sd = fma(rx, ax, fma(ry, ay, rz * az));
                const double qx = fma(-sd, ax, rx), qy = fma(-sd, ay, ry), qz = fma(-sd, az, rz);
                const double ql = sqrt(fma(qx, qx, fma(qy, qy, qz * qz)));
                // the surface the point lies on: the side or the nearer cap
                const double d_side = fabs(ql - (double)F.bond_radius), d_a = fabs(sd), d_b = fabs(sd - L);
                if (d_side <= fmin(d_a, d_b)) {
                    nx = (float)qx; ny = (float)qy; nz = (float)qz;
                    s.alb = sd < 0.5 * L ? col[ia] : col[ib];
                } else if (d_a <= d_b) {
                    nx = (float)-ax; ny = (float)-ay; nz = (float)-az;
                    s.alb = col[ia];
                } else {
                    nx = (float)ax; ny = (float)ay; nz = (float)az;
                    s.alb = col[ib];
                }
            }
        }
        // (as above: a squared surface offset of an atom or bond, far above
        // the smallest normal float)
        const float inv = __builtin_amdgcn_rsqf(fmaf(nx, nx, fmaf(ny, ny, nz * nz)));
        nx *= inv; ny *= inv; nz *= inv;
    }
    s.nx = nx; s.ny = ny; s.nz = nz;
    return s;
}

// Ambient occlusion of a hit surface at pixel (x, y): K hemisphere samples
// in the normal's tangent frame (kTurn: turned about the normal by the
// cosine and sine (rc, rs)), each compared with the depth of the pixel it
// projects to (kPersp: perspective projection, else orthographic).
template <bool kTurn, bool kPersp>
__device__ inline float ssao_at_proj(const Frame& F, const SampleKernel& K, const global_t<const float>* depth, int x, int y,
                                const Surface& s, float rc, float rs) {
    const float nx = s.nx, ny = s.ny, nz = s.nz, Px = s.Px, Py = s.Py, Pz = s.Pz;
    // orthonormal basis from the normal (Duff et al., JCGT 2017, branchless
    // form), turned about the normal: T' = rc T + rs B, B' = rc B - rs T
    const float sg = copysignf(1.0f, nz);
    const float a = -1.0f / (sg + nz);
    const float bb = nx * ny * a;
    const float T0x = 1.0f + sg * nx * nx * a, T0y = sg * bb, T0z = -sg * nx;
    const float B0x = bb, B0y = sg + ny * ny * a, B0z = -ny;
    const float Tx = kTurn ? fmaf(rc, T0x, rs * B0x) : T0x, Ty = kTurn ? fmaf(rc, T0y, rs * B0y) : T0y,
                Tz = kTurn ? fmaf(rc, T0z, rs * B0z) : T0z;
    const float Bx = kTurn ? fmaf(rc, B0x, -rs * T0x) : B0x, By = kTurn ? fmaf(rc, B0y, -rs * T0y) : B0y,
                Bz = kTurn ? fmaf(rc, B0z, -rs * T0z) : B0z;
    const float fpx = F.ssao_fpx, osc = F.ssao_osc;
    float occ = 0.0f;
    // Samples are taken kBatch at a time: every address first, then the
    // loads, then the tests in sample order, so the loads of a batch are
    // in flight together.  Branch-free: an invalid sample (past the count, behind the near
    // plane, off the image) reads the pixel's own depth and is masked out
    // (sz = -inf); entries of h past the count exist (zero).  Byte offsets
    // into the depth image fit 32 bits (at most 4^2 x 7680 x 4320 pixels).
    const float hw = 0.5f * (float)F.W, hh = 0.5f * (float)F.H;
    const uint32_t own = (uint32_t)(y * F.W + x) << 2;
    for (int k0 = 0; k0 < K.count; k0 += kBatch) {
        float zq[kBatch], sz[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int k = k0 + u;
            const float4 h = K.h[k];   // offset in the (T, B, n) frame, scaled
            const float Sx = fmaf(h.x, Tx, fmaf(h.y, Bx, fmaf(h.z, nx, Px)));
            const float Sy = fmaf(h.x, Ty, fmaf(h.y, By, fmaf(h.z, ny, Py)));
            const float Sz = fmaf(h.x, Tz, fmaf(h.y, Bz, fmaf(h.z, nz, Pz)));
            // hardware reciprocal (1 ulp): moves the sample by far less than
            // the 1e-3 px within which a pixel edge makes a sample unstable
            const float sc = kPersp ? fpx * __builtin_amdgcn_rcpf(Sz) : osc;
            const float spx = fmaf(Sx, sc, hw), spy = fmaf(-Sy, sc, hh);
            // on the image: 0 <= spx < W and 0 <= spy < H, tested as the
            // floors' unsigned ranges (the floors are then the pixel's indices)
            const uint32_t ix = (uint32_t)floor_to_int(spx), iy = (uint32_t)floor_to_int(spy);
            // & rather than &&: all tests evaluated, no branches per sample
            const bool ok = (k < K.count) & (Sz > F.znear) & (ix < (uint32_t)F.W) & (iy < (uint32_t)F.H);
            // a 24-bit multiply (full rate): the pixel indices are below 2^16
            // where ok, and the offset is discarded elsewhere
            const uint32_t off = ok ? (__umul24(iy, (uint32_t)F.W) + ix) << 2 : own;
            zq[u] = *reinterpret_cast<const global_t<const float>*>(reinterpret_cast<const global_t<const char>*>(depth) + off);
            sz[u] = ok ? Sz : -INFINITY;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (zq[u] <= sz[u] - K.bias) occ += smooth01(K.radius * __builtin_amdgcn_rcpf(fabsf(Pz - zq[u])));
    }
    return 1.0f - occ / (float)K.count;
}

// The projection is the frame's (one branch per pixel, none per sample).
template <bool kTurn>
__device__ inline float ssao_at(const Frame& F, const SampleKernel& K, const global_t<const float>* depth, int x, int y,
                                const Surface& s, float rc, float rs) {
    return F.proj == 0 ? ssao_at_proj<kTurn, true>(F, K, depth, x, y, s, rc, rs)
                       : ssao_at_proj<kTurn, false>(F, K, depth, x, y, s, rc, rs);
}

// Rank of pixel (x, y) in the 4x4 ordered-dither (Bayer) tile: the index of
// its sample rotation.
__device__ inline int noise_rank(int x, int y) {
    constexpr uint32_t kRows[4] = {0xA280u, 0x6E4Cu, 0x91B3u, 0x5D7Fu};   // 4 bits per column, column 0 lowest
    return (int)((kRows[y & 3] >> (4 * (x & 3))) & 15u);
}

// Work block t of a job is that job's 16x16 tile t.  kNoise: the
// instantiation that can take the noise form (launched when a job asks for
// it; the plain one carries none of its code).
template <class JS, bool kNoise>
__global__ void __launch_bounds__(kBlock) k_shade(JS js) {
    // noise form: the raw AO of the tile and of the 2 pixels left and above
    // and 1 right and below it that the 4x4 blur reads (-1: not a hit)
    constexpr int kHalo = kTile + 3;
    __shared__ float raw[kNoise ? kHalo * kHalo : 1];
    uint32_t tu;
    const int ji = js.find((uint32_t)xcd_contiguous(blockIdx.x, gridDim.x), tu);
    if (ji < 0) return;
    const Job& J = js.job(ji);
    const Frame F = J.F;
    const SampleKernel& K = js.samples(ji);
    const global_t<const float>* __restrict__ const depth = to_global(J.depth);
    const global_t<const uint32_t>* __restrict__ const ids = to_global(J.id);
    global_t<uint32_t>* __restrict__ const rgba = to_global(J.rgba);
    global_t<float>* __restrict__ const normal_out = to_global(J.normal);
    global_t<uint32_t>* __restrict__ const albedo_out = to_global(J.albedo);
    global_t<float>* __restrict__ const ao_out = to_global(J.ao);
    const int tiles_x = (F.W + kTile - 1) / kTile;
    const int t = (int)tu;
    const int tid = threadIdx.x;
    const int tx0 = (t % tiles_x) * kTile, ty0 = (t / tiles_x) * kTile;
    const int x = tx0 + (tid & (kTile - 1)), y = ty0 + (tid >> 4);
    const bool noise = kNoise && K.noise && K.count > 0;   // the same for the whole workgroup (one job)
    if (noise) {
        for (int i = tid; i < kHalo * kHalo; i += kBlock) {
            const int qx = tx0 - 2 + i % kHalo, qy = ty0 - 2 + i / kHalo;
            float v = -1.0f;
            if (qx >= 0 && qx < F.W && qy >= 0 && qy < F.H) {
                const size_t q = (size_t)qy * F.W + qx;
                const Surface sq = surface_at(J, F, qx, qy, ids[q], depth[q]);
                if (sq.hit) {
                    const float2 r = K.rot[noise_rank(qx, qy)];
                    v = ssao_at<true>(F, K, depth, qx, qy, sq, r.x, r.y);
                }
            }
            raw[i] = v;
        }
        __syncthreads();
    }
    if (x >= F.W || y >= F.H) return;
    const size_t p = (size_t)y * F.W + x;
    const float z = depth[p];
    const Surface sf = surface_at(J, F, x, y, ids[p], z);
    const bool hit = sf.hit;
    const float nx = sf.nx, ny = sf.ny, nz = sf.nz, Vx = sf.Vx, Vy = sf.Vy, Vz = sf.Vz;
    const uint32_t alb = sf.alb;

    float ao = 1.0f;
    if (hit && noise) {
        // the mean of the raw AO over the hit pixels of the 4x4 block at
        // offsets -2..1 (the halo holds the ones outside the tile)
        const int lx = x - tx0 + 2, ly = y - ty0 + 2;
        float sum = 0.0f;
        int cnt = 0;
#pragma unroll
        for (int dy = -2; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -2; dx <= 1; ++dx) {
                const float v = raw[(ly + dy) * kHalo + (lx + dx)];
                if (v >= 0.0f) {
                    sum += v;
                    ++cnt;
                }
            }
        ao = sum / (float)cnt;
    } else if (hit && K.count > 0) {
        ao = ssao_at<false>(F, K, depth, x, y, sf, 1.0f, 0.0f);
    }

    uint32_t out = K.background;
    if (hit) {
        const float nv = fmaxf(0.0f, fmaf(nx, Vx, fmaf(ny, Vy, nz * Vz)));
        // shading mode: a diffuse factor on the albedo and a white specular term
        float diff, spec = 0.0f;
        if (F.shading == 2) {                                  // flat
            diff = ao;
        } else if (F.shading == 3) {                           // toon: four bands of n.V
            diff = fmaf(kKd, fminf(floorf(4.0f * nv), 3.0f) * (1.0f / 3.0f), kKa) * ao;
        } else {                                               // glossy, matte
            diff = fmaf(kKd, nv, kKa) * ao;
            if (F.shading == 0) {
                float sp = fmaxf(0.0f, fmaf(2.0f * nv, nv, -1.0f));
                sp *= sp; sp *= sp; sp *= sp; sp *= sp; sp *= sp;     // ^32
                spec = kKs * sp;
            }
        }
        float c[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) c[ch] = fmaf((float)((alb >> (8 * ch)) & 255u) * (1.0f / 255.0f), diff, spec);
        if (F.fog_inv > 0.0f) {
            const float f = fminf(fmaxf((z - F.fog_start) * F.fog_inv, 0.0f), 1.0f);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) c[ch] = fmaf(f, F.fog_rgb[ch] - c[ch], c[ch]);
        }
        out = quantize(c[0]) | (quantize(c[1]) << 8) | (quantize(c[2]) << 16) | (255u << 24);
        if (F.outline_t > 0.0f) {
            // a neighbour in the image that is background or deeper by the step
            const float zt = z * (1.0f + F.outline_t);
            bool edge = false;
            if (x + 1 < F.W) edge = edge || depth[p + 1] > zt;
            if (x > 0) edge = edge || depth[p - 1] > zt;
            if (y + 1 < F.H) edge = edge || depth[p + (size_t)F.W] > zt;
            if (y > 0) edge = edge || depth[p - (size_t)F.W] > zt;
            if (edge) out = F.outline_rgba;
        }
    }
    rgba[p] = out;
    if (normal_out) {
        normal_out[3 * p] = nx;
        normal_out[3 * p + 1] = ny;
        normal_out[3 * p + 2] = nz;
    }
    if (albedo_out) albedo_out[p] = hit ? alb : 0u;
    if (ao_out) ao_out[p] = ao;
}

// One output pixel per thread: its S x S samples are reduced to the rounded
// mean of each RGBA channel and the nearest (depth, id).
__global__ void __launch_bounds__(kBlock) k_downsample(const float* __restrict__ sdepth,
                                                       const uint32_t* __restrict__ sid,
                                                       const uint32_t* __restrict__ srgba, int W, int H, int S,
                                                       float* __restrict__ depth, uint32_t* __restrict__ id,
                                                       uint32_t* __restrict__ rgba) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (size_t)W * H) return;
    const int x = (int)(p % (size_t)W), y = (int)(p / (size_t)W);
    const size_t SW = (size_t)W * S;
    unsigned long long best = ~0ull;
    uint32_t sum[4] = {0u, 0u, 0u, 0u};
    for (int sy = 0; sy < S; ++sy)
        for (int sx = 0; sx < S; ++sx) {
            const size_t q = ((size_t)y * S + sy) * SW + (size_t)x * S + sx;
            const unsigned long long key = ((unsigned long long)__float_as_uint(sdepth[q]) << 32) | sid[q];
            best = key < best ? key : best;
            const uint32_t c = srgba[q];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) sum[ch] += (c >> (8 * ch)) & 255u;
        }
    const uint32_t n = (uint32_t)(S * S);
    uint32_t out = 0;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) out |= ((sum[ch] + n / 2) / n) << (8 * ch);
    rgba[p] = out;
    depth[p] = __uint_as_float((uint32_t)(best >> 32));
    id[p] = (uint32_t)(best & 0xFFFFFFFFull);
}

}  // namespace

hipError_t launch_downsample(const float* sdepth, const uint32_t* sid, const uint32_t* srgba, int W, int H, int S,
                             float* depth, uint32_t* id, uint32_t* rgba, hipStream_t stream) {
    const size_t px = (size_t)W * H;
    if (px == 0) return hipSuccess;
    return dispatch(k_downsample, (unsigned)((px + kBlock - 1) / kBlock), kBlock, 0, stream, sdepth, sid, srgba, W, H, S,
                    depth, id, rgba);
}

template <class JS>
hipError_t shade_impl(const JS& js, uint32_t grid, bool noise, hipStream_t stream) {
    if (grid == 0) return hipSuccess;
    if (noise) return dispatch(k_shade<JS, true>, (unsigned)xcd_grid((int)grid), kBlock, 0, stream, js);
    return dispatch(k_shade<JS, false>, (unsigned)xcd_grid((int)grid), kBlock, 0, stream, js);
}

hipError_t launch_shade(const OneJob& js, uint32_t grid, bool noise, hipStream_t stream) {
    return shade_impl(js, grid, noise, stream);
}
hipError_t launch_shade(const JobList& js, uint32_t grid, bool noise, hipStream_t stream) {
    return shade_impl(js, grid, noise, stream);
}

}  // namespace vtx
