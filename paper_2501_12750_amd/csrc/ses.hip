// Solvent excluded surface on a grid, extracted by marching cubes (paper,
// Methods, "Cartoon and SES representations": a discrete SES, as in Lindow
// et al., extracted with marching cubes).
//
// Readings (the paper gives no formulas):
//  - grid point (i, j, k) is at o + h (i, j, k) in FP64; it lies inside the
//    solvent-accessible region when some atom has |p - c|^2 < (r + rp)^2,
//    each square and sum rounded once in FP64; the others are positions a
//    probe centre can take ("exterior");
//  - f(p) = min(h sqrt(g), W h) - rp, g the least squared grid distance from
//    p to an exterior point, W = ceil(rp / h) + 2 (beyond W h only the sign
//    matters), rounded to FP32; the SES encloses f >= 0;
//  - marching cubes over f >= 0 with a case table built from the cube's
//    faces: each face with two crossing edges gives a segment, a face whose
//    inside corners are diagonal gives two segments cutting off the inside
//    corners; segments close into loops, oriented from the inside corners to
//    the outside ones and started at their lowest edge; a 3-edge loop is a
//    triangle, a longer one a fan around the mean of its vertices.
//
// Passes: mark the SAS interior per atom; the exact squared distance to
// the nearest exterior point within a W-box by three separable 1-D passes
// in integers (x: nearest exterior point on the row; y and z: the least of
// g + d^2 over the window); triangle counts per cube; an exclusive scan of
// the counts (scan.hip); emission of the triangles of the cubes that have
// any, each at its offset.
#include <mutex>

#include "vtx_internal.h"

namespace vtx {

namespace {

constexpr int kSesBlock = 256;
constexpr int kSesMarkBlock = 64;      // one wave per atom: its box setup is paid once per wave
constexpr int32_t kFar = 0x3FFFFFFF;   // no exterior point within the window

// Case table: for each case, its loops as a byte string: loop length, then
// its edges, ..., then 0.  Edges 0-3 run along x, 4-7 along y, 8-11 along z
// (corner pairs below); corner c sits at (c & 1, c >> 1 & 1, c >> 2 & 1).
constexpr int kCaseBytes = 24;
__constant__ uint8_t c_cases[256 * kCaseBytes];
__constant__ uint8_t c_case_tris[256];

constexpr int kEdgeA[12] = {0, 2, 4, 6, 0, 1, 4, 5, 0, 1, 2, 3};
constexpr int kEdgeB[12] = {1, 3, 5, 7, 2, 3, 6, 7, 4, 5, 6, 7};
__constant__ int8_t c_edge_corner[12][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3},
                                            {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

int edge_of(int a, int b) {
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    for (int e = 0; e < 12; ++e)
        if (kEdgeA[e] == a && kEdgeB[e] == b) return e;
    return -1;
}

// The loops of case m, built as the table's rule states.
void build_case(int m, uint8_t* out, uint8_t* ntri) {
    static const int faces[6][4] = {{0, 2, 6, 4}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 3, 7, 6}, {0, 1, 3, 2}, {4, 5, 7, 6}};
    int in[8];
    for (int c = 0; c < 8; ++c) in[c] = (m >> c) & 1;
    int nb[12][2], deg[12] = {};
    auto link = [&](int a, int b) {
        nb[a][deg[a]++] = b;
        nb[b][deg[b]++] = a;
    };
    for (const auto& f : faces) {
        int e[4], s[4], nc = 0, cr[4];
        for (int i = 0; i < 4; ++i) {
            s[i] = in[f[i]];
            e[i] = edge_of(f[i], f[(i + 1) & 3]);
        }
        for (int i = 0; i < 4; ++i)
            if (s[i] != s[(i + 1) & 3]) cr[nc++] = i;
        if (nc == 2) {
            link(e[cr[0]], e[cr[1]]);
        } else if (nc == 4) {
            for (int i = 0; i < 4; ++i)
                if (s[i]) link(e[(i + 3) & 3], e[i]);
        }
    }
    bool used[12] = {};
    int pos = 0, tris = 0;
    for (int start = 0; start < 12; ++start) {
        if (deg[start] == 0 || used[start]) continue;
        int loop[12], k = 0;
        loop[k++] = start;
        used[start] = true;
        int prev = start, cur = nb[start][0];
        while (cur != start) {
            loop[k++] = cur;
            used[cur] = true;
            const int nxt = nb[cur][0] == prev ? nb[cur][1] : nb[cur][0];
            prev = cur;
            cur = nxt;
        }
        // orientation: the loop's normal over its edge midpoints against the
        // sum of the inside -> outside directions of its edges
        double mid[12][3], nrm[3] = {0, 0, 0}, dir[3] = {0, 0, 0};
        for (int i = 0; i < k; ++i) {
            const int a = kEdgeA[loop[i]], b = kEdgeB[loop[i]];
            for (int d = 0; d < 3; ++d) {
                const double pa = (a >> d) & 1, pb = (b >> d) & 1;
                mid[i][d] = 0.5 * (pa + pb);
                dir[d] += in[a] ? pb - pa : pa - pb;
            }
        }
        for (int i = 0; i < k; ++i) {
            const double* p = mid[i];
            const double* q = mid[(i + 1) % k];
            nrm[0] += p[1] * q[2] - p[2] * q[1];
            nrm[1] += p[2] * q[0] - p[0] * q[2];
            nrm[2] += p[0] * q[1] - p[1] * q[0];
        }
        if (nrm[0] * dir[0] + nrm[1] * dir[1] + nrm[2] * dir[2] < 0.0)
            for (int i = 0; i < k / 2; ++i) {
                const int t = loop[i];
                loop[i] = loop[k - 1 - i];
                loop[k - 1 - i] = t;
            }
        int lo = 0;
        for (int i = 1; i < k; ++i)
            if (loop[i] < loop[lo]) lo = i;
        out[pos++] = (uint8_t)k;
        for (int i = 0; i < k; ++i) out[pos++] = (uint8_t)loop[(lo + i) % k];
        tris += k == 3 ? 1 : k;
    }
    out[pos] = 0;
    *ntri = (uint8_t)tris;
}

std::mutex g_case_mu;
bool g_case_ready[64] = {};

hipError_t ensure_cases(int device) {
    std::lock_guard<std::mutex> lk(g_case_mu);
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    if (g_case_ready[device]) return hipSuccess;
    static uint8_t cases[256 * kCaseBytes];
    static uint8_t ntri[256];
    for (int m = 0; m < 256; ++m) build_case(m, cases + m * kCaseBytes, ntri + m);
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_cases), cases, sizeof(cases));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_case_tris), ntri, sizeof(ntri));
    if (e == hipSuccess) g_case_ready[device] = true;
    return e;
}

struct SesGrid {
    double o[3];
    double h;
    double inv_h;       // 1 / h (bounding boxes only)
    int nx, ny, nz;
    int W;              // distance window in grid steps
    double rp;
};

__device__ inline size_t gidx(const SesGrid& G, int i, int j, int k) {
    return (size_t)i + (size_t)G.nx * ((size_t)j + (size_t)G.ny * k);
}

// One wave per atom: marks the grid points inside its solvent-accessible
// sphere (interior = 1; points no atom marks stay 0: exterior).  Each lane
// takes (i, j) columns of the atom's box and walks them along k with
// dx^2 + dy^2 computed once per column.
__global__ void __launch_bounds__(kSesMarkBlock) k_ses_mark(const float* __restrict__ pos,
                                                            const float* __restrict__ rad, uint32_t n, SesGrid G,
                                                            uint8_t* __restrict__ mark) {
#pragma clang fp contract(off)
    const uint32_t a = blockIdx.x;
    if (a >= n) return;
    const double cx = pos[3 * (size_t)a], cy = pos[3 * (size_t)a + 1], cz = pos[3 * (size_t)a + 2];
    const double R = (double)rad[a] + G.rp;
    if (!(R > 0.0)) return;
    const double R2 = R * R;
    int lo[3], hi[3];
    const double c[3] = {cx, cy, cz};
    const int nmax[3] = {G.nx - 1, G.ny - 1, G.nz - 1};
    // the box only has to hold every point the test can mark: a step of
    // margin on each side covers the rounding of the product by 1 / h
    for (int d = 0; d < 3; ++d) {
        lo[d] = max(0, (int)floor((c[d] - R - G.o[d]) * G.inv_h) - 1);
        hi[d] = min(nmax[d], (int)ceil((c[d] + R - G.o[d]) * G.inv_h) + 1);
        if (lo[d] > hi[d]) return;
    }
    const int bx = hi[0] - lo[0] + 1, ncol = bx * (hi[1] - lo[1] + 1);
    const size_t plane = (size_t)G.nx * G.ny;
    for (int q = threadIdx.x; q < ncol; q += kSesMarkBlock) {
        const int j = lo[1] + q / bx, i = lo[0] + q % bx;
        const double dx = (G.o[0] + G.h * i) - cx, dy = (G.o[1] + G.h * j) - cy;
        const double sxy = dx * dx + dy * dy;
        size_t p = gidx(G, i, j, lo[2]);
        for (int k = lo[2]; k <= hi[2]; ++k, p += plane) {
            const double dz = (G.o[2] + G.h * k) - cz;
            if (sxy + dz * dz < R2) mark[p] = 1;
        }
    }
}

// The per-point and per-cube passes run one thread per point (or cube) in
// x-fastest order; the grid holds fewer than 2^31 points, so the index and
// its decomposition stay in 32 bits.
__device__ inline bool flat_item(uint32_t n, int nx, int ny, int& i, int& j, int& k, uint32_t& p) {
    p = blockIdx.x * (uint32_t)kSesBlock + threadIdx.x;
    if (p >= n) return false;
    const uint32_t r = p / (uint32_t)nx;
    i = (int)(p - r * (uint32_t)nx);
    j = (int)(r % (uint32_t)ny);
    k = (int)(r / (uint32_t)ny);
    return true;
}

// x pass: squared distance along the row to the nearest exterior point
// within W steps (kFar if none).
__global__ void __launch_bounds__(kSesBlock) k_ses_edt_x(SesGrid G, uint32_t np, const uint8_t* __restrict__ mark,
                                                         int32_t* __restrict__ g) {
    int i, j, k;
    uint32_t p;
    if (!flat_item(np, G.nx, G.ny, i, j, k, p)) return;
    int32_t best = kFar;
    for (int d = 0; d <= G.W; ++d) {
        const bool l = i - d >= 0 && !mark[p - d];
        const bool r = i + d < G.nx && !mark[p + d];
        if (l || r) {
            best = d * d;
            break;
        }
    }
    g[p] = best;
}

// The x pass through LDS (W <= kEdtMaxW): work block b takes kSesBlock
// consecutive points of one row (x block b mod nxb of row b / nxb) and
// stages their marks and W more on each side.
template <int kMaxW>
__global__ void __launch_bounds__(kSesBlock) k_ses_edt_x_lds(SesGrid G, uint32_t nxb,
                                                             const uint8_t* __restrict__ mark,
                                                             int32_t* __restrict__ g) {
    __shared__ uint8_t row[kSesBlock + 2 * kMaxW];
    const uint32_t r = blockIdx.x / nxb, xb = blockIdx.x - r * nxb;
    const int W = G.W, x0 = (int)xb * kSesBlock;
    const size_t base = (size_t)r * G.nx;   // row r = j + ny k starts at r nx
    for (int t = threadIdx.x; t < kSesBlock + 2 * W; t += kSesBlock) {
        const int x = x0 - W + t;
        row[t] = (x >= 0 && x < G.nx) ? mark[base + x] : (uint8_t)2;   // 2: outside the grid
    }
    __syncthreads();
    const int i = x0 + (int)threadIdx.x;
    if (i >= G.nx) return;
    int32_t best = kFar;
    for (int d = 0; d <= W; ++d) {
        const uint8_t l = row[threadIdx.x + W - d], rr = row[threadIdx.x + W + d];
        if (l == 0 || rr == 0) {
            best = d * d;
            break;
        }
    }
    g[base + i] = best;
}

// y or z pass: the least of g(p + d e) + d^2 over |d| <= W along the axis.
// The z pass also writes the field.
template <bool kLast>
__global__ void __launch_bounds__(kSesBlock) k_ses_edt_yz(SesGrid G, uint32_t np, const int32_t* __restrict__ gin,
                                                          int32_t* __restrict__ gout, float* __restrict__ field) {
    int i, j, k;
    uint32_t p;
    if (!flat_item(np, G.nx, G.ny, i, j, k, p)) return;
    const int stride = kLast ? G.nx * G.ny : G.nx;
    const int len = kLast ? G.nz : G.ny;
    const int at = kLast ? k : j;
    int32_t best = kFar;
    for (int d = -G.W; d <= G.W; ++d) {
        const int q = at + d;
        if (q < 0 || q >= len) continue;
        const int32_t v = gin[(int)p + d * stride];
        if (v < kFar) best = min(best, v + d * d);
    }
    if (!kLast) {
        gout[p] = best;
        return;
    }
    const double cap = G.W * G.h;
    const double D = best > G.W * G.W ? cap : fmin(G.h * sqrt((double)best), cap);
    field[p] = (float)(D - G.rp);
}

// The same passes through LDS (windows of W <= kEdtMaxW): work block b
// takes kEdtX consecutive x of one slice (z for the y pass, y for the z pass)
// and kEdtRows consecutive positions along the axis, stages those rows and
// W more on each side in LDS (one load per staged value), and each thread
// then takes the window minima of its column from LDS.
constexpr int kEdtX = 64, kEdtRows = 32, kEdtMaxW = 32;

template <bool kLast>
__global__ void __launch_bounds__(kSesBlock) k_ses_edt_yz_lds(SesGrid G, uint32_t nxb, uint32_t nrb,
                                                              const int32_t* __restrict__ gin,
                                                              int32_t* __restrict__ gout, float* __restrict__ field) {
    __shared__ int32_t tile[(kEdtRows + 2 * kEdtMaxW) * kEdtX];
    const uint32_t b = blockIdx.x, xb = b % nxb, rest = b / nxb, rb = rest % nrb, sl = rest / nrb;
    const int tx = threadIdx.x % kEdtX, ty = threadIdx.x / kEdtX;
    constexpr int kLanes = kSesBlock / kEdtX;
    const int x = (int)xb * kEdtX + tx, a0 = (int)rb * kEdtRows, W = G.W;
    const int len = kLast ? G.nz : G.ny;
    // element (x, axis position a) of this slice
    auto at = [&](int a) -> size_t {
        return kLast ? gidx(G, x, (int)sl, a) : gidx(G, x, a, (int)sl);
    };
    const int staged = kEdtRows + 2 * W;
    for (int r = ty; r < staged; r += kLanes) {
        const int a = a0 - W + r;
        tile[r * kEdtX + tx] = (x < G.nx && a >= 0 && a < len) ? gin[at(a)] : kFar;
    }
    __syncthreads();
    if (x >= G.nx) return;
    for (int o = ty; o < kEdtRows; o += kLanes) {
        const int a = a0 + o;
        if (a >= len) break;
        int32_t best = kFar;
        for (int d = -W; d <= W; ++d) {
            const int32_t v = tile[(o + W + d) * kEdtX + tx];
            if (v < kFar) best = min(best, v + d * d);
        }
        const size_t p = at(a);
        if (!kLast) {
            gout[p] = best;
        } else {
            const double cap = G.W * G.h;
            const double D = best > G.W * G.W ? cap : fmin(G.h * sqrt((double)best), cap);
            field[p] = (float)(D - G.rp);
        }
    }
}

__device__ inline int cube_case(const SesGrid& G, const float* __restrict__ f, int i, int j, int k, float v[8]) {
    int m = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        v[c] = f[gidx(G, i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1))];
        m |= (v[c] >= 0.0f ? 1 : 0) << c;
    }
    return m;
}

// Triangles per cube, and per workgroup of kSesBlock cubes the list of its
// cubes that have any: active[b * kSesBlock + s] for s < n_active[b].
__global__ void __launch_bounds__(kSesBlock) k_ses_count(SesGrid G, uint32_t nc, const float* __restrict__ f,
                                                         uint32_t* __restrict__ cnt, uint32_t* __restrict__ active,
                                                         uint32_t* __restrict__ n_active) {
    __shared__ uint32_t wave_n[kSesBlock / 64];
    int i, j, k;
    uint32_t q;
    uint32_t nt = 0;
    if (flat_item(nc, G.nx - 1, G.ny - 1, i, j, k, q)) {
        float v[8];
        nt = c_case_tris[cube_case(G, f, i, j, k, v)];
        cnt[q] = nt;
    }
    const unsigned long long act = __ballot(nt != 0);
    const int wave = threadIdx.x >> 6;
    if (__lane_id() == 0) wave_n[wave] = (uint32_t)__popcll(act);
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kSesBlock / 64; ++w) {
        before += w < wave ? wave_n[w] : 0u;
        all += wave_n[w];
    }
    if (nt) active[(size_t)blockIdx.x * kSesBlock + before + (uint32_t)__popcll(act & __lanemask_lt())] = q;
    if (threadIdx.x == 0) n_active[blockIdx.x] = all;
}

// The triangles of each cube its count workgroup listed, at the cube's
// offset (those past the capacity are dropped).
__global__ void __launch_bounds__(kSesBlock) k_ses_emit(SesGrid G, const uint32_t* __restrict__ active,
                                                        const uint32_t* __restrict__ n_active,
                                                        const float* __restrict__ f, const uint32_t* __restrict__ off,
                                                        float* __restrict__ tri, unsigned long long capacity) {
    if (threadIdx.x >= n_active[blockIdx.x]) return;
    const uint32_t q = active[(size_t)blockIdx.x * kSesBlock + threadIdx.x];
    const uint32_t r = q / (uint32_t)(G.nx - 1);
    const int i = (int)(q - r * (uint32_t)(G.nx - 1)), j = (int)(r % (uint32_t)(G.ny - 1)),
              k = (int)(r / (uint32_t)(G.ny - 1));
    float v[8];
    const int m = cube_case(G, f, i, j, k, v);
    unsigned long long t = off[q];
    const float ox = (float)G.o[0], oy = (float)G.o[1], oz = (float)G.o[2], h = (float)G.h;
    const uint8_t* cs = c_cases + m * kCaseBytes;
    for (int at = 0; cs[at] != 0;) {
        const int len = cs[at];
        float px[8], py[8], pz[8];
        float sx = 0.f, sy = 0.f, sz = 0.f;
        for (int e = 0; e < len; ++e) {
            const int ed = cs[at + 1 + e];
            const int a = c_edge_corner[ed][0], b = c_edge_corner[ed][1];
            const float tt = v[a] / (v[a] - v[b]);
            const float fx = (float)((a & 1) + tt * ((b & 1) - (a & 1)));
            const float fy = (float)(((a >> 1) & 1) + tt * (((b >> 1) & 1) - ((a >> 1) & 1)));
            const float fz = (float)(((a >> 2) & 1) + tt * (((b >> 2) & 1) - ((a >> 2) & 1)));
            px[e] = ox + h * ((float)i + fx);
            py[e] = oy + h * ((float)j + fy);
            pz[e] = oz + h * ((float)k + fz);
            sx += px[e];
            sy += py[e];
            sz += pz[e];
        }
        auto put = [&](float ax, float ay, float az, int b, int c) {
            if (t < capacity) {
                float* o = tri + 9 * t;
                o[0] = ax; o[1] = ay; o[2] = az;
                o[3] = px[b]; o[4] = py[b]; o[5] = pz[b];
                o[6] = px[c]; o[7] = py[c]; o[8] = pz[c];
            }
            ++t;
        };
        if (len == 3) {
            put(px[0], py[0], pz[0], 1, 2);
        } else {
            const float inv = 1.0f / (float)len;
            for (int e = 0; e < len; ++e) put(sx * inv, sy * inv, sz * inv, e, (e + 1) % len);
        }
        at += 1 + len;
    }
}
}  // namespace

hipError_t ses_run(const float* pos, const float* rad, uint64_t n, float probe, const float origin[3], float spacing,
                   const int dims[3], float* field, float* tri, uint64_t capacity, unsigned long long* n_tri,
                   SesScratch& s, hipStream_t stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((e = ensure_cases(dev)) != hipSuccess) return e;
    SesGrid G;
    for (int d = 0; d < 3; ++d) G.o[d] = (double)origin[d];
    G.h = (double)spacing;
    G.inv_h = 1.0 / G.h;
    G.nx = dims[0];
    G.ny = dims[1];
    G.nz = dims[2];
    G.rp = (double)probe;
    G.W = (int)ceil(G.rp / G.h) + 2;
    const size_t np = (size_t)G.nx * G.ny * G.nz;
    const size_t nc = (size_t)(G.nx - 1) * (G.ny - 1) * (G.nz - 1);
    if ((e = launch_zero(reinterpret_cast<uint32_t*>(s.mark), (np + 3) / 4, stream)) != hipSuccess) return e;
    if (n && (e = dispatch(k_ses_mark, (unsigned)n, kSesMarkBlock, 0, stream, pos, rad, (uint32_t)n, G, s.mark)))
        return e;
    // rows of points along x (y-z rows), then rows of cubes
    const unsigned gp = (unsigned)((np + kSesBlock - 1) / kSesBlock);
    const uint64_t nxr = (uint64_t)(G.nx + kSesBlock - 1) / kSesBlock, gx = nxr * (uint64_t)G.ny * (uint64_t)G.nz;
    if (G.W <= kEdtMaxW && gx * kSesBlock < (1ull << 31)) {
        if ((e = dispatch(k_ses_edt_x_lds<kEdtMaxW>, (uint32_t)gx, kSesBlock, 0, stream, G, (uint32_t)nxr,
                          (const uint8_t*)s.mark, s.ga)))
            return e;
    } else if ((e = dispatch(k_ses_edt_x, gp, kSesBlock, 0, stream, G, (uint32_t)np, (const uint8_t*)s.mark, s.ga))) {
        return e;
    }
    const uint64_t nxb = (uint64_t)(G.nx + kEdtX - 1) / kEdtX;
    const uint64_t gy = nxb * (uint64_t)((G.ny + kEdtRows - 1) / kEdtRows) * (uint64_t)G.nz;
    const uint64_t gz = nxb * (uint64_t)((G.nz + kEdtRows - 1) / kEdtRows) * (uint64_t)G.ny;
    if (G.W <= kEdtMaxW && gy * kSesBlock < (1ull << 31) && gz * kSesBlock < (1ull << 31)) {
        if ((e = dispatch(k_ses_edt_yz_lds<false>, (uint32_t)gy, kSesBlock, 0, stream, G, (uint32_t)nxb,
                          (uint32_t)((G.ny + kEdtRows - 1) / kEdtRows), (const int32_t*)s.ga, s.gb, (float*)nullptr)))
            return e;
        if ((e = dispatch(k_ses_edt_yz_lds<true>, (uint32_t)gz, kSesBlock, 0, stream, G, (uint32_t)nxb,
                          (uint32_t)((G.nz + kEdtRows - 1) / kEdtRows), (const int32_t*)s.gb, s.ga, field)))
            return e;
    } else {
        if ((e = dispatch(k_ses_edt_yz<false>, gp, kSesBlock, 0, stream, G, (uint32_t)np, (const int32_t*)s.ga, s.gb,
                          (float*)nullptr)))
            return e;
        if ((e = dispatch(k_ses_edt_yz<true>, gp, kSesBlock, 0, stream, G, (uint32_t)np, (const int32_t*)s.gb, s.ga,
                          field)))
            return e;
    }
    // the distance buffers are free once the z pass has run: the y pass's
    // holds the per-workgroup lists of cubes with triangles, the other one
    // their lengths
    uint32_t* const active = reinterpret_cast<uint32_t*>(s.gb);
    uint32_t* const n_active = reinterpret_cast<uint32_t*>(s.ga);
    const unsigned gc = (unsigned)((nc + kSesBlock - 1) / kSesBlock);
    if ((e = dispatch(k_ses_count, gc, kSesBlock, 0, stream, G, (uint32_t)nc, (const float*)field, s.cnt, active,
                      n_active)))
        return e;
    if ((e = exclusive_scan(s.cnt, nc, s.bsum, n_tri, stream))) return e;
    return dispatch(k_ses_emit, gc, kSesBlock, 0, stream, G, (const uint32_t*)active, (const uint32_t*)n_active,
                    (const float*)field, (const uint32_t*)s.cnt, tri, (unsigned long long)capacity);
}

size_t ses_scratch_words(const int dims[3], size_t* mark_words, size_t* g_words, size_t* cnt_words, size_t* bsum_words) {
    const size_t np = (size_t)dims[0] * dims[1] * dims[2];
    const size_t nc = (size_t)(dims[0] - 1) * (dims[1] - 1) * (dims[2] - 1);
    *mark_words = (np + 3) / 4;
    *g_words = np;
    *cnt_words = nc;
    *bsum_words = scan_scratch_words(nc);
    return *mark_words + 2 * *g_words + *cnt_words + *bsum_words;
}

}  // namespace vtx
