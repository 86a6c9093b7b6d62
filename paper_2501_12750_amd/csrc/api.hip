// C ABI of the renderer (declared in include/vtx.h): argument checks, frame
// constants, per-stream scratch (tile bins) and the launch sequence
// bin -> resolve -> shade.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "vtx.h"
#include "vtx_internal.h"

namespace {

using vtx::BinBuffers;
using vtx::Counters;
using vtx::Frame;

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

#define VTX_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return fail(VTX_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int kTimingRing = 64;
constexpr int kMarks = 7;   // before clear, project, scan, scatter, resolve, shade; after shade

struct TimingSlot {
    hipEvent_t ev[kMarks] = {};
    bool inflight = false;
};

// Scratch of one (device, stream): tile bins, the compacted visible list and
// the frame counters, plus a pinned copy of the counters that the host reads
// once the frame's event has completed.
struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    BinBuffers bb{};
    size_t tiles_cap = 0;
    size_t vis_cap = 0;
    size_t groups_cap = 0;
    size_t hist_cap = 0;
    size_t list_alloc = 0;          // allocated bin entries (>= bb.capacity, the entries in use)
    Counters* host_ctr = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
    bool have_stats = false;
    uint64_t pending_capacity = 0;
    uint64_t want_capacity = 0;
    bool fixed_capacity = false;
    bool dirty = true;              // tile counts / counters must be zeroed before the next frame
    uint64_t sized_nprim = ~0ull;   // scene and image size the bins were last sized for
    int sized_w = -1, sized_h = -1;
    vtx_stats last{};
    TimingSlot* tslots = nullptr;   // ring of kTimingRing, created on first timed frame
    int tnext = 0;
    uint64_t tframes = 0;
    double tsum[kMarks - 1] = {};
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

constexpr uint64_t kMaxCapacity = 1ull << 28;        // bin entries (8 GiB of 32-byte records)
constexpr uint64_t kMinCapacity = 1ull << 20;

int free_ws_buffers(Workspace* ws) {
    hipFree(ws->bb.tile_cnt);
    hipFree(ws->bb.tile_off);
    hipFree(ws->bb.tile_fill);
    hipFree(ws->bb.vis_rec);
    hipFree(ws->bb.vis_rect);
    hipFree(ws->bb.vis_cnt);
    hipFree(ws->bb.vis_box);
    hipFree(ws->bb.hist);
    ws->bb.vis_box = nullptr;
    hipFree(ws->bb.list);
    ws->bb.vis_cnt = nullptr;
    ws->bb.hist = nullptr;
    ws->groups_cap = 0;
    ws->hist_cap = 0;
    ws->bb.tile_cnt = nullptr;
    ws->bb.tile_off = nullptr;
    ws->bb.tile_fill = nullptr;
    ws->bb.vis_rec = nullptr;
    ws->bb.vis_rect = nullptr;
    ws->bb.list = nullptr;
    ws->bb.capacity = 0;
    ws->tiles_cap = 0;
    ws->vis_cap = 0;
    ws->list_alloc = 0;
    return VTX_OK;
}

// Reads the counters of a completed frame into ws->last.
void harvest(Workspace* ws) {
    if (!ws->pending) return;
    if (hipEventQuery(ws->done) != hipSuccess) return;
    const Counters& c = *ws->host_ctr;
    ws->last.visible = c.vis_count;
    ws->last.pairs = c.pairs;
    ws->last.fragments_tested = c.frag_tested;
    ws->last.fragments_hit = c.frag_hit;
    ws->last.fragments_hit_bond = c.frag_hit_bond;
    ws->last.overflow_tiles = c.overflow_tiles;
    ws->last.bin_capacity = ws->pending_capacity;
    ws->last.bad_bonds = c.bad_bonds;
    ws->have_stats = true;
    ws->pending = false;
    if (c.pairs > ws->bb.capacity && !ws->fixed_capacity) {
        uint64_t want = c.pairs + c.pairs / 2 + 1024;
        if (want > kMaxCapacity) want = kMaxCapacity;
        if (want > ws->want_capacity) ws->want_capacity = want;
    }
}

void harvest_timings(Workspace* ws, bool wait) {
    if (!ws->tslots) return;
    for (int k = 0; k < kTimingRing; ++k) {
        const int i = (ws->tnext + k) % kTimingRing;   // oldest first
        TimingSlot& t = ws->tslots[i];
        if (!t.inflight) continue;
        if (wait) (void)hipEventSynchronize(t.ev[kMarks - 1]);
        if (hipEventQuery(t.ev[kMarks - 1]) != hipSuccess) break;
        for (int m = 0; m < kMarks - 1; ++m) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, t.ev[m], t.ev[m + 1]) == hipSuccess) ws->tsum[m] += ms;
        }
        ws->tframes += 1;
        t.inflight = false;
    }
}

// Next free slot of the timing ring (waits for the oldest if all are in flight).
int timing_slot(Workspace* ws, TimingSlot** out) {
    if (!ws->tslots) {
        ws->tslots = new TimingSlot[kTimingRing];
        for (int i = 0; i < kTimingRing; ++i)
            for (int m = 0; m < kMarks; ++m)
                if (hipEventCreate(&ws->tslots[i].ev[m]) != hipSuccess) return fail(VTX_EHIP, "hipEventCreate failed");
    }
    TimingSlot* t = &ws->tslots[ws->tnext];
    if (t->inflight) harvest_timings(ws, true);
    ws->tnext = (ws->tnext + 1) % kTimingRing;
    t->inflight = true;
    *out = t;
    return VTX_OK;
}

int get_workspace(hipStream_t stream, Workspace** out) {
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return VTX_OK;
    }
    Workspace* ws = new Workspace();
    ws->device = dev;
    ws->stream = stream;
    if (hipMalloc(&ws->bb.ctr, sizeof(Counters)) != hipSuccess) {
        delete ws;
        return fail(VTX_ENOMEM, "cannot allocate frame counters");
    }
    if (hipHostMalloc(&ws->host_ctr, sizeof(Counters), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        hipFree(ws->bb.ctr);
        delete ws;
        return fail(VTX_ENOMEM, "cannot allocate pinned counters");
    }
    std::memset(ws->host_ctr, 0, sizeof(Counters));
    void* dptr = nullptr;
    if (hipHostGetDevicePointer(&dptr, ws->host_ctr, 0) != hipSuccess) {
        hipFree(ws->bb.ctr);
        hipHostFree(ws->host_ctr);
        delete ws;
        return fail(VTX_EHIP, "cannot map pinned counters");
    }
    ws->bb.host_ctr = static_cast<Counters*>(dptr);
    if (hipEventCreateWithFlags(&ws->done, hipEventDisableTiming) != hipSuccess) {
        hipFree(ws->bb.ctr);
        hipHostFree(ws->host_ctr);
        delete ws;
        return fail(VTX_EHIP, "cannot create event");
    }
    g_ws[key] = ws;
    *out = ws;
    return VTX_OK;
}

template <class T>
int grow(T** p, size_t& cap, size_t want, hipStream_t stream, const char* what) {
    if (want <= cap && *p) return VTX_OK;
    VTX_HIP(hipStreamSynchronize(stream));   // in-flight frames may still read the old buffer
    hipFree(*p);
    *p = nullptr;
    cap = 0;
    if (hipMalloc(p, want * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(VTX_ENOMEM, "cannot allocate %zu bytes for %s", want * sizeof(T), what);
    }
    cap = want;
    return VTX_OK;
}

int ensure_buffers(Workspace* ws, int T, uint64_t nprim, uint32_t groups, uint32_t chunk) {
    size_t tc = ws->tiles_cap;
    int rc;
    if ((size_t)T > ws->tiles_cap || !ws->bb.tile_cnt) {
        size_t c1 = tc, c2 = tc, c3 = tc;
        if ((rc = grow(&ws->bb.tile_cnt, c1, (size_t)T, ws->stream, "tile counts"))) return rc;
        if ((rc = grow(&ws->bb.tile_off, c2, (size_t)T, ws->stream, "tile offsets"))) return rc;
        if ((rc = grow(&ws->bb.tile_fill, c3, (size_t)T, ws->stream, "tile cursors"))) return rc;
        ws->tiles_cap = (size_t)T;
        ws->dirty = true;
    }
    if (ws->dirty) {
        // every frame leaves the tile counts and the counters zeroed for the
        // next one; fresh or abandoned scratch is zeroed here instead
        VTX_HIP(vtx::launch_zero(ws->bb.tile_cnt, ws->tiles_cap, ws->stream));
        VTX_HIP(vtx::launch_zero(ws->bb.tile_fill, ws->tiles_cap, ws->stream));
        VTX_HIP(vtx::launch_zero(reinterpret_cast<uint32_t*>(ws->bb.ctr), sizeof(Counters) / sizeof(uint32_t),
                                 ws->stream));
        ws->dirty = false;
    }
    ws->bb.groups = groups;
    ws->bb.chunk = chunk;
    const size_t nv = (size_t)groups * chunk;
    if (nv > ws->vis_cap || !ws->bb.vis_rec) {
        size_t c1 = ws->vis_cap, c2 = ws->vis_cap;
        if ((rc = grow(&ws->bb.vis_rec, c1, nv, ws->stream, "visible records"))) return rc;
        if ((rc = grow(&ws->bb.vis_rect, c2, nv, ws->stream, "visible rectangles"))) return rc;
        ws->vis_cap = nv;
    }
    if ((size_t)groups > ws->groups_cap || !ws->bb.vis_cnt) {
        size_t c1 = ws->groups_cap, c2 = ws->groups_cap;
        if ((rc = grow(&ws->bb.vis_cnt, c1, (size_t)vtx::kMaxBinGroups, ws->stream, "visible counts"))) return rc;
        if ((rc = grow(&ws->bb.vis_box, c2, (size_t)vtx::kMaxBinGroups, ws->stream, "visible boxes"))) return rc;
        ws->groups_cap = vtx::kMaxBinGroups;
    }
    const size_t nh = (size_t)groups * (size_t)T;
    if (nh > ws->hist_cap || !ws->bb.hist) {
        size_t c1 = ws->hist_cap;
        if ((rc = grow(&ws->bb.hist, c1, nh, ws->stream, "tile histograms"))) return rc;
        ws->hist_cap = nh;
    }
    uint64_t want = ws->want_capacity;
    if (want == 0) {
        want = nprim / 2;
        if (want < kMinCapacity) want = kMinCapacity;
        if (want > kMaxCapacity) want = kMaxCapacity;
        ws->want_capacity = want;
    }
    if (want > ws->list_alloc || !ws->bb.list) {
        if ((rc = grow(&ws->bb.list, ws->list_alloc, (size_t)want, ws->stream, "tile lists"))) return rc;
    }
    ws->bb.capacity = want;
    return VTX_OK;
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

int make_frame(const vtx_camera* cam, const vtx_options& o, int32_t W, int32_t H, int64_t n, int64_t m,
               Frame* F) {
    if (!cam) return fail(VTX_EINVAL, "camera is NULL");
    if (W < 1 || H < 1 || (int64_t)W * H > VTX_MAX_PIXELS)
        return fail(VTX_EINVAL, "image %dx%d outside 1..%d pixels", W, H, VTX_MAX_PIXELS);
    if (n < 0 || m < 0 || n + m >= (int64_t)0xFFFFFFFFll)
        return fail(VTX_EINVAL, "n_atoms=%lld n_bonds=%lld out of range", (long long)n, (long long)m);
    if (!finite3(cam->eye) || !finite3(cam->target) || !finite3(cam->up))
        return fail(VTX_EINVAL, "camera vectors must be finite");
    if (!(cam->znear > 0.0f) || !(cam->zfar > cam->znear) || !std::isfinite(cam->zfar))
        return fail(VTX_EINVAL, "need 0 < znear < zfar < inf");
    if (cam->projection != VTX_PERSPECTIVE && cam->projection != VTX_ORTHOGRAPHIC)
        return fail(VTX_EINVAL, "unknown projection %d", cam->projection);
    if (cam->projection == VTX_PERSPECTIVE && !(cam->fovy > 0.0f && cam->fovy < 3.1415f))
        return fail(VTX_EINVAL, "fovy must be in (0, pi)");
    if (cam->projection == VTX_ORTHOGRAPHIC && !(cam->ortho_half_height > 0.0f && std::isfinite(cam->ortho_half_height)))
        return fail(VTX_EINVAL, "ortho_half_height must be > 0");
    if (!(o.bond_radius > 0.0f) || !std::isfinite(o.bond_radius)) return fail(VTX_EINVAL, "bond_radius must be > 0");
    if (o.ssao_samples < 0 || o.ssao_samples > VTX_MAX_SSAO_SAMPLES)
        return fail(VTX_EINVAL, "ssao_samples must be in 0..%d", VTX_MAX_SSAO_SAMPLES);
    if (o.ssao_samples > 0 && (!(o.ssao_radius >= 0.0f) || !std::isfinite(o.ssao_radius) || !std::isfinite(o.ssao_bias)))
        return fail(VTX_EINVAL, "ssao radius/bias must be finite, radius >= 0");
    if (o.tile_size != 0 && o.tile_size != 8 && o.tile_size != 16 && o.tile_size != 32 && o.tile_size != 64)
        return fail(VTX_EINVAL, "tile_size must be 0, 8, 16, 32 or 64");

    double e[3], f[3], up[3], s[3], u[3];
    for (int k = 0; k < 3; ++k) {
        e[k] = cam->eye[k];
        f[k] = (double)cam->target[k] - cam->eye[k];
        up[k] = cam->up[k];
    }
    const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0)) return fail(VTX_EINVAL, "eye and target coincide");
    for (double& v : f) v /= fl;
    s[0] = f[1] * up[2] - f[2] * up[1];
    s[1] = f[2] * up[0] - f[0] * up[2];
    s[2] = f[0] * up[1] - f[1] * up[0];
    const double sl = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    if (!(sl > 1e-12)) return fail(VTX_EINVAL, "up is parallel to the view direction");
    for (double& v : s) v /= sl;
    u[0] = s[1] * f[2] - s[2] * f[1];
    u[1] = s[2] * f[0] - s[0] * f[2];
    u[2] = s[0] * f[1] - s[1] * f[0];

    std::memset(F, 0, sizeof(Frame));
    for (int k = 0; k < 3; ++k) {
        F->eye[k] = e[k];
        F->s[k] = s[k];
        F->u[k] = u[k];
        F->f[k] = f[k];
    }
    const double aspect = (double)W / (double)H;
    const double th = std::tan((double)cam->fovy / 2.0);
    F->tx = th * aspect;
    F->ty = th;
    F->hx = (double)cam->ortho_half_height * aspect;
    F->hy = (double)cam->ortho_half_height;
    F->txf = (float)F->tx;
    F->tyf = (float)F->ty;
    F->sxf = (float)std::sqrt(1.0 + F->tx * F->tx) * (1.0f + 1e-6f);
    F->syf = (float)std::sqrt(1.0 + F->ty * F->ty) * (1.0f + 1e-6f);
    F->hxf = (float)F->hx;
    F->hyf = (float)F->hy;
    F->inv_w2 = 2.0f / (float)W;
    F->inv_h2 = 2.0f / (float)H;
    F->znear = cam->znear;
    F->zfar = cam->zfar;
    F->bond_radius = o.bond_radius;
    F->proj = cam->projection;
    F->W = W;
    F->H = H;
    // the binner keeps one tile histogram per workgroup in LDS: raise the tile
    // size until the tile grid fits it
    int ts = o.tile_size ? o.tile_size : 16;
    while ((int64_t)((W + ts - 1) / ts) * ((H + ts - 1) / ts) > vtx::kMaxLdsTiles) ts *= 2;
    if (ts > 64) return fail(VTX_EINVAL, "image %dx%d needs more than %d tiles of 64 pixels", W, H, vtx::kMaxLdsTiles);
    F->tile = ts;
    F->tiles_x = (W + F->tile - 1) / F->tile;
    F->tiles_y = (H + F->tile - 1) / F->tile;
    F->n_atoms = (uint32_t)n;
    F->n_bonds = (uint32_t)m;
    F->flags = o.flags;
    return VTX_OK;
}

vtx_options resolve_options(const vtx_options* opt) {
    vtx_options o;
    o.bond_radius = 0.15f;
    o.ssao_samples = 0;
    o.ssao_radius = 2.0f;
    o.ssao_bias = 0.05f;
    o.background = 0u;
    o.tile_size = 0;
    o.flags = 0u;
    return opt ? *opt : o;
}

int check_inputs(const float* positions, const float* radii, const uint32_t* colors, int64_t n,
                 const uint32_t* bonds, int64_t m, bool need_colors) {
    if (n > 0 && (!positions || !radii)) return fail(VTX_EINVAL, "positions/radii are NULL");
    if (n > 0 && need_colors && !colors) return fail(VTX_EINVAL, "colors are NULL");
    if (m > 0 && !bonds) return fail(VTX_EINVAL, "bonds are NULL");
    return VTX_OK;
}

// SSAO sample set: direction k on the hemisphere at polar angle
// acos(1 - (k + 1/2)/K) and azimuth 2 pi frac(k phi^-1), radius scale
// 0.1 + 0.9 ((k + 1)/K)^2; evaluated in double, stored in float.
void sample_kernel(const vtx_options& o, vtx::SampleKernel* K) {
    std::memset(K, 0, sizeof(*K));
    K->count = o.ssao_samples;
    K->radius = o.ssao_radius;
    K->bias = o.ssao_bias;
    K->background = o.background;
    const double golden = 0.6180339887498949;
    const double two_pi = 6.283185307179586;
    for (int k = 0; k < o.ssao_samples; ++k) {
        const double ct = 1.0 - (k + 0.5) / o.ssao_samples;
        const double st = std::sqrt(1.0 - ct * ct);
        const double ph = two_pi * std::fmod(k * golden, 1.0);
        const double sc = (k + 1.0) / o.ssao_samples;
        K->h[k] = make_float4((float)(st * std::cos(ph)), (float)(st * std::sin(ph)), (float)ct,
                              (float)(0.1 + 0.9 * sc * sc));
    }
}

int gbuffer_locked(const float* positions, const float* radii, int64_t n, const uint32_t* bonds, int64_t m,
                   const Frame& F, int32_t W, int32_t H, float* depth, uint32_t* id, hipStream_t stream,
                   hipEvent_t* marks = nullptr, const vtx::SceneDev* scene = nullptr) {
    Workspace* ws = nullptr;
    int rc = get_workspace(stream, &ws);
    if (rc) return rc;
    harvest(ws);
    const int T = F.tiles_x * F.tiles_y;
    uint32_t groups, chunk;
    if (!scene) {
        vtx::bin_grid((uint64_t)n + (uint64_t)m, &groups, &chunk);
    } else {
        // resident scene: each binning workgroup takes whole clusters
        const uint64_t nc = (uint64_t)scene->atom_clusters + scene->bond_clusters;
        vtx::bin_grid((uint64_t)n + (uint64_t)m, &groups, &chunk);
        const uint64_t cpw = (nc + groups - 1) / groups;
        chunk = (uint32_t)((cpw ? cpw : 1) * vtx::kCluster);
    }
    if ((rc = ensure_buffers(ws, T, (uint64_t)n + (uint64_t)m, groups, chunk))) return rc;
    ws->dirty = true;   // until the resolve that re-zeroes the tile counts is queued
    if (!scene) {
        VTX_HIP(vtx::launch_count(F, positions, radii, bonds, ws->bb, stream, marks));
    } else {
        if (marks) VTX_HIP(hipEventRecord(marks[0], stream));
        VTX_HIP(vtx::launch_cluster_cull(F, *scene, ws->bb.ctr, stream));
        VTX_HIP(vtx::launch_count_scene(F, *scene, ws->bb, stream, marks));
    }
    const uint64_t nprim = (uint64_t)n + (uint64_t)m;
    if (!ws->fixed_capacity && (nprim != ws->sized_nprim || W != ws->sized_w || H != ws->sized_h)) {
        // first frame of a new scene or image size: wait for the tile counts
        // and size the bins, so the frame does not take the overflow path
        unsigned long long counted = 0;
        VTX_HIP(hipMemcpyAsync(&counted, &ws->bb.ctr->pairs_counted, sizeof(counted), hipMemcpyDeviceToHost, stream));
        VTX_HIP(hipStreamSynchronize(stream));
        uint64_t want = counted + counted / 2 + 1024;
        if (want > kMaxCapacity) want = kMaxCapacity;
        if (want > ws->want_capacity) ws->want_capacity = want;
        if (ws->want_capacity > ws->list_alloc) {
            if ((rc = grow(&ws->bb.list, ws->list_alloc, (size_t)ws->want_capacity, ws->stream, "tile lists"))) return rc;
        }
        ws->bb.capacity = ws->want_capacity;
        ws->sized_nprim = nprim;
        ws->sized_w = W;
        ws->sized_h = H;
    }
    VTX_HIP(vtx::launch_scatter(F, ws->bb, stream, marks));
    if (marks) VTX_HIP(hipEventRecord(marks[4], stream));
    VTX_HIP(vtx::launch_resolve(F, positions, radii, bonds, ws->bb, depth, id, stream));
    ws->dirty = false;
    // The resolve's last workgroup writes the counters into the mapped pinned
    // buffer; the host reads them once the latest recorded event has completed.
    VTX_HIP(hipEventRecord(ws->done, stream));
    ws->pending = true;
    ws->pending_capacity = ws->bb.capacity;
    return VTX_OK;
}

}  // namespace

struct vtx_context {
    int device = 0;
    size_t budget = 0;       // bytes of scenes this context may keep resident (0 = no limit)
    size_t used = 0;
    std::mutex mu;
};

struct vtx_scene {
    vtx_context* ctx = nullptr;
    int device = 0;
    int64_t n = 0, m = 0;
    uint32_t bad_bonds = 0;
    size_t bytes = 0;
    vtx::SceneDev S{};
    float4* xyzr = nullptr;
    uint32_t* atom_id = nullptr;
    uint4* bond_rec = nullptr;
    float4* cluster_box = nullptr;
    uint32_t* vis_clusters = nullptr;
    // caller's arrays in their original order (the deferred pass reads them by id)
    float* pos = nullptr;
    float* rad = nullptr;
    uint32_t* col = nullptr;
    uint32_t* bonds = nullptr;
};

namespace {

size_t scene_bytes(int64_t n, int64_t m) {
    const size_t nc = (size_t)((n + vtx::kCluster - 1) / vtx::kCluster + (m + vtx::kCluster - 1) / vtx::kCluster);
    return (size_t)n * (sizeof(float4) + sizeof(uint32_t) + 3 * sizeof(float) + sizeof(float) + sizeof(uint32_t)) +
           (size_t)m * (sizeof(uint4) + 2 * sizeof(uint32_t)) + nc * (2 * sizeof(float4) + sizeof(uint32_t));
}

void scene_free(vtx_scene* sc) {
    hipFree(sc->xyzr);
    hipFree(sc->atom_id);
    hipFree(sc->bond_rec);
    hipFree(sc->cluster_box);
    hipFree(sc->vis_clusters);
    hipFree(sc->pos);
    hipFree(sc->rad);
    hipFree(sc->col);
    hipFree(sc->bonds);
}

template <class T>
int dev_alloc(T** p, size_t count, const char* what) {
    *p = nullptr;
    if (hipMalloc(p, (count ? count : 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(VTX_ENOMEM, "cannot allocate %zu bytes for %s", (count ? count : 1) * sizeof(T), what);
    }
    return VTX_OK;
}

}  // namespace

extern "C" {

int vtx_gbuffer(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
                const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
                int32_t W, int32_t H, float* depth, uint32_t* id, void* stream) {
    const vtx_options o = resolve_options(opt);
    Frame F;
    int rc = make_frame(cam, o, W, H, n_atoms, n_bonds, &F);
    if (rc) return rc;
    if ((rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, false))) return rc;
    if (!depth || !id) return fail(VTX_EINVAL, "depth/id outputs are NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    return gbuffer_locked(positions, radii, n_atoms, bonds, n_bonds, F, W, H, depth, id, (hipStream_t)stream);
}

int vtx_shade(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
              const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt, int32_t W,
              int32_t H, const float* depth, const uint32_t* id, uint32_t* rgba, float* normal, uint32_t* albedo,
              float* ao, void* stream) {
    const vtx_options o = resolve_options(opt);
    Frame F;
    int rc = make_frame(cam, o, W, H, n_atoms, n_bonds, &F);
    if (rc) return rc;
    if ((rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, true))) return rc;
    if (!depth || !id || !rgba) return fail(VTX_EINVAL, "depth/id/rgba are NULL");
    vtx::SampleKernel K;
    sample_kernel(o, &K);
    VTX_HIP(vtx::launch_shade(F, K, positions, radii, colors, bonds, depth, id, rgba, normal, albedo, ao,
                              (hipStream_t)stream));
    return VTX_OK;
}

int vtx_render(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
               const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
               int32_t W, int32_t H, uint32_t* rgba, float* depth, uint32_t* id, void* stream) {
    const vtx_options o = resolve_options(opt);
    Frame F;
    int rc = make_frame(cam, o, W, H, n_atoms, n_bonds, &F);
    if (rc) return rc;
    if ((rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, true))) return rc;
    if (!depth || !id || !rgba) return fail(VTX_EINVAL, "rgba/depth/id outputs are NULL");
    vtx::SampleKernel K;
    sample_kernel(o, &K);
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t* marks = nullptr;
    if (o.flags & VTX_FLAG_TIMING) {
        Workspace* ws = nullptr;
        if ((rc = get_workspace((hipStream_t)stream, &ws))) return rc;
        TimingSlot* slot = nullptr;
        if ((rc = timing_slot(ws, &slot))) return rc;
        marks = slot->ev;
    }
    rc = gbuffer_locked(positions, radii, n_atoms, bonds, n_bonds, F, W, H, depth, id, (hipStream_t)stream, marks);
    if (rc) return rc;
    if (marks) VTX_HIP(hipEventRecord(marks[5], (hipStream_t)stream));
    VTX_HIP(vtx::launch_shade(F, K, positions, radii, colors, bonds, depth, id, rgba, nullptr, nullptr, nullptr,
                              (hipStream_t)stream));
    if (marks) VTX_HIP(hipEventRecord(marks[6], (hipStream_t)stream));
    return VTX_OK;
}

int vtx_context_create(int device, size_t hbm_budget_bytes, vtx_context** out) {
    if (!out) return fail(VTX_EINVAL, "out is NULL");
    int count = 0;
    VTX_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(VTX_EINVAL, "device %d not in 0..%d", device, count - 1);
    vtx_context* c = new vtx_context();
    c->device = device;
    c->budget = hbm_budget_bytes;
    *out = c;
    return VTX_OK;
}

void vtx_context_destroy(vtx_context* ctx) { delete ctx; }

size_t vtx_context_bytes_in_use(const vtx_context* ctx) { return ctx ? ctx->used : 0; }

size_t vtx_scene_footprint_bytes(int64_t n_atoms, int64_t n_bonds) {
    if (n_atoms < 0 || n_bonds < 0) return 0;
    return scene_bytes(n_atoms, n_bonds);
}

size_t vtx_frame_scratch_bytes(int32_t W, int32_t H, int64_t n_atoms, int64_t n_bonds) {
    if (W < 1 || H < 1 || n_atoms < 0 || n_bonds < 0) return 0;
    int ts = 16;
    while ((int64_t)((W + ts - 1) / ts) * ((H + ts - 1) / ts) > vtx::kMaxLdsTiles) ts *= 2;
    const uint64_t T = (uint64_t)((W + ts - 1) / ts) * ((H + ts - 1) / ts);
    const uint64_t nprim = (uint64_t)n_atoms + (uint64_t)n_bonds;
    uint32_t groups, chunk;
    vtx::bin_grid(nprim, &groups, &chunk);
    uint64_t cap = nprim / 2;
    if (cap < kMinCapacity) cap = kMinCapacity;
    return (size_t)(T * 16 + (uint64_t)groups * chunk * (sizeof(vtx::PrimRec) + sizeof(uint2)) +
                    (uint64_t)groups * T * 4 + cap * sizeof(vtx::PrimRec) + sizeof(Counters) + 4096);
}

int vtx_scene_create(vtx_context* ctx, const float* positions, const float* radii, const uint32_t* colors,
                     int64_t n_atoms, const uint32_t* bonds, int64_t n_bonds, void* stream, vtx_scene** out) {
    if (!ctx || !out) return fail(VTX_EINVAL, "context/out is NULL");
    if (n_atoms < 0 || n_bonds < 0 || n_atoms + n_bonds >= (int64_t)0xFFFFFFFFll)
        return fail(VTX_EINVAL, "n_atoms=%lld n_bonds=%lld out of range", (long long)n_atoms, (long long)n_bonds);
    int rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, true);
    if (rc) return rc;
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    if (dev != ctx->device) return fail(VTX_EINVAL, "current device %d is not the context's %d", dev, ctx->device);
    const size_t bytes = scene_bytes(n_atoms, n_bonds);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->budget && ctx->used + bytes > ctx->budget)
            return fail(VTX_EBUSY, "scene of %zu bytes exceeds the context budget (%zu of %zu in use)", bytes,
                        ctx->used, ctx->budget);
        ctx->used += bytes;
    }
    hipStream_t st = (hipStream_t)stream;
    vtx_scene* sc = new vtx_scene();
    sc->ctx = ctx;
    sc->device = dev;
    sc->n = n_atoms;
    sc->m = n_bonds;
    sc->bytes = bytes;
    const size_t na = (size_t)n_atoms, nb = (size_t)n_bonds;
    const size_t ncl = (na + vtx::kCluster - 1) / vtx::kCluster + (nb + vtx::kCluster - 1) / vtx::kCluster;
    void* tmp = nullptr;
    const size_t tmp_bytes = vtx::scene_build_temp_bytes(na, nb);
    uint32_t m_valid = 0, n_bad = 0;
    auto bail = [&](int code) {
        scene_free(sc);
        hipFree(tmp);
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->used -= bytes;
        delete sc;
        return code;
    };
    if ((rc = dev_alloc(&sc->xyzr, na, "atom stream")) || (rc = dev_alloc(&sc->atom_id, na, "atom ids")) ||
        (rc = dev_alloc(&sc->bond_rec, nb, "bond records")) || (rc = dev_alloc(&sc->cluster_box, 2 * ncl, "cluster boxes")) ||
        (rc = dev_alloc(&sc->vis_clusters, ncl, "visible clusters")) || (rc = dev_alloc(&sc->pos, 3 * na, "positions")) ||
        (rc = dev_alloc(&sc->rad, na, "radii")) || (rc = dev_alloc(&sc->col, na, "colours")) ||
        (rc = dev_alloc(&sc->bonds, 2 * nb, "bonds")))
        return bail(rc);
    if (hipMalloc(&tmp, tmp_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(VTX_ENOMEM, "cannot allocate %zu bytes of build scratch", tmp_bytes));
    }
    if ((na && (hipMemcpyAsync(sc->pos, positions, 3 * na * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(sc->rad, radii, na * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(sc->col, colors, na * sizeof(uint32_t), hipMemcpyDeviceToDevice, st) != hipSuccess)) ||
        (nb && hipMemcpyAsync(sc->bonds, bonds, 2 * nb * sizeof(uint32_t), hipMemcpyDeviceToDevice, st) != hipSuccess))
        return bail(fail(VTX_EHIP, "copying the scene arrays failed"));
    sc->S.n_atoms = (uint32_t)na;
    sc->S.n_bonds_total = (uint32_t)nb;
    sc->S.xyzr = sc->xyzr;
    sc->S.atom_id = sc->atom_id;
    sc->S.bond_rec = sc->bond_rec;
    sc->S.vis_clusters = sc->vis_clusters;
    hipError_t e = vtx::scene_build(sc->pos, sc->rad, sc->bonds, na, nb, sc->S, sc->xyzr, sc->atom_id, sc->bond_rec,
                                    sc->cluster_box, tmp, tmp_bytes, &m_valid, &n_bad, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(VTX_EHIP, "building the scene failed: %s", hipGetErrorString(e)));
    hipFree(tmp);
    sc->bad_bonds = n_bad;
    *out = sc;
    return VTX_OK;
}

int vtx_scene_update_positions(vtx_scene* scene, const float* positions, void* stream) {
    if (!scene || (scene->n > 0 && !positions)) return fail(VTX_EINVAL, "scene/positions is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (scene->n)
        VTX_HIP(hipMemcpyAsync(scene->pos, positions, 3 * (size_t)scene->n * sizeof(float), hipMemcpyDeviceToDevice, st));
    VTX_HIP(vtx::scene_update_positions(scene->pos, scene->S, scene->xyzr, scene->cluster_box, st));
    return VTX_OK;
}

int vtx_scene_info(const vtx_scene* scene, int64_t* n_atoms, int64_t* n_bonds, uint64_t* bad_bonds,
                   size_t* bytes) {
    if (!scene) return fail(VTX_EINVAL, "scene is NULL");
    if (n_atoms) *n_atoms = scene->n;
    if (n_bonds) *n_bonds = scene->m;
    if (bad_bonds) *bad_bonds = scene->bad_bonds;
    if (bytes) *bytes = scene->bytes;
    return VTX_OK;
}

void vtx_scene_destroy(vtx_scene* scene) {
    if (!scene) return;
    (void)hipDeviceSynchronize();
    scene_free(scene);
    if (scene->ctx) {
        std::lock_guard<std::mutex> lk(scene->ctx->mu);
        scene->ctx->used -= scene->bytes;
    }
    delete scene;
}

int vtx_render_scene(vtx_scene* scene, const vtx_camera* cam, const vtx_options* opt, int32_t W, int32_t H,
                     uint32_t* rgba, float* depth, uint32_t* id, void* stream) {
    if (!scene) return fail(VTX_EINVAL, "scene is NULL");
    const vtx_options o = resolve_options(opt);
    Frame F;
    int rc = make_frame(cam, o, W, H, scene->n, scene->m, &F);
    if (rc) return rc;
    if (!depth || !id || !rgba) return fail(VTX_EINVAL, "rgba/depth/id outputs are NULL");
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    if (dev != scene->device) return fail(VTX_EINVAL, "scene lives on device %d, current is %d", scene->device, dev);
    vtx::SampleKernel K;
    sample_kernel(o, &K);
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t* marks = nullptr;
    if (o.flags & VTX_FLAG_TIMING) {
        Workspace* ws = nullptr;
        if ((rc = get_workspace((hipStream_t)stream, &ws))) return rc;
        TimingSlot* slot = nullptr;
        if ((rc = timing_slot(ws, &slot))) return rc;
        marks = slot->ev;
    }
    rc = gbuffer_locked(scene->pos, scene->rad, scene->n, scene->bonds, scene->m, F, W, H, depth, id,
                        (hipStream_t)stream, marks, &scene->S);
    if (rc) return rc;
    if (marks) VTX_HIP(hipEventRecord(marks[5], (hipStream_t)stream));
    VTX_HIP(vtx::launch_shade(F, K, scene->pos, scene->rad, scene->col, scene->bonds, depth, id, rgba, nullptr,
                              nullptr, nullptr, (hipStream_t)stream));
    if (marks) VTX_HIP(hipEventRecord(marks[6], (hipStream_t)stream));
    return VTX_OK;
}

int vtx_read_stats(void* stream, vtx_stats* out) {
    if (!out) return fail(VTX_EINVAL, "out is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    auto it = g_ws.find(std::make_pair(dev, (hipStream_t)stream));
    if (it == g_ws.end()) return fail(VTX_EINVAL, "no frame was rendered on this stream");
    Workspace* ws = it->second;
    if (ws->pending) VTX_HIP(hipEventSynchronize(ws->done));
    harvest(ws);
    if (!ws->have_stats) return fail(VTX_EINVAL, "no frame was rendered on this stream");
    *out = ws->last;
    return VTX_OK;
}

int vtx_set_bin_capacity(void* stream, uint64_t entries) {
    if (entries > kMaxCapacity) return fail(VTX_EINVAL, "capacity %llu > 2^28", (unsigned long long)entries);
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace* ws = nullptr;
    int rc = get_workspace((hipStream_t)stream, &ws);
    if (rc) return rc;
    VTX_HIP(hipStreamSynchronize(ws->stream));
    harvest(ws);
    ws->fixed_capacity = entries > 0;
    ws->want_capacity = entries;   // 0: re-derived from the next frame's size
    return VTX_OK;
}

int vtx_read_timings(void* stream, vtx_timings* out) {
    if (!out) return fail(VTX_EINVAL, "out is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace* ws = nullptr;
    int rc = get_workspace((hipStream_t)stream, &ws);
    if (rc) return rc;
    VTX_HIP(hipStreamSynchronize(ws->stream));
    harvest_timings(ws, true);
    std::memset(out, 0, sizeof(*out));
    out->frames = ws->tframes;
    if (ws->tframes) {
        const double n = (double)ws->tframes;
        out->ms_clear = ws->tsum[0] / n;
        out->ms_project = ws->tsum[1] / n;
        out->ms_scan = ws->tsum[2] / n;
        out->ms_scatter = ws->tsum[3] / n;
        out->ms_resolve = ws->tsum[4] / n;
        out->ms_shade = ws->tsum[5] / n;
    }
    return VTX_OK;
}

int vtx_reset_timings(void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace* ws = nullptr;
    int rc = get_workspace((hipStream_t)stream, &ws);
    if (rc) return rc;
    VTX_HIP(hipStreamSynchronize(ws->stream));
    harvest_timings(ws, true);
    ws->tframes = 0;
    for (double& v : ws->tsum) v = 0.0;
    return VTX_OK;
}

int vtx_release_scratch(void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    auto it = g_ws.find(std::make_pair(dev, (hipStream_t)stream));
    if (it == g_ws.end()) return VTX_OK;
    Workspace* ws = it->second;
    VTX_HIP(hipStreamSynchronize(ws->stream));
    free_ws_buffers(ws);
    if (ws->tslots) {
        for (int i = 0; i < kTimingRing; ++i)
            for (int m = 0; m < kMarks; ++m) hipEventDestroy(ws->tslots[i].ev[m]);
        delete[] ws->tslots;
    }
    hipFree(ws->bb.ctr);
    hipHostFree(ws->host_ctr);
    hipEventDestroy(ws->done);
    delete ws;
    g_ws.erase(it);
    return VTX_OK;
}

const char* vtx_last_error(void) { return g_error.c_str(); }

const char* vtx_version(void) { return "vtx-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"
