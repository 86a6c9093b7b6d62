// C ABI of the renderer (declared in include/vtx.h): argument checks, frame
// constants, per-stream scratch (tile bins) and the launch sequence
// cull -> count -> scatter -> resolve -> shade, for one render or a batch.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "vtx.h"
#include "vtx_internal.h"

namespace vtx {
KernelClock*& kernel_clock() {
    thread_local KernelClock* c = nullptr;
    return c;
}
}  // namespace vtx

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
constexpr int kTimeCats = 6;  // clear, project, scan, scatter, resolve, shade
constexpr int kMaxBatch = 4096;

// Events of one timed frame: a start and a stop event per kernel dispatch.
struct TimingSlot {
    vtx::KernelClock clock{};
    bool inflight = false;
};

// Sets the host thread's kernel clock for the lifetime of a render call.
struct ClockScope {
    explicit ClockScope(vtx::KernelClock* c) { vtx::kernel_clock() = c; }
    ~ClockScope() { vtx::kernel_clock() = nullptr; }
    void category(int cat) {
        if (vtx::kernel_clock()) vtx::kernel_clock()->cur = cat;
    }
};

// Binning scratch of one render slot: a single render uses slot 0, job i of a
// batch uses slot i.  Every frame leaves the tile counts, cursors and counters
// zeroed for the next one.
struct Bins {
    BinBuffers bb{};
    size_t tiles_cap = 0;
    size_t vis_cap = 0;
    size_t groups_cap = 0;
    size_t hist_cap = 0;
    size_t list_alloc = 0;          // allocated bin entries (>= bb.capacity, the entries in use)
    size_t vc_cap = 0;
    size_t hz16_cap = 0;
    uint32_t* vis_clusters = nullptr;   // resident scenes: the clusters that passed the frustum test
    // supersampled renders: the full-size depth, id and colour images
    float* ss_depth = nullptr;
    uint32_t* ss_id = nullptr;
    uint32_t* ss_rgba = nullptr;
    size_t ss_cap = 0;
    Counters* host_ctr = nullptr;       // host view of the mapped counters
    uint64_t want_capacity = 0;
    uint64_t pending_capacity = 0;
    uint64_t pending_uid = 0;       // resident scene of the render queued in this slot (0: none)
    int pending_w = 0, pending_h = 0;
    bool dirty = true;              // tile counts / counters must be zeroed before the next frame
    // (primitives, width, height) of the renders the lists were sized for,
    // most recent last; the lists only grow, so a render of a known size
    // needs no new sizing
    std::vector<std::array<int64_t, 3>> sized;
    bool was_sized(uint64_t nprim, int w, int h) const {
        for (const auto& k : sized)
            if (k[0] == (int64_t)nprim && k[1] == w && k[2] == h) return true;
        return false;
    }
    void mark_sized(uint64_t nprim, int w, int h) {
        if (was_sized(nprim, w, h)) return;
        if (sized.size() >= 16) sized.erase(sized.begin());
        sized.push_back({(int64_t)nprim, (int64_t)w, (int64_t)h});
    }
};

// Scratch of one (device, stream).
struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<Bins*> slots;
    hipEvent_t done = nullptr;
    bool pending = false;
    int pending_n = 0;
    bool have_stats = false;
    bool fixed_capacity = false;
    uint64_t fixed_entries = 0;
    vtx_stats last{};
    TimingSlot* tslots = nullptr;   // ring of kTimingRing, created on first timed frame
    int tnext = 0;
    uint64_t tframes = 0;
    double tsum[kTimeCats] = {};
    // overflowed tiles of a resolve launch (job << 32 | tile) and its two
    // counters, left zeroed by every launch
    unsigned long long* d_ovf = nullptr;
    size_t ovf_cap = 0;
    uint32_t* d_ovf_n = nullptr;
    // solvent excluded surface calls: scratch words and the field when the
    // caller takes none
    uint32_t* ses = nullptr;
    size_t ses_cap = 0;
    // job tables of batched launches: device copy and pinned staging
    char* d_tab = nullptr;
    char* h_tab = nullptr;
    size_t tab_cap = 0;
    hipEvent_t staged = nullptr;
    bool stage_busy = false;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
// Largest (primitive, tile) pair count seen per resident scene and image
// size: a slot that meets a known scene and size sizes its lists from it
// instead of waiting for the frame's count (serving many scenes in
// alternation).  Keyed by the scenes' unique ids; guarded by g_mu.
std::map<uint64_t, std::map<std::pair<int, int>, uint64_t>> g_pairs_seen;
uint64_t g_next_scene_uid = 1;

void note_pairs(uint64_t uid, int w, int h, uint64_t pairs) {
    if (!uid) return;
    uint64_t& v = g_pairs_seen[uid][{w, h}];
    if (pairs > v) v = pairs;
}

uint64_t seen_pairs(uint64_t uid, int w, int h) {
    if (!uid) return 0;
    auto it = g_pairs_seen.find(uid);
    if (it == g_pairs_seen.end()) return 0;
    auto jt = it->second.find({w, h});
    return jt == it->second.end() ? 0 : jt->second;
}

constexpr uint64_t kMaxCapacity = 1ull << 28;        // bin entries (2 GiB of 8-byte entries)
constexpr uint64_t kMinCapacity = 1ull << 20;

void bins_free(Bins* b) {
    hipFree(b->bb.tile_cnt);
    hipFree(b->bb.tile_off);
    hipFree(b->bb.tile_fill);
    hipFree(b->bb.layer_off);
    hipFree(b->bb.layer_sum);
    hipFree(b->bb.hz16);
    hipFree(b->bb.vis_src);
    hipFree(b->bb.vis_rect);
    hipFree(b->bb.vis_cnt);
    hipFree(b->bb.vis_box);
    hipFree(b->bb.hist);
    hipFree(b->bb.list);
    hipFree(b->bb.ctr);
    hipFree(b->vis_clusters);
    hipFree(b->ss_depth);
    hipFree(b->ss_id);
    hipFree(b->ss_rgba);
    hipHostFree(b->host_ctr);
    delete b;
}

int bins_new(Bins** out) {
    Bins* b = new Bins();
    if (hipMalloc(&b->bb.ctr, sizeof(Counters)) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(VTX_ENOMEM, "cannot allocate frame counters");
    }
    if (hipHostMalloc(&b->host_ctr, sizeof(Counters), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        hipFree(b->bb.ctr);
        delete b;
        return fail(VTX_ENOMEM, "cannot allocate pinned counters");
    }
    std::memset(b->host_ctr, 0, sizeof(Counters));
    void* dptr = nullptr;
    if (hipHostGetDevicePointer(&dptr, b->host_ctr, 0) != hipSuccess) {
        (void)hipGetLastError();
        hipFree(b->bb.ctr);
        hipHostFree(b->host_ctr);
        delete b;
        return fail(VTX_EHIP, "cannot map pinned counters");
    }
    b->bb.host_ctr = static_cast<Counters*>(dptr);
    *out = b;
    return VTX_OK;
}

// Reads the counters of a completed call into ws->last (sums over its renders)
// and grows the bins of any render whose lists overflowed.
void harvest(Workspace* ws) {
    if (!ws->pending) return;
    if (hipEventQuery(ws->done) != hipSuccess) return;
    vtx_stats s{};
    for (int i = 0; i < ws->pending_n; ++i) {
        Bins* b = ws->slots[i];
        const Counters& c = *b->host_ctr;
        s.visible += c.vis_count;
        s.pairs += c.pairs;
        s.fragments_tested += c.frag_tested;
        s.fragments_hit += c.frag_hit;
        s.fragments_hit_bond += c.frag_hit_bond;
        s.fragments_tested_bond += c.frag_tested_bond;
        s.fragments_skipped += c.frag_skipped;
        s.records_culled += c.rec_culled;
        s.lists_stopped += c.lists_stopped;
        s.chunks_stopped += c.chunks_stopped;
        s.overflow_tiles += c.overflow_tiles;
        s.bin_capacity += b->pending_capacity;
        s.bad_bonds += c.bad_bonds;
        note_pairs(b->pending_uid, b->pending_w, b->pending_h, c.pairs);
        if (c.pairs > b->bb.capacity && !ws->fixed_capacity) {
            uint64_t want = c.pairs + c.pairs / 2 + 1024;
            if (want > kMaxCapacity) want = kMaxCapacity;
            if (want > b->want_capacity) b->want_capacity = want;
        }
    }
    ws->last = s;
    ws->have_stats = true;
    ws->pending = false;
}

void harvest_timings(Workspace* ws, bool wait) {
    if (!ws->tslots) return;
    for (int k = 0; k < kTimingRing; ++k) {
        const int i = (ws->tnext + k) % kTimingRing;   // oldest first
        TimingSlot& t = ws->tslots[i];
        if (!t.inflight) continue;
        const vtx::KernelClock& c = t.clock;
        if (c.used < 1) {   // the frame failed before a kernel was queued
            t.inflight = false;
            continue;
        }
        const int last = c.used - 1;
        if (wait) (void)hipEventSynchronize(c.stop[last]);
        if (hipEventQuery(c.stop[last]) != hipSuccess) break;
        for (int m = 0; m < c.used; ++m) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, c.start[m], c.stop[m]) == hipSuccess) ws->tsum[c.cat[m]] += ms;
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
            for (int m = 0; m < vtx::KernelClock::kMax; ++m)
                if (hipEventCreate(&ws->tslots[i].clock.start[m]) != hipSuccess ||
                    hipEventCreate(&ws->tslots[i].clock.stop[m]) != hipSuccess)
                    return fail(VTX_EHIP, "hipEventCreate failed");
    }
    TimingSlot* t = &ws->tslots[ws->tnext];
    if (t->inflight) harvest_timings(ws, true);
    ws->tnext = (ws->tnext + 1) % kTimingRing;
    t->inflight = true;
    t->clock.used = 0;
    t->clock.cur = 0;
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
    if (hipEventCreateWithFlags(&ws->done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ws->staged, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (ws->done) hipEventDestroy(ws->done);
        delete ws;
        return fail(VTX_EHIP, "cannot create events");
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

// Sizes slot b for a render with T tiles, nprim primitives binned by
// `groups` workgroups of `chunk`, and nc scene clusters (0 for the plain path).
int ensure_bins(Workspace* ws, Bins* b, int T, uint64_t nprim, uint32_t groups, uint32_t chunk, uint32_t nc, int W,
                int H) {
    int rc;
    hipStream_t st = ws->stream;
    if ((size_t)T > b->tiles_cap || !b->bb.tile_cnt) {
        size_t c1 = b->tiles_cap, c2 = b->tiles_cap, c3 = b->tiles_cap * vtx::kLayers, c4 = c3;
        if ((rc = grow(&b->bb.tile_cnt, c1, (size_t)T, st, "tile counts"))) return rc;
        if ((rc = grow(&b->bb.tile_off, c2, (size_t)T, st, "tile offsets"))) return rc;
        if ((rc = grow(&b->bb.tile_fill, c3, (size_t)T * vtx::kLayers, st, "tile cursors"))) return rc;
        if ((rc = grow(&b->bb.layer_off, c4, (size_t)T * vtx::kLayers, st, "tile layer starts"))) return rc;
        size_t c5 = b->tiles_cap * vtx::kLayers;
        if ((rc = grow(&b->bb.layer_sum, c5, (size_t)T * vtx::kLayers, st, "tile layer totals"))) return rc;
        b->tiles_cap = (size_t)T;
        b->dirty = true;
    }
    if (b->dirty) {
        // fresh or abandoned scratch: zero what every frame otherwise leaves zeroed
        VTX_HIP(vtx::launch_zero(b->bb.tile_cnt, b->tiles_cap, st));
        VTX_HIP(vtx::launch_zero(b->bb.tile_fill, b->tiles_cap * vtx::kLayers, st));
        VTX_HIP(vtx::launch_zero(b->bb.layer_sum, b->tiles_cap * vtx::kLayers, st));
        VTX_HIP(vtx::launch_zero(reinterpret_cast<uint32_t*>(b->bb.ctr), sizeof(Counters) / sizeof(uint32_t), st));
        b->dirty = false;
    }
    b->bb.groups = groups;
    b->bb.chunk = chunk;
    const size_t nv = (size_t)groups * chunk;
    if (nv > b->vis_cap || !b->bb.vis_src) {
        size_t c1 = b->vis_cap, c2 = b->vis_cap;
        if ((rc = grow(&b->bb.vis_src, c1, nv, st, "visible sources"))) return rc;
        if ((rc = grow(&b->bb.vis_rect, c2, nv, st, "visible rectangles"))) return rc;
        b->vis_cap = nv;
    }
    if ((size_t)groups > b->groups_cap || !b->bb.vis_cnt) {
        size_t c1 = b->groups_cap, c2 = b->groups_cap;
        if ((rc = grow(&b->bb.vis_cnt, c1, (size_t)vtx::kMaxBinGroups, st, "visible counts"))) return rc;
        if ((rc = grow(&b->bb.vis_box, c2, (size_t)vtx::kMaxBinGroups, st, "visible boxes"))) return rc;
        b->groups_cap = vtx::kMaxBinGroups;
    }
    const size_t nh = (size_t)groups * (size_t)T;
    if (nh > b->hist_cap || !b->bb.hist) {
        size_t c1 = b->hist_cap;
        if ((rc = grow(&b->bb.hist, c1, nh, st, "tile histograms"))) return rc;
        b->hist_cap = nh;
    }
    if (nc) {   // resident scenes: 16x16-cell depths of the occlusion pre-pass
        const size_t cw = (size_t)(W + vtx::kHzCell - 1) / vtx::kHzCell, ch = (size_t)(H + vtx::kHzCell - 1) / vtx::kHzCell;
        if (cw * ch > b->hz16_cap || !b->bb.hz16) {
            if ((rc = grow(&b->bb.hz16, b->hz16_cap, cw * ch, st, "cell depths"))) return rc;
        }
        b->bb.hz16_w = (int32_t)cw;
    }
    if (nc && ((size_t)nc * vtx::kDepthBuckets > b->vc_cap || !b->vis_clusters)) {
        if ((rc = grow(&b->vis_clusters, b->vc_cap, (size_t)nc * vtx::kDepthBuckets, st, "visible clusters"))) return rc;
    }
    uint64_t want = ws->fixed_capacity ? ws->fixed_entries : b->want_capacity;
    if (want == 0) {
        want = nprim / 2;
        if (want < kMinCapacity) want = kMinCapacity;
        if (want > kMaxCapacity) want = kMaxCapacity;
        b->want_capacity = want;
    }
    if (want > b->list_alloc || !b->bb.list) {
        if ((rc = grow(&b->bb.list, b->list_alloc, (size_t)want, st, "tile lists"))) return rc;
    }
    b->bb.capacity = want;
    return VTX_OK;
}

size_t xcd_round(uint32_t n) { return ((size_t)n + 7) / 8 * 8; }

template <class T>
int dev_alloc_zeroed(T** p, size_t count, hipStream_t stream) {
    if (hipMalloc(p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(VTX_ENOMEM, "cannot allocate %zu bytes", count * sizeof(T));
    }
    VTX_HIP(vtx::launch_zero(reinterpret_cast<uint32_t*>(*p), count * sizeof(T) / sizeof(uint32_t), stream));
    return VTX_OK;
}

void workspace_free(Workspace* ws) {
    for (Bins* b : ws->slots) bins_free(b);
    ws->slots.clear();
    if (ws->tslots) {
        for (int i = 0; i < kTimingRing; ++i)
            for (int m = 0; m < vtx::KernelClock::kMax; ++m) {
                hipEventDestroy(ws->tslots[i].clock.start[m]);
                hipEventDestroy(ws->tslots[i].clock.stop[m]);
            }
        delete[] ws->tslots;
    }
    hipFree(ws->ses);
    hipFree(ws->d_tab);
    hipHostFree(ws->h_tab);
    hipFree(ws->d_ovf);
    hipFree(ws->d_ovf_n);
    hipEventDestroy(ws->done);
    hipEventDestroy(ws->staged);
    delete ws;
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

int make_frame(const vtx_camera* cam, const vtx_options& o, int32_t W, int32_t H, int64_t n, int64_t m,
               Frame* F) {
    if (!cam) return fail(VTX_EINVAL, "camera is NULL");
    if (o.supersample < 0 || o.supersample > 4) return fail(VTX_EINVAL, "supersample must be in 0..4");
    if (W < 1 || H < 1 || (int64_t)W * H > VTX_MAX_PIXELS)
        return fail(VTX_EINVAL, "image %dx%d outside 1..%d pixels", W, H, VTX_MAX_PIXELS);
    // a supersampled frame is rendered at S times the size on each side
    const int ss = o.supersample > 1 ? o.supersample : 1;
    if ((int64_t)W * ss * H * ss > VTX_MAX_PIXELS)
        return fail(VTX_EINVAL, "image %dx%d supersampled %d times exceeds %d pixels", W, H, ss, VTX_MAX_PIXELS);
    W *= ss;
    H *= ss;
    if (W > VTX_MAX_SIDE || H > VTX_MAX_SIDE)
        return fail(VTX_EINVAL, "image %dx%d has a side above %d pixels", W, H, VTX_MAX_SIDE);
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
    if (o.ssao_noise != 0 && o.ssao_noise != 1) return fail(VTX_EINVAL, "ssao_noise must be 0 or 1");
    if (o.tile_size != 0 && o.tile_size != 8 && o.tile_size != 16 && o.tile_size != 32 && o.tile_size != 64)
        return fail(VTX_EINVAL, "tile_size must be 0, 8, 16, 32 or 64");
    if (o.representation < VTX_REP_BALL_AND_STICK || o.representation > VTX_REP_SAS)
        return fail(VTX_EINVAL, "unknown representation %d", o.representation);
    if (o.representation == VTX_REP_SAS && !(o.probe_radius >= 0.0f && std::isfinite(o.probe_radius)))
        return fail(VTX_EINVAL, "probe_radius must be finite and >= 0");
    if (o.shading < VTX_SHADE_GLOSSY || o.shading > VTX_SHADE_TOON) return fail(VTX_EINVAL, "unknown shading %d", o.shading);
    if (!std::isfinite(o.fog_start) || !std::isfinite(o.fog_end)) return fail(VTX_EINVAL, "fog depths must be finite");
    if (!(o.outline_depth >= 0.0f) || !std::isfinite(o.outline_depth))
        return fail(VTX_EINVAL, "outline_depth must be finite and >= 0");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(o.clip_plane[k])) return fail(VTX_EINVAL, "clip_plane must be finite");
    const bool clip_on = o.clip_plane[0] != 0.0f || o.clip_plane[1] != 0.0f || o.clip_plane[2] != 0.0f;
    if (!clip_on && o.clip_plane[3] != 0.0f) return fail(VTX_EINVAL, "clip_plane has a zero normal");

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
    F->itx = 1.0 / F->tx;
    F->ity = 1.0 / F->ty;
    F->ihx = 1.0 / F->hx;
    F->ihy = 1.0 / F->hy;
    F->txf = (float)F->tx;
    F->tyf = (float)F->ty;
    F->itxf = (float)F->itx;
    F->ityf = (float)F->ity;
    F->sxf = (float)std::sqrt(1.0 + F->tx * F->tx) * (1.0f + 1e-6f);
    F->syf = (float)std::sqrt(1.0 + F->ty * F->ty) * (1.0f + 1e-6f);
    F->hxf = (float)F->hx;
    F->hyf = (float)F->hy;
    F->inv_w2 = 2.0f / (float)W;
    F->inv_h2 = 2.0f / (float)H;
    F->ssao_fpx = 0.5f * (float)H / F->tyf;
    F->ssao_osc = 0.5f * (float)H / F->hyf;
    F->inv_w2d = 2.0 / (double)W;
    F->inv_h2d = 2.0 / (double)H;
    F->znear = cam->znear;
    F->zfar = cam->zfar;
    // depth classes from znear to zfar (resident scenes narrow them to the scene)
    F->cls_z0 = cam->znear;
    F->cls_k = (float)(vtx::kDepthBuckets / std::log2((double)cam->zfar / (double)cam->znear));
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
    F->tile_shift = ts == 8 ? 3 : ts == 16 ? 4 : ts == 32 ? 5 : 6;
    F->tiles_x = (W + F->tile - 1) / F->tile;
    F->tiles_y = (H + F->tile - 1) / F->tile;
    F->n_atoms = (uint32_t)n;
    const bool bonds_drawn = o.representation == VTX_REP_BALL_AND_STICK || o.representation == VTX_REP_STICKS;
    F->n_bonds = bonds_drawn ? (uint32_t)m : 0u;
    F->flags = o.flags;
    F->rep = o.representation;
    F->probe = o.probe_radius;
    F->shading = o.shading;
    F->fog_start = o.fog_start;
    F->fog_inv = o.fog_end > o.fog_start ? (float)(1.0 / ((double)o.fog_end - (double)o.fog_start)) : 0.0f;
    for (int ch = 0; ch < 3; ++ch) F->fog_rgb[ch] = (float)((o.fog_color >> (8 * ch)) & 255u) * (1.0f / 255.0f);
    F->outline_t = o.outline_depth;
    F->outline_rgba = o.outline_color | 0xFF000000u;
    F->clip_on = clip_on ? 1 : 0;
    // ids are below n + m: the top bit is free for the resolve's refine mark
    F->refine_flag = n + m < (int64_t)0x7FFFFFFF ? 1 : 0;
    if (clip_on) {
        // a.x + d with x = eye + X s + Y u + Z f: (a.s, a.u, a.f, a.eye + d)
        const double a[3] = {o.clip_plane[0], o.clip_plane[1], o.clip_plane[2]};
        F->clip[0] = (float)(a[0] * s[0] + a[1] * s[1] + a[2] * s[2]);
        F->clip[1] = (float)(a[0] * u[0] + a[1] * u[1] + a[2] * u[2]);
        F->clip[2] = (float)(a[0] * f[0] + a[1] * f[1] + a[2] * f[2]);
        F->clip[3] = (float)(a[0] * e[0] + a[1] * e[1] + a[2] * e[2] + (double)o.clip_plane[3]);
    }
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
    o.representation = VTX_REP_BALL_AND_STICK;
    o.probe_radius = 1.4f;
    o.shading = VTX_SHADE_GLOSSY;
    o.fog_color = 0u;
    o.fog_start = 0.0f;
    o.fog_end = 0.0f;
    o.outline_color = 0u;
    o.outline_depth = 0.0f;
    for (float& v : o.clip_plane) v = 0.0f;
    o.supersample = 1;
    o.ssao_noise = 0;
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
    K->noise = o.ssao_noise;
    const double golden = 0.6180339887498949;
    const double two_pi = 6.283185307179586;
    for (int b = 0; b < 16; ++b) {
        const double th = two_pi * (b + 0.5) / 16.0;
        K->rot[b] = make_float2((float)std::cos(th), (float)std::sin(th));
    }
    for (int k = 0; k < o.ssao_samples; ++k) {
        const double ct = 1.0 - (k + 0.5) / o.ssao_samples;
        const double st = std::sqrt(1.0 - ct * ct);
        const double ph = two_pi * std::fmod(k * golden, 1.0);
        const double sc = (k + 1.0) / o.ssao_samples;
        const double len = (double)o.ssao_radius * (0.1 + 0.9 * sc * sc);   // offset length
        K->h[k] = make_float4((float)(len * st * std::cos(ph)), (float)(len * st * std::sin(ph)), (float)(len * ct),
                              (float)len);
    }
}


}  // namespace

// Choices of vtx_autotune for one shape.
struct TunedShape {
    int tile = 0;            // tile size (0: none)
    int ssao = -1;           // SSAO samples of VTX_SSAO_AUTO renders (-1: none chosen)
    uint64_t capacity = 0;   // tile-list entries for a render's new scratch (0: none)
};
constexpr int kAutoSsaoDefault = 16;

struct vtx_context {
    int device = 0;
    size_t budget = 0;       // bytes of scenes this context may keep resident (0 = no limit)
    size_t used = 0;
    std::mutex mu;
    std::map<std::string, TunedShape> tuned;   // shape key -> choices of vtx_autotune
};

// Positions of one stored trajectory frame.
struct SceneFrame {
    float* pos;              // caller's order (deferred pass)
    float4* xyzr;            // stored (Morton) order
    float4* cluster_box;
};

struct vtx_scene {
    vtx_context* ctx = nullptr;
    uint64_t uid = 0;        // unique per scene of the process
    int device = 0;
    int64_t n = 0, m = 0;
    uint32_t bad_bonds = 0;
    size_t bytes = 0;
    vtx::SceneDev S{};       // frame 0
    float4* xyzr = nullptr;
    uint32_t* atom_id = nullptr;
    uint4* bond_rec = nullptr;
    float4* cluster_box = nullptr;
    // caller's arrays in their original order (the deferred pass reads them by id)
    float* pos = nullptr;
    float* rad = nullptr;
    uint32_t* col = nullptr;
    uint32_t* bonds = nullptr;
    std::vector<SceneFrame> frames;     // frames 1, 2, ... added after creation
    std::vector<void*> frame_blocks;    // their allocations
    bool have_box = false;              // bounding box of the atoms at creation
    double box_lo[3] = {}, box_hi[3] = {};
};

// Depth classes of a resident scene's render: log-spaced over the view depths
// of the scene's bounding box at creation (trajectory frames and updated
// positions may stray from it; classes only order the tile lists).
static void scene_depth_classes(const vtx_scene* sc, Frame* F) {
    if (!sc->have_box) return;
    double zlo = INFINITY, zhi = -INFINITY;
    for (int c = 0; c < 8; ++c) {
        const double p[3] = {(c & 1) ? sc->box_hi[0] : sc->box_lo[0], (c & 2) ? sc->box_hi[1] : sc->box_lo[1],
                             (c & 4) ? sc->box_hi[2] : sc->box_lo[2]};
        const double z = (p[0] - F->eye[0]) * F->f[0] + (p[1] - F->eye[1]) * F->f[1] + (p[2] - F->eye[2]) * F->f[2];
        zlo = std::min(zlo, z);
        zhi = std::max(zhi, z);
    }
    zlo = std::max(zlo, (double)F->znear);
    zhi = std::min(zhi, (double)F->zfar);
    if (!(zlo > 0.0 && zhi > zlo * 1.001)) return;
    F->cls_z0 = (float)zlo;
    F->cls_k = (float)(vtx::kDepthBuckets / std::log2(zhi / zlo));
}


namespace {

size_t scene_clusters(int64_t n, int64_t m) {
    return (size_t)((n + vtx::kCluster - 1) / vtx::kCluster + (m + vtx::kCluster - 1) / vtx::kCluster);
}

size_t scene_bytes(int64_t n, int64_t m) {
    return (size_t)n * (sizeof(float4) + sizeof(uint32_t) + 3 * sizeof(float) + sizeof(float) + sizeof(uint32_t)) +
           (size_t)m * (sizeof(uint4) + 2 * sizeof(uint32_t)) + scene_clusters(n, m) * 2 * sizeof(float4);
}

// Device bytes of one added trajectory frame.
size_t frame_bytes(int64_t n, int64_t m) {
    return (size_t)n * (3 * sizeof(float) + sizeof(float4)) + scene_clusters(n, m) * 2 * sizeof(float4);
}

void scene_free(vtx_scene* sc) {
    hipFree(sc->xyzr);
    hipFree(sc->atom_id);
    hipFree(sc->bond_rec);
    hipFree(sc->cluster_box);
    hipFree(sc->pos);
    hipFree(sc->rad);
    hipFree(sc->col);
    hipFree(sc->bonds);
    for (void* p : sc->frame_blocks) hipFree(p);
    sc->frame_blocks.clear();
    sc->frames.clear();
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

// The scene arrays of trajectory frame f (0 = the positions given at creation
// or by the last update).
void scene_frame(const vtx_scene* sc, int f, vtx::SceneDev* S, const float** pos) {
    *S = sc->S;
    *pos = sc->pos;
    if (f > 0) {
        const SceneFrame& fr = sc->frames[(size_t)f - 1];
        S->xyzr = fr.xyzr;
        S->cluster_box = fr.cluster_box;
        *pos = fr.pos;
    }
}

// Shape the tuned choices apply to: image size, primitive count (by powers
// of two) and projection.
std::string shape_key(int32_t W, int32_t H, int64_t n, int64_t m, int32_t projection) {
    int lg = 0;
    for (uint64_t v = (uint64_t)(n + m); v > 1; v >>= 1) ++lg;
    char buf[96];
    snprintf(buf, sizeof(buf), "%dx%d/p%d/%s", W, H, lg, projection == VTX_ORTHOGRAPHIC ? "ortho" : "persp");
    return buf;
}

// Options with the choices the context tuned for this shape where the
// caller left them to the library (tile size 0, VTX_SSAO_AUTO samples), and
// the tuned tile-list capacity (0: none).
vtx_options tuned_options(vtx_context* ctx, vtx_options o, const vtx_camera* cam, int32_t W, int32_t H,
                          int64_t n, int64_t m, uint64_t* capacity = nullptr) {
    if (capacity) *capacity = 0;
    if (ctx && cam) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->tuned.find(shape_key(W, H, n, m, cam->projection));
        if (it != ctx->tuned.end()) {
            if (o.tile_size == 0) o.tile_size = it->second.tile;
            if (o.ssao_samples == VTX_SSAO_AUTO && it->second.ssao >= 0) o.ssao_samples = it->second.ssao;
            if (capacity) *capacity = it->second.capacity;
        }
    }
    if (o.ssao_samples == VTX_SSAO_AUTO) o.ssao_samples = kAutoSsaoDefault;
    return o;
}

// The same for renders without a context.
vtx_options untuned_options(vtx_options o) {
    if (o.ssao_samples == VTX_SSAO_AUTO) o.ssao_samples = kAutoSsaoDefault;
    return o;
}

// Host description of one render.
struct JobDesc {
    Frame F;
    vtx::SampleKernel K;
    const float* pos;
    const float* rad;
    const uint32_t* col;
    const uint32_t* bonds;
    bool scene;
    uint64_t scene_uid;
    uint64_t tuned_capacity = 0;   // tile-list entries the tuner chose for this render's shape (0: none)
    int ss = 1;                    // samples per pixel side: F is S times the outputs' size
    vtx::SceneDev S;
    float* depth;
    uint32_t* id;
    uint32_t* rgba;
    float* normal;
    uint32_t* albedo;
    float* ao;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Copies the job tables of a batched launch to the device (through pinned
// staging that is reused once the previous copy has finished).
int upload_tables(Workspace* ws, const std::vector<vtx::Job>& jobs, const std::vector<JobDesc>& d,
                  const std::vector<uint32_t>& starts, size_t* k_off, size_t* s_off) {
    const size_t n = jobs.size();
    *k_off = align_up(n * sizeof(vtx::Job), 256);
    *s_off = align_up(*k_off + n * sizeof(vtx::SampleKernel), 256);
    const size_t bytes = *s_off + starts.size() * sizeof(uint32_t);
    if (ws->stage_busy) VTX_HIP(hipEventSynchronize(ws->staged));
    ws->stage_busy = false;
    if (bytes > ws->tab_cap) {
        VTX_HIP(hipStreamSynchronize(ws->stream));   // the old device table may still be read
        hipFree(ws->d_tab);
        hipHostFree(ws->h_tab);
        ws->d_tab = nullptr;
        ws->h_tab = nullptr;
        ws->tab_cap = 0;
        const size_t cap = align_up(bytes + bytes / 2, 4096);
        if (hipMalloc(&ws->d_tab, cap) != hipSuccess || hipHostMalloc(&ws->h_tab, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(VTX_ENOMEM, "cannot allocate %zu bytes of job tables", cap);
        }
        ws->tab_cap = cap;
    }
    std::memcpy(ws->h_tab, jobs.data(), n * sizeof(vtx::Job));
    for (size_t i = 0; i < n; ++i)
        std::memcpy(ws->h_tab + *k_off + i * sizeof(vtx::SampleKernel), &d[i].K, sizeof(vtx::SampleKernel));
    std::memcpy(ws->h_tab + *s_off, starts.data(), starts.size() * sizeof(uint32_t));
    VTX_HIP(hipMemcpyAsync(ws->d_tab, ws->h_tab, bytes, hipMemcpyHostToDevice, ws->stream));
    VTX_HIP(hipEventRecord(ws->staged, ws->stream));
    ws->stage_busy = true;
    return VTX_OK;
}

// Queues the renders `d` on `stream`: binning and resolve into each job's
// depth/id when `bin`, the deferred pass into its rgba when `shade`.  One
// render launches with its job in the kernel arguments; several launch each
// kernel once over all of them, from device tables.  Caller holds g_mu.
//
// `own`: a workspace of the caller's (a batch graph's private one) instead of
// the stream's.  `capture`: the launches are being captured into a graph:
// nothing may allocate, copy or wait, so the scratch must already be sized and
// the device job tables already hold these jobs (a first, eager call on the
// same workspace does both); timing events are left out.
int render_locked(std::vector<JobDesc>& d, bool bin, bool shade, hipStream_t stream, Workspace* own = nullptr,
                  bool capture = false) {
    Workspace* ws = own;
    int rc = VTX_OK;
    if (!ws && (rc = get_workspace(stream, &ws))) return rc;
    if (!capture) harvest(ws);
    const size_t n = d.size();
    if (n == 0) return VTX_OK;
    // one resolve launch per tile size: keep the jobs of a size together
    if (n > 1) std::stable_sort(d.begin(), d.end(), [](const JobDesc& a, const JobDesc& b) { return a.F.tile < b.F.tile; });
    bool timing = false, scene = false, count = false;
    for (const JobDesc& j : d) {
        timing |= (j.F.flags & VTX_FLAG_TIMING) != 0;
        count |= (j.F.flags & (VTX_FLAG_STATS | VTX_FLAG_COUNT)) != 0;
        scene |= j.scene;
    }
    TimingSlot* tslot = nullptr;
    if (timing && !capture && (rc = timing_slot(ws, &tslot))) return rc;
    // timed frames: each kernel's own start and stop events, filed under the
    // time category set before its launch
    ClockScope clock(tslot ? &tslot->clock : nullptr);
    auto mark = [&](int cat) -> hipError_t {
        clock.category(cat);
        return hipSuccess;
    };
    while (bin && ws->slots.size() < n) {
        Bins* b = nullptr;
        if ((rc = bins_new(&b))) return rc;
        ws->slots.push_back(b);
    }
    std::vector<vtx::Job> jobs(n);
    std::vector<uint64_t> nprims(n, 0);
    uint32_t g_cull = 0, g_bin = 0, g_shade = 0;
    int max_tiles = 0;
    std::vector<uint32_t> starts;
    // start tables: cull, bin, shade (n + 1 each), then one per tile-size group
    starts.assign(3 * (n + 1), 0);
    for (size_t i = 0; i < n; ++i) {
        vtx::Job& J = jobs[i];
        std::memset(&J, 0, sizeof(J));
        const JobDesc& s = d[i];
        J.F = s.F;
        J.pos = s.pos;
        J.rad = s.rad;
        J.col = s.col;
        J.bonds = s.bonds;
        J.depth = s.depth;
        J.id = s.id;
        J.rgba = s.rgba;
        J.normal = s.normal;
        J.albedo = s.albedo;
        J.ao = s.ao;
        if (s.ss > 1) {
            // rendered at full size into the slot's images, reduced afterwards
            Bins* b = ws->slots[i];
            const size_t px = (size_t)s.F.W * s.F.H;
            if (px > b->ss_cap) {
                if (capture) return fail(VTX_EINVAL, "job %zu: supersampling scratch not sized for capture", i);
                VTX_HIP(hipStreamSynchronize(stream));   // in-flight frames may still use the old images
                hipFree(b->ss_depth);
                hipFree(b->ss_id);
                hipFree(b->ss_rgba);
                b->ss_depth = nullptr;
                b->ss_id = nullptr;
                b->ss_rgba = nullptr;
                b->ss_cap = 0;
                if (hipMalloc(&b->ss_depth, px * sizeof(float)) != hipSuccess ||
                    hipMalloc(&b->ss_id, px * sizeof(uint32_t)) != hipSuccess ||
                    hipMalloc(&b->ss_rgba, px * sizeof(uint32_t)) != hipSuccess) {
                    (void)hipGetLastError();
                    return fail(VTX_ENOMEM, "cannot allocate %zu supersampled pixels", px);
                }
                b->ss_cap = px;
            }
            J.depth = b->ss_depth;
            J.id = b->ss_id;
            J.rgba = b->ss_rgba;
        }
        starts[2 * (n + 1) + i] = g_shade;
        g_shade += vtx::shade_blocks(s.F);
        if (!bin) continue;
        const int T = s.F.tiles_x * s.F.tiles_y;
        max_tiles = std::max(max_tiles, T);
        const uint64_t nprim = (uint64_t)s.F.n_atoms + s.F.n_bonds;
        nprims[i] = nprim;
        uint32_t groups, chunk, nc = 0;
        vtx::bin_grid(nprim, &groups, &chunk);
        if (s.scene) {
            // each binning workgroup takes whole clusters
            nc = s.S.atom_clusters + s.S.bond_clusters;
            const uint64_t cpw = ((uint64_t)nc + groups - 1) / groups;
            chunk = (uint32_t)((cpw ? cpw : 1) * vtx::kCluster);
        }
        Bins* b = ws->slots[i];
        if (capture && (b->dirty || !b->was_sized(nprim, s.F.W, s.F.H) || (size_t)T > b->tiles_cap ||
                        (size_t)groups * chunk > b->vis_cap || (size_t)groups * T > b->hist_cap ||
                        (nc && (size_t)nc * vtx::kDepthBuckets > b->vc_cap) ||
                        (nc && (size_t)((s.F.W + vtx::kHzCell - 1) / vtx::kHzCell) *
                                       ((s.F.H + vtx::kHzCell - 1) / vtx::kHzCell) > b->hz16_cap)))
            return fail(VTX_EINVAL, "job %zu: scratch not sized for capture", i);
        if (!ws->fixed_capacity && !b->was_sized(nprim, s.F.W, s.F.H)) {
            // a shape the tuner sized, or a scene and image size counted
            // before: size from that, without counting first
            const uint64_t seen = seen_pairs(s.scene_uid, s.F.W, s.F.H);
            if (s.tuned_capacity || seen) {
                uint64_t want = s.tuned_capacity ? s.tuned_capacity : seen + seen / 2 + 1024;
                if (want > kMaxCapacity) want = kMaxCapacity;
                if (want > b->want_capacity) b->want_capacity = want;
                b->mark_sized(nprim, s.F.W, s.F.H);
            }
        }
        if ((rc = ensure_bins(ws, b, T, nprim, groups, chunk, nc, s.F.W, s.F.H))) return rc;
        b->pending_uid = s.scene_uid;
        b->pending_w = s.F.W;
        b->pending_h = s.F.H;
        b->dirty = true;   // until the resolve that re-zeroes the tile counts is queued
        J.bb = b->bb;
        J.bb.layers = 1;
        if (s.scene) {
            J.S = s.S;
            J.S.vis_clusters = b->vis_clusters;
            // binning workgroups run front to back: keep that order in the lists
            J.bb.layers = std::min<uint32_t>(vtx::kLayers, groups);
        }
        starts[i] = g_cull;
        starts[(n + 1) + i] = g_bin;
        g_cull += s.scene ? vtx::cull_blocks(s.S) : 0u;
        g_bin += groups;
    }
    starts[n] = g_cull;
    starts[2 * (n + 1) - 1] = g_bin;
    starts[3 * (n + 1) - 1] = g_shade;
    // tile-size groups [a, b) of the sorted jobs
    std::vector<std::pair<size_t, size_t>> groups_ts;
    std::vector<size_t> groups_off;
    std::vector<uint32_t> groups_grid;
    for (size_t a = 0; a < n;) {
        size_t b = a;
        while (b < n && d[b].F.tile == d[a].F.tile) ++b;
        groups_ts.push_back({a, b});
        groups_off.push_back(starts.size());
        uint32_t acc = 0;
        for (size_t i = a; i < b; ++i) {
            starts.push_back(acc);
            acc += (uint32_t)(d[i].F.tiles_x * d[i].F.tiles_y);
        }
        starts.push_back(acc);
        groups_grid.push_back(acc);
        a = b;
    }

    size_t k_off = 0, s_off = 0;
    auto list_of = [&](size_t first, size_t count, size_t start_index) {
        const vtx::Job* dj = reinterpret_cast<const vtx::Job*>(ws->d_tab) + first;
        const vtx::SampleKernel* dk = reinterpret_cast<const vtx::SampleKernel*>(ws->d_tab + k_off) + first;
        const uint32_t* ds = reinterpret_cast<const uint32_t*>(ws->d_tab + s_off) + start_index;
        // jobs of one size (a batch of equal views): the job of a block is a
        // division rather than a search of the start table
        uint32_t per = starts[start_index + 1] - starts[start_index];
        for (size_t i = 1; per && i <= count; ++i)
            if (starts[start_index + i] - starts[start_index] != (uint32_t)i * per) per = 0;
        uint32_t no_bonds = 1;
        for (size_t i = first; i < first + count; ++i)
            if (jobs[i].S.bond_clusters || jobs[i].F.n_bonds) no_bonds = 0;
        return vtx::JobList{dj, dk, ds, (uint32_t)count, per, no_bonds};
    };
    if (n > 1 && capture) {
        // the tables must be the ones the eager call uploaded
        k_off = align_up(n * sizeof(vtx::Job), 256);
        s_off = align_up(k_off + n * sizeof(vtx::SampleKernel), 256);
        const size_t bytes = s_off + starts.size() * sizeof(uint32_t);
        bool same = ws->h_tab && bytes <= ws->tab_cap && std::memcmp(ws->h_tab, jobs.data(), n * sizeof(vtx::Job)) == 0 &&
                    std::memcmp(ws->h_tab + s_off, starts.data(), starts.size() * sizeof(uint32_t)) == 0;
        for (size_t i = 0; same && i < n; ++i)
            same = std::memcmp(ws->h_tab + k_off + i * sizeof(vtx::SampleKernel), &d[i].K, sizeof(vtx::SampleKernel)) == 0;
        if (!same) return fail(VTX_EINVAL, "job tables changed between the sizing call and the capture");
    } else if (n > 1 && (rc = upload_tables(ws, jobs, d, starts, &k_off, &s_off))) {
        return rc;
    }
    auto one = [&](uint32_t blocks) {
        vtx::OneJob o;
        o.j = jobs[0];
        o.K = d[0].K;
        o.blocks = blocks;
        return o;
    };

    if (bin) {
        uint32_t gmax = 0;
        for (uint32_t gg : groups_grid) gmax = std::max(gmax, gg);
        if (!ws->d_ovf_n) {
            if ((rc = dev_alloc_zeroed(&ws->d_ovf_n, 2, stream))) return rc;
        }
        if ((size_t)xcd_round(gmax) > ws->ovf_cap || !ws->d_ovf) {
            if ((rc = grow(&ws->d_ovf, ws->ovf_cap, (size_t)xcd_round(gmax), stream, "overflow tiles"))) return rc;
        }
    }
    VTX_HIP(mark(0));
    VTX_HIP(mark(1));
    if (bin) {
        // first frame of a new scene or image size in a slot: wait for the
        // tile counts and size its lists, so the frame does not take the
        // overflow path
        std::vector<size_t> need;
        for (size_t i = 0; i < n; ++i) {
            const Bins* b = ws->slots[i];
            if (!ws->fixed_capacity && !b->was_sized(nprims[i], d[i].F.W, d[i].F.H)) need.push_back(i);
        }
        if (!need.empty() && capture) return fail(VTX_EINVAL, "scratch not sized for capture");
        // Occlusion pre-pass (asked for by every job, resident scenes with
        // sized lists): bin and resolve the nearest clusters first, then only
        // the clusters not hidden behind that pass's depths.
        bool two_pass = scene && need.empty();
        for (size_t i = 0; i < n && two_pass; ++i)
            two_pass = d[i].scene && (d[i].F.flags & VTX_FLAG_TWO_PASS) &&
                       !(d[i].F.flags & (VTX_FLAG_STATS | VTX_FLAG_COUNT | VTX_FLAG_ONE_PASS)) &&
                       d[i].F.tile >= vtx::kHzCell;
        if (scene) {
            if (n == 1) VTX_HIP(vtx::launch_cluster_cull(one(g_cull), g_cull, stream));
            else VTX_HIP(vtx::launch_cluster_cull(list_of(0, n, 0), g_cull, stream));
        }
        for (int pass = 0; pass < (two_pass ? 2 : 1); ++pass) {
            const int phase = two_pass ? (pass == 0 ? vtx::kPhaseFront : vtx::kPhaseRest) : vtx::kPhaseAll;
            if (pass > 0) VTX_HIP(mark(1));
            if (n == 1) VTX_HIP(vtx::launch_count(one(g_bin), scene, phase, g_bin, max_tiles, stream));
            else VTX_HIP(vtx::launch_count(list_of(0, n, n + 1), scene, phase, g_bin, max_tiles, stream));
            if (!need.empty()) {
                std::vector<unsigned long long> counted(n, 0);
                for (size_t i : need)
                    VTX_HIP(hipMemcpyAsync(&counted[i], &ws->slots[i]->bb.ctr->pairs_counted,
                                           sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
                VTX_HIP(hipStreamSynchronize(stream));
                for (size_t i : need) {
                    Bins* b = ws->slots[i];
                    uint64_t want = counted[i] + counted[i] / 2 + 1024;
                    if (want > kMaxCapacity) want = kMaxCapacity;
                    if (want > b->want_capacity) b->want_capacity = want;
                    if (b->want_capacity > b->list_alloc) {
                        if ((rc = grow(&b->bb.list, b->list_alloc, (size_t)b->want_capacity, stream, "tile lists")))
                            return rc;
                    }
                    b->bb.capacity = b->want_capacity;
                    b->mark_sized(nprims[i], d[i].F.W, d[i].F.H);
                    note_pairs(d[i].scene_uid, d[i].F.W, d[i].F.H, counted[i]);
                    jobs[i].bb.list = b->bb.list;
                    jobs[i].bb.capacity = b->bb.capacity;
                }
                if (n > 1 && (rc = upload_tables(ws, jobs, d, starts, &k_off, &s_off))) return rc;
            }
            VTX_HIP(mark(2));
            if (scene) {
                if (n == 1) VTX_HIP(vtx::launch_layers(one(g_bin), g_bin, stream));
                else VTX_HIP(vtx::launch_layers(list_of(0, n, n + 1), g_bin, stream));
            }
            if (n == 1) VTX_HIP(vtx::launch_tile_offsets(one(g_bin), stream));
            else VTX_HIP(vtx::launch_tile_offsets(list_of(0, n, n + 1), stream));
            VTX_HIP(mark(3));
            if (n == 1) VTX_HIP(vtx::launch_scatter(one(g_bin), phase, g_bin, max_tiles, stream));
            else VTX_HIP(vtx::launch_scatter(list_of(0, n, n + 1), phase, g_bin, max_tiles, stream));
            VTX_HIP(mark(4));
            for (size_t g = 0; g < groups_ts.size(); ++g) {
                const size_t a = groups_ts[g].first, b = groups_ts[g].second;
                if (n == 1)
                    VTX_HIP(vtx::launch_resolve(one(groups_grid[g]), d[0].F.tile, phase, groups_grid[g], count,
                                                ws->d_ovf, ws->d_ovf_n, stream));
                else
                    VTX_HIP(vtx::launch_resolve(list_of(a, b - a, groups_off[g]), d[a].F.tile, phase, groups_grid[g],
                                                count, ws->d_ovf, ws->d_ovf_n, stream));
            }
        }
        // batches: FP64 depths of the winners the resolve marked (a single
        // render's resolve writes them itself)
        if (n > 1) VTX_HIP(vtx::launch_refine(list_of(0, n, 2 * (n + 1)), g_shade, stream));
        for (size_t i = 0; i < n; ++i) {
            ws->slots[i]->dirty = false;
            ws->slots[i]->pending_capacity = ws->slots[i]->bb.capacity;
        }
        // The scatter's first workgroup (and, with statistics on, the
        // resolve's last one) writes each render's counters into its mapped
        // pinned buffer; the host reads them once this event has completed.
        if (!capture) {
            VTX_HIP(hipEventRecord(ws->done, stream));
            ws->pending = true;
            ws->pending_n = (int)n;
        }
    } else {
        for (int k = 2; k <= 4; ++k) VTX_HIP(mark(k));
    }
    VTX_HIP(mark(5));
    if (shade) {
        bool noise = false;
        for (size_t i = 0; i < n; ++i) noise |= d[i].K.noise != 0 && d[i].K.count > 0;
        if (n == 1) VTX_HIP(vtx::launch_shade(one(g_shade), g_shade, noise, stream));
        else VTX_HIP(vtx::launch_shade(list_of(0, n, 2 * (n + 1)), g_shade, noise, stream));
        for (size_t i = 0; i < n; ++i)
            if (d[i].ss > 1)
                VTX_HIP(vtx::launch_downsample(jobs[i].depth, jobs[i].id, jobs[i].rgba, d[i].F.W / d[i].ss,
                                               d[i].F.H / d[i].ss, d[i].ss, d[i].depth, d[i].id, d[i].rgba, stream));
    }
    VTX_HIP(mark(5));
    return VTX_OK;
}

JobDesc plain_desc(const Frame& F, const vtx_options& o, const float* pos, const float* rad, const uint32_t* col,
                   const uint32_t* bonds) {
    JobDesc j;
    std::memset(&j, 0, sizeof(j));
    j.F = F;
    sample_kernel(o, &j.K);
    j.pos = pos;
    j.rad = rad;
    j.col = col;
    j.bonds = bonds;
    j.scene = false;
    j.ss = o.supersample > 1 ? o.supersample : 1;
    return j;
}

}  // namespace

extern "C" {

int vtx_gbuffer(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
                const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
                int32_t W, int32_t H, float* depth, uint32_t* id, void* stream) {
    const vtx_options o = untuned_options(resolve_options(opt));
    Frame F;
    int rc = make_frame(cam, o, W, H, n_atoms, n_bonds, &F);
    if (rc) return rc;
    if ((rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, false))) return rc;
    if (!depth || !id) return fail(VTX_EINVAL, "depth/id outputs are NULL");
    if (o.supersample > 1) return fail(VTX_EINVAL, "vtx_gbuffer does not supersample (use vtx_render)");
    std::vector<JobDesc> d{plain_desc(F, o, positions, radii, colors, bonds)};
    d[0].depth = depth;
    d[0].id = id;
    std::lock_guard<std::mutex> lk(g_mu);
    return render_locked(d, true, false, (hipStream_t)stream);
}

int vtx_shade(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
              const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt, int32_t W,
              int32_t H, const float* depth, const uint32_t* id, uint32_t* rgba, float* normal, uint32_t* albedo,
              float* ao, void* stream) {
    const vtx_options o = untuned_options(resolve_options(opt));
    Frame F;
    int rc = make_frame(cam, o, W, H, n_atoms, n_bonds, &F);
    if (rc) return rc;
    if ((rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, true))) return rc;
    if (!depth || !id || !rgba) return fail(VTX_EINVAL, "depth/id/rgba are NULL");
    if (o.supersample > 1) return fail(VTX_EINVAL, "vtx_shade does not supersample (use vtx_render)");
    std::vector<JobDesc> d{plain_desc(F, o, positions, radii, colors, bonds)};
    d[0].depth = const_cast<float*>(depth);
    d[0].id = const_cast<uint32_t*>(id);
    d[0].rgba = rgba;
    d[0].normal = normal;
    d[0].albedo = albedo;
    d[0].ao = ao;
    std::lock_guard<std::mutex> lk(g_mu);
    return render_locked(d, false, true, (hipStream_t)stream);
}

int vtx_render(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
               const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
               int32_t W, int32_t H, uint32_t* rgba, float* depth, uint32_t* id, void* stream) {
    const vtx_options o = untuned_options(resolve_options(opt));
    Frame F;
    int rc = make_frame(cam, o, W, H, n_atoms, n_bonds, &F);
    if (rc) return rc;
    if ((rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, true))) return rc;
    if (!depth || !id || !rgba) return fail(VTX_EINVAL, "rgba/depth/id outputs are NULL");
    std::vector<JobDesc> d{plain_desc(F, o, positions, radii, colors, bonds)};
    d[0].depth = depth;
    d[0].id = id;
    d[0].rgba = rgba;
    std::lock_guard<std::mutex> lk(g_mu);
    return render_locked(d, true, true, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// vtx_render_static: vtx_render with every scratch buffer carved from one
// static device array, for callers that cannot allocate.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxStaticDevices = 64;

// The array itself.  In host code `scratch` names a host-side stand-in, not
// the device memory: only the address hipGetSymbolAddress returns for it on
// a device may be handed to kernels or copies.
__device__ __align__(256) static unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
unsigned char* g_static_ptr[kMaxStaticDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int static_scratch(int* device, unsigned char** out) {
    VTX_HIP(hipGetDevice(device));
    if (*device < 0 || *device >= kMaxStaticDevices) return fail(VTX_EINVAL, "device %d out of range", *device);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[*device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(VTX_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", *device, hipGetErrorString(e));
        }
        g_static_ptr[*device] = static_cast<unsigned char*>(p);
    }
    *out = g_static_ptr[*device];
    return VTX_OK;
}

// Byte layout of one frame's binning scratch in the static array (each
// buffer 256-aligned).  The first region holds what must start at zero and
// is cleared by a fill kernel at every call: the tile counts and cursors,
// the frame counters and the overflow counters.  The tile lists take what is
// left.
struct StaticLayout {
    size_t tile_cnt, tile_fill, ctr, ovf_n, zero_end;
    size_t tile_off, vis_cnt, vis_box, vis_src, vis_rect, hist, ovf, list, fixed_end;
    uint64_t list_entries;
};

StaticLayout static_layout(int T, uint32_t groups, uint32_t chunk) {
    StaticLayout L{};
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at = align_up(at + bytes, 256);
        return o;
    };
    L.tile_cnt = take((size_t)T * sizeof(uint32_t));
    L.tile_fill = take((size_t)T * sizeof(uint32_t));
    L.ctr = take(sizeof(Counters));
    L.ovf_n = take(2 * sizeof(uint32_t));
    L.zero_end = at;
    L.tile_off = take((size_t)T * sizeof(uint64_t));
    L.vis_cnt = take((size_t)vtx::kMaxBinGroups * sizeof(uint32_t));
    L.vis_box = take((size_t)vtx::kMaxBinGroups * sizeof(uint2));
    const size_t nv = (size_t)groups * chunk;
    L.vis_src = take(nv * sizeof(uint32_t));
    L.vis_rect = take(nv * sizeof(uint2));
    L.hist = take((size_t)groups * T * sizeof(uint32_t));
    L.ovf = take(xcd_round((uint32_t)T) * sizeof(unsigned long long));
    L.list = at;
    L.fixed_end = at;
    L.list_entries = at < kStaticScratchBytes ? (kStaticScratchBytes - at) / sizeof(uint2) : 0;
    if (L.list_entries > kMaxCapacity) L.list_entries = kMaxCapacity;
    return L;
}

}  // namespace

extern "C" {

int vtx_render_static(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
                      const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
                      int32_t W, int32_t H, uint32_t* rgba, float* depth, uint32_t* id, void* stream) {
    vtx_options o = untuned_options(resolve_options(opt));
    if (o.supersample > 1) return fail(VTX_EINVAL, "vtx_render_static does not supersample (supersample %d)", o.supersample);
    o.flags &= ~(uint32_t)VTX_FLAG_TIMING;
    Frame F;
    int rc = make_frame(cam, o, W, H, n_atoms, n_bonds, &F);
    if (rc) return rc;
    if ((rc = check_inputs(positions, radii, colors, n_atoms, bonds, n_bonds, true))) return rc;
    if (!depth || !id || !rgba) return fail(VTX_EINVAL, "rgba/depth/id outputs are NULL");
    const int T = F.tiles_x * F.tiles_y;
    const uint64_t nprim = (uint64_t)F.n_atoms + F.n_bonds;
    uint32_t groups, chunk;
    vtx::bin_grid(nprim, &groups, &chunk);
    const StaticLayout L = static_layout(T, groups, chunk);
    if (L.fixed_end + 256 * sizeof(uint2) > kStaticScratchBytes)
        return fail(VTX_EOVERFLOW,
                    "vtx_render_static: %lld primitives at %dx%d need %zu bytes of binning scratch before the tile "
                    "lists; the static scratch holds %zu",
                    (long long)nprim, W, H, L.fixed_end, kStaticScratchBytes);
    int device = 0;
    unsigned char* base = nullptr;
    if ((rc = static_scratch(&device, &base))) return rc;
    const hipStream_t st = (hipStream_t)stream;

    vtx::OneJob js;
    std::memset(&js, 0, sizeof(js));
    vtx::Job& J = js.j;
    J.F = F;
    J.pos = positions;
    J.rad = radii;
    J.col = colors;
    J.bonds = bonds;
    J.depth = depth;
    J.id = id;
    J.rgba = rgba;
    sample_kernel(o, &js.K);
    BinBuffers& bb = J.bb;
    bb.tile_cnt = reinterpret_cast<uint32_t*>(base + L.tile_cnt);
    bb.tile_fill = reinterpret_cast<uint32_t*>(base + L.tile_fill);
    bb.ctr = reinterpret_cast<Counters*>(base + L.ctr);
    bb.host_ctr = nullptr;
    bb.tile_off = reinterpret_cast<uint64_t*>(base + L.tile_off);
    bb.vis_cnt = reinterpret_cast<uint32_t*>(base + L.vis_cnt);
    bb.vis_box = reinterpret_cast<uint2*>(base + L.vis_box);
    bb.vis_src = reinterpret_cast<uint32_t*>(base + L.vis_src);
    bb.vis_rect = reinterpret_cast<uint2*>(base + L.vis_rect);
    bb.hist = reinterpret_cast<uint32_t*>(base + L.hist);
    bb.list = reinterpret_cast<uint2*>(base + L.list);
    bb.capacity = L.list_entries;
    bb.groups = groups;
    bb.chunk = chunk;
    bb.layers = 1;   // the caller's primitive order: one layer, no layer tables
    unsigned long long* ovf = reinterpret_cast<unsigned long long*>(base + L.ovf);
    uint32_t* ovf_n = reinterpret_cast<uint32_t*>(base + L.ovf_n);
    // the array keeps the last call's contents: clear the counts, cursors
    // and counters this frame adds to (a fill kernel, no memset node)
    VTX_HIP(vtx::launch_zero(reinterpret_cast<uint32_t*>(base), L.zero_end / sizeof(uint32_t), st));
    const bool count = (F.flags & (VTX_FLAG_STATS | VTX_FLAG_COUNT)) != 0;
    js.blocks = groups;
    VTX_HIP(vtx::launch_count(js, false, vtx::kPhaseAll, groups, T, st));
    VTX_HIP(vtx::launch_tile_offsets(js, st));
    VTX_HIP(vtx::launch_scatter(js, vtx::kPhaseAll, groups, T, st));
    js.blocks = (uint32_t)T;
    VTX_HIP(vtx::launch_resolve(js, F.tile, vtx::kPhaseAll, (uint32_t)T, count, ovf, ovf_n, st));
    js.blocks = vtx::shade_blocks(F);
    VTX_HIP(vtx::launch_shade(js, js.blocks, js.K.noise != 0 && js.K.count > 0, st));
    return VTX_OK;
}

int vtx_ses(const float* positions, const float* radii, int64_t n_atoms, float probe_radius,
            const vtx_ses_grid* grid, float* field, float* triangles, int64_t capacity, uint64_t* n_triangles,
            void* stream) {
    if (!grid || !n_triangles) return fail(VTX_EINVAL, "grid/n_triangles is NULL");
    if (n_atoms < 0 || n_atoms > 0xFFFFFFFFll) return fail(VTX_EINVAL, "n_atoms=%lld out of range", (long long)n_atoms);
    if (n_atoms > 0 && (!positions || !radii)) return fail(VTX_EINVAL, "positions/radii are NULL");
    if (!(probe_radius >= 0.0f) || !std::isfinite(probe_radius)) return fail(VTX_EINVAL, "probe_radius must be >= 0");
    if (!(grid->spacing > 0.0f) || !std::isfinite(grid->spacing) || !finite3(grid->origin))
        return fail(VTX_EINVAL, "grid spacing must be > 0 and the origin finite");
    int64_t np = 1;
    for (int d = 0; d < 3; ++d) {
        if (grid->dims[d] < 2) return fail(VTX_EINVAL, "grid dims must be >= 2");
        np *= grid->dims[d];
    }
    if (np >= ((int64_t)1 << 31)) return fail(VTX_EINVAL, "grid of %lld points is too large", (long long)np);
    if (capacity < 0 || (capacity > 0 && !triangles)) return fail(VTX_EINVAL, "triangles is NULL or capacity < 0");
    if ((double)probe_radius / (double)grid->spacing > 1e6) return fail(VTX_EINVAL, "probe_radius / spacing too large");
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace* ws = nullptr;
    const hipStream_t st = (hipStream_t)stream;
    int rc = get_workspace(st, &ws);
    if (rc) return rc;
    const int dims[3] = {grid->dims[0], grid->dims[1], grid->dims[2]};
    size_t wm, wg, wc, wb;
    size_t words = vtx::ses_scratch_words(dims, &wm, &wg, &wc, &wb);
    const size_t wf = field ? 0 : (size_t)np;
    words += wf + 64;
    if ((rc = grow(&ws->ses, ws->ses_cap, words, st, "surface scratch"))) return rc;
    vtx::SesScratch sc;
    uint32_t* at = ws->ses;
    sc.mark = reinterpret_cast<uint8_t*>(at);
    at += wm;
    sc.ga = reinterpret_cast<int32_t*>(at);
    at += wg;
    sc.gb = reinterpret_cast<int32_t*>(at);
    at += wg;
    sc.cnt = at;
    at += wc;
    sc.bsum = at;
    at += wb;
    float* f = field ? field : reinterpret_cast<float*>(at);
    VTX_HIP(vtx::ses_run(positions, radii, (uint64_t)n_atoms, probe_radius, grid->origin, grid->spacing, dims, f,
                         triangles, (uint64_t)capacity, reinterpret_cast<unsigned long long*>(n_triangles), sc, st));
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

size_t vtx_scene_frame_bytes(int64_t n_atoms, int64_t n_bonds) {
    if (n_atoms < 0 || n_bonds < 0) return 0;
    return frame_bytes(n_atoms, n_bonds);
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
    // tile counts and offsets, per-layer cursors, starts and totals, visible lists,
    // histograms, lists, visible clusters per depth class, cell depths, counters
    return (size_t)(T * 16 + T * 12 * vtx::kLayers + (uint64_t)groups * chunk * (sizeof(uint32_t) + sizeof(uint2)) +
                    (uint64_t)groups * T * 4 + cap * sizeof(uint2) +
                    scene_clusters(n_atoms, n_bonds) * 4 * vtx::kDepthBuckets +
                    (uint64_t)((W + vtx::kHzCell - 1) / vtx::kHzCell) * ((H + vtx::kHzCell - 1) / vtx::kHzCell) * 4 +
                    sizeof(Counters) + 4096);
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
    {
        std::lock_guard<std::mutex> lk(g_mu);
        sc->uid = g_next_scene_uid++;
    }
    sc->device = dev;
    sc->n = n_atoms;
    sc->m = n_bonds;
    sc->bytes = bytes;
    const size_t na = (size_t)n_atoms, nb = (size_t)n_bonds;
    const size_t ncl = scene_clusters(n_atoms, n_bonds);
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
        (rc = dev_alloc(&sc->pos, 3 * na, "positions")) || (rc = dev_alloc(&sc->rad, na, "radii")) ||
        (rc = dev_alloc(&sc->col, na, "colours")) || (rc = dev_alloc(&sc->bonds, 2 * nb, "bonds")))
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
    sc->S.vis_clusters = nullptr;   // per render, in the stream's scratch
    uint32_t box_bits[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
    hipError_t e = vtx::scene_build(sc->pos, sc->rad, sc->bonds, na, nb, sc->S, sc->xyzr, sc->atom_id, sc->bond_rec,
                                    sc->cluster_box, tmp, tmp_bytes, &m_valid, &n_bad, box_bits, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(VTX_EHIP, "building the scene failed: %s", hipGetErrorString(e)));
    if (na > 0) {
        auto from_ordered = [](uint32_t u) {
            const uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
            float f;
            std::memcpy(&f, &b, sizeof f);
            return (double)f;
        };
        for (int k = 0; k < 3; ++k) {
            sc->box_lo[k] = from_ordered(box_bits[k]);
            sc->box_hi[k] = from_ordered(box_bits[3 + k]);
        }
        sc->have_box = std::isfinite(sc->box_lo[0] + sc->box_lo[1] + sc->box_lo[2] + sc->box_hi[0] + sc->box_hi[1] +
                                     sc->box_hi[2]);
    }
    hipFree(tmp);
    sc->bad_bonds = n_bad;
    *out = sc;
    return VTX_OK;
}

int vtx_scene_add_frames(vtx_scene* scene, const float* positions, int32_t n_frames, void* stream,
                         int32_t* first_frame) {
    if (!scene) return fail(VTX_EINVAL, "scene is NULL");
    if (n_frames < 1) return fail(VTX_EINVAL, "n_frames must be >= 1");
    if (scene->n > 0 && !positions) return fail(VTX_EINVAL, "positions are NULL");
    if ((int64_t)scene->frames.size() + n_frames > 1000000) return fail(VTX_EINVAL, "too many frames");
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    if (dev != scene->device) return fail(VTX_EINVAL, "scene lives on device %d, current is %d", scene->device, dev);
    const size_t na = (size_t)scene->n, nc = scene_clusters(scene->n, scene->m);
    const size_t pos_b = align_up(na * 3 * sizeof(float), 256), xyzr_b = align_up(na * sizeof(float4), 256),
                 box_b = align_up(nc * 2 * sizeof(float4), 256);
    const size_t bytes = (size_t)n_frames * frame_bytes(scene->n, scene->m);
    vtx_context* ctx = scene->ctx;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->budget && ctx->used + bytes > ctx->budget)
            return fail(VTX_EBUSY, "%d frames of %zu bytes exceed the context budget (%zu of %zu in use)", n_frames,
                        bytes, ctx->used, ctx->budget);
        ctx->used += bytes;
    }
    char* block = nullptr;
    const size_t per = pos_b + xyzr_b + box_b;
    if (hipMalloc(&block, per * (size_t)n_frames) != hipSuccess) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->used -= bytes;
        return fail(VTX_ENOMEM, "cannot allocate %zu bytes for %d frames", per * (size_t)n_frames, n_frames);
    }
    hipStream_t st = (hipStream_t)stream;
    const int32_t first = (int32_t)scene->frames.size() + 1;
    for (int32_t f = 0; f < n_frames; ++f) {
        SceneFrame fr;
        char* base = block + per * (size_t)f;
        fr.pos = reinterpret_cast<float*>(base);
        fr.xyzr = reinterpret_cast<float4*>(base + pos_b);
        fr.cluster_box = reinterpret_cast<float4*>(base + pos_b + xyzr_b);
        hipError_t e = hipSuccess;
        if (na) e = hipMemcpyAsync(fr.pos, positions + (size_t)f * na * 3, na * 3 * sizeof(float), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = vtx::scene_update_positions(fr.pos, scene->S, fr.xyzr, fr.cluster_box, st);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);
            hipFree(block);
            scene->frames.resize((size_t)first - 1);
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->used -= bytes;
            return fail(VTX_EHIP, "storing frame %d failed: %s", f, hipGetErrorString(e));
        }
        scene->frames.push_back(fr);
    }
    scene->frame_blocks.push_back(block);
    scene->bytes += bytes;
    if (first_frame) *first_frame = first;
    return VTX_OK;
}

int32_t vtx_scene_frames(const vtx_scene* scene) { return scene ? (int32_t)scene->frames.size() + 1 : 0; }

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

int vtx_scene_order(const vtx_scene* scene, uint32_t* atom_order, uint32_t* bond_order, void* stream) {
    if (!scene) return fail(VTX_EINVAL, "scene is NULL");
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    if (dev != scene->device) return fail(VTX_EINVAL, "scene lives on device %d, current is %d", scene->device, dev);
    VTX_HIP(vtx::scene_order(scene->S, atom_order, bond_order, (hipStream_t)stream));
    return VTX_OK;
}

void vtx_scene_destroy(vtx_scene* scene) {
    if (!scene) return;
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_pairs_seen.erase(scene->uid);
    }
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
    uint64_t tuned_cap = 0;
    const vtx_options o = tuned_options(scene->ctx, resolve_options(opt), cam, W, H, scene->n, scene->m, &tuned_cap);
    Frame F;
    int rc = make_frame(cam, o, W, H, scene->n, scene->m, &F);
    if (rc) return rc;
    scene_depth_classes(scene, &F);
    if (!depth || !id || !rgba) return fail(VTX_EINVAL, "rgba/depth/id outputs are NULL");
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    if (dev != scene->device) return fail(VTX_EINVAL, "scene lives on device %d, current is %d", scene->device, dev);
    std::vector<JobDesc> d{plain_desc(F, o, scene->pos, scene->rad, scene->col, scene->bonds)};
    d[0].scene = true;
    d[0].scene_uid = scene->uid;
    d[0].tuned_capacity = tuned_cap;
    d[0].S = scene->S;
    d[0].depth = depth;
    d[0].id = id;
    d[0].rgba = rgba;
    std::lock_guard<std::mutex> lk(g_mu);
    return render_locked(d, true, true, (hipStream_t)stream);
}

int vtx_check_job(const vtx_context* ctx, const vtx_job* j) {
    if (!j) return fail(VTX_EINVAL, "job is NULL");
    const vtx_scene* sc = j->scene;
    if (!sc) return fail(VTX_EINVAL, "scene is NULL");
    if (ctx && sc->ctx != ctx) return fail(VTX_EINVAL, "scene belongs to another context");
    if (j->frame < 0 || j->frame > (int32_t)sc->frames.size())
        return fail(VTX_EINVAL, "frame %d not in 0..%zu", j->frame, sc->frames.size());
    if (!j->rgba || !j->depth || !j->id) return fail(VTX_EINVAL, "rgba/depth/id outputs are NULL");
    const vtx_options o = untuned_options(resolve_options(&j->options));
    Frame F;
    return make_frame(&j->camera, o, j->width, j->height, sc->n, sc->m, &F);
}

}  // extern "C"

namespace {

// Checks a batch and builds its render descriptions.
int build_batch(vtx_context* ctx, const vtx_job* jobs, int32_t n_jobs, std::vector<JobDesc>& d) {
    if (!ctx) return fail(VTX_EINVAL, "context is NULL");
    if (n_jobs < 0 || n_jobs > kMaxBatch) return fail(VTX_EINVAL, "n_jobs=%d not in 0..%d", n_jobs, kMaxBatch);
    if (n_jobs > 0 && !jobs) return fail(VTX_EINVAL, "jobs is NULL");
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    if (dev != ctx->device) return fail(VTX_EINVAL, "current device %d is not the context's %d", dev, ctx->device);
    d.resize((size_t)n_jobs);
    for (int32_t i = 0; i < n_jobs; ++i) {
        const vtx_job& j = jobs[i];
        const vtx_scene* sc = j.scene;
        if (!sc) return fail(VTX_EINVAL, "job %d: scene is NULL", i);
        if (sc->ctx != ctx) return fail(VTX_EINVAL, "job %d: scene belongs to another context", i);
        if (j.frame < 0 || j.frame > (int32_t)sc->frames.size())
            return fail(VTX_EINVAL, "job %d: frame %d not in 0..%zu", i, j.frame, sc->frames.size());
        if (!j.rgba || !j.depth || !j.id) return fail(VTX_EINVAL, "job %d: rgba/depth/id outputs are NULL", i);
        uint64_t tuned_cap = 0;
        const vtx_options o =
            tuned_options(ctx, resolve_options(&j.options), &j.camera, j.width, j.height, sc->n, sc->m, &tuned_cap);
        Frame F;
        int rc = make_frame(&j.camera, o, j.width, j.height, sc->n, sc->m, &F);
        if (rc) return fail(rc, "job %d: %s", i, g_error.c_str());
        scene_depth_classes(sc, &F);
        vtx::SceneDev S;
        const float* pos = nullptr;
        scene_frame(sc, j.frame, &S, &pos);
        d[(size_t)i] = plain_desc(F, o, pos, sc->rad, sc->col, sc->bonds);
        d[(size_t)i].scene = true;
        d[(size_t)i].scene_uid = sc->uid;
        d[(size_t)i].tuned_capacity = tuned_cap;
        d[(size_t)i].S = S;
        d[(size_t)i].depth = j.depth;
        d[(size_t)i].id = j.id;
        d[(size_t)i].rgba = j.rgba;
    }
    return VTX_OK;
}

}  // namespace

struct vtx_batch_graph {
    vtx_context* ctx = nullptr;
    int device = 0;
    hipStream_t cap = nullptr;       // private stream the batch was sized on and captured from
    Workspace* ws = nullptr;         // private scratch the graph's kernels use
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int vtx_render_batch(vtx_context* ctx, const vtx_job* jobs, int32_t n_jobs, void* stream) {
    std::vector<JobDesc> d;
    int rc = build_batch(ctx, jobs, n_jobs, d);
    if (rc) return rc;
    if (d.empty()) return VTX_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    return render_locked(d, true, true, (hipStream_t)stream);
}

void vtx_batch_graph_destroy(vtx_batch_graph* g) {
    if (!g) return;
    if (g->cap) (void)hipStreamSynchronize(g->cap);
    (void)hipDeviceSynchronize();   // replays on other streams may still run
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->ws) workspace_free(g->ws);
    if (g->cap) hipStreamDestroy(g->cap);
    delete g;
}

int vtx_batch_graph_create(vtx_context* ctx, const vtx_job* jobs, int32_t n_jobs, vtx_batch_graph** out) {
    if (!out) return fail(VTX_EINVAL, "out is NULL");
    std::vector<JobDesc> d;
    int rc = build_batch(ctx, jobs, n_jobs, d);
    if (rc) return rc;
    if (d.empty()) return fail(VTX_EINVAL, "a batch graph needs at least one job");
    for (JobDesc& j : d) j.F.flags &= ~VTX_FLAG_TIMING;
    vtx_batch_graph* g = new vtx_batch_graph();
    g->ctx = ctx;
    VTX_HIP(hipGetDevice(&g->device));
    if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        return fail(VTX_EHIP, "cannot create the capture stream");
    }
    g->ws = new Workspace();
    g->ws->device = g->device;
    g->ws->stream = g->cap;
    if (hipEventCreateWithFlags(&g->ws->done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ws->staged, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        vtx_batch_graph_destroy(g);
        return fail(VTX_EHIP, "cannot create events");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        // an eager run sizes the private scratch and uploads the job tables
        std::vector<JobDesc> d0 = d;
        rc = render_locked(d0, true, true, g->cap, g->ws, false);
        if (rc == VTX_OK && hipStreamSynchronize(g->cap) != hipSuccess) rc = fail(VTX_EHIP, "sizing run failed");
        if (rc == VTX_OK) {
            if (hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                (void)hipGetLastError();
                rc = fail(VTX_EHIP, "hipStreamBeginCapture failed");
            } else {
                std::vector<JobDesc> d1 = d;
                rc = render_locked(d1, true, true, g->cap, g->ws, true);
                hipGraph_t graph = nullptr;
                const hipError_t e = hipStreamEndCapture(g->cap, &graph);
                g->graph = graph;
                if (rc == VTX_OK && e != hipSuccess) rc = fail(VTX_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            }
        }
    }
    if (rc == VTX_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(VTX_EHIP, "hipGraphInstantiate failed");
    }
    if (rc != VTX_OK) {
        vtx_batch_graph_destroy(g);
        return rc;
    }
    *out = g;
    return VTX_OK;
}

int vtx_batch_graph_launch(vtx_batch_graph* g, void* stream) {
    if (!g || !g->exec) return fail(VTX_EINVAL, "graph is NULL");
    int dev = 0;
    VTX_HIP(hipGetDevice(&dev));
    if (dev != g->device) return fail(VTX_EINVAL, "graph lives on device %d, current is %d", g->device, dev);
    VTX_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return VTX_OK;
}

int vtx_autotune(vtx_context* ctx, const vtx_job* jobs, int32_t n_jobs, const char* cache_path, void* stream,
                 vtx_tuning* out) {
    if (!ctx) return fail(VTX_EINVAL, "context is NULL");
    if (n_jobs < 1 || n_jobs > kMaxBatch || !jobs) return fail(VTX_EINVAL, "need 1..%d sample jobs", kMaxBatch);
    const float budget = out ? out->frame_budget_ms : 0.0f;
    // the shapes of the sample jobs; the batch is timed as a whole and its
    // choices kept for each of them
    std::vector<std::string> keys, job_key;
    bool want_ssao = false;
    for (int32_t i = 0; i < n_jobs; ++i) {
        if (!jobs[i].scene) return fail(VTX_EINVAL, "job %d: scene is NULL", i);
        const std::string k =
            shape_key(jobs[i].width, jobs[i].height, jobs[i].scene->n, jobs[i].scene->m, jobs[i].camera.projection);
        job_key.push_back(k);
        if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
        want_ssao = want_ssao || jobs[i].options.ssao_samples == VTX_SSAO_AUTO;
    }
    const std::string key = keys[0];
    std::map<std::string, TunedShape> cached;
    vtx_tuning t;
    std::memset(&t, 0, sizeof(t));
    std::snprintf(t.key, sizeof(t.key), "%s", key.c_str());
    t.frame_budget_ms = budget;
    t.ssao_samples = -1;
    // cached choices: one line per shape
    //   {"key": K, "tile_size": T, "ssao_samples": S, "bin_capacity": C, "ms_per_batch": M}
    std::vector<std::pair<std::string, std::string>> lines;   // key -> its cache line
    if (cache_path && *cache_path) {
        if (FILE* fh = std::fopen(cache_path, "r")) {
            char buf[512];
            while (std::fgets(buf, sizeof(buf), fh)) {
                char k[160];
                int tile = 0, ssao = -1;
                unsigned long long cap = 0;
                if (std::sscanf(buf, " {\"key\": \"%159[^\"]\", \"tile_size\": %d, \"ssao_samples\": %d, \"bin_capacity\": %llu",
                                k, &tile, &ssao, &cap) >= 2) {
                    std::string line(buf);
                    while (!line.empty() && (line.back() == '\n' || line.back() == ',' || line.back() == ' '))
                        line.pop_back();
                    lines.push_back({k, line});
                    if (tile == 8 || tile == 16 || tile == 32 || tile == 64) {
                        TunedShape ts;
                        ts.tile = tile;
                        ts.ssao = ssao >= 0 && ssao <= VTX_MAX_SSAO_SAMPLES ? ssao : -1;
                        ts.capacity = cap <= kMaxCapacity ? (uint64_t)cap : 0;
                        cached[k] = ts;
                    }
                }
            }
            std::fclose(fh);
        }
    }
    bool all_cached = true;
    for (const std::string& k : keys)
        all_cached = all_cached && cached.count(k) && cached[k].capacity && (!want_ssao || cached[k].ssao >= 0);
    if (all_cached) {
        t.from_cache = 1;
        t.tile_size = cached[key].tile;
        t.ssao_samples = want_ssao ? cached[key].ssao : -1;
        t.bin_capacity = cached[key].capacity;
    } else {
        hipStream_t st = (hipStream_t)stream;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        VTX_HIP(hipEventCreate(&e0));
        VTX_HIP(hipEventCreate(&e1));
        std::vector<vtx_job> trial(jobs, jobs + n_jobs);
        for (vtx_job& j : trial) {
            j.options.flags = 0;
            if (j.options.ssao_samples == VTX_SSAO_AUTO) j.options.ssao_samples = kAutoSsaoDefault;
        }
        // device time of one sample batch (the first run sizes the bins and
        // is not timed)
        auto time_batch = [&](float* ms_out) -> int {
            int rc = VTX_OK;
            for (int rep = 0; rep < 4 && rc == VTX_OK; ++rep) {
                if (rep == 1) rc = hipEventRecord(e0, st) == hipSuccess ? VTX_OK : fail(VTX_EHIP, "hipEventRecord failed");
                if (rc == VTX_OK) rc = vtx_render_batch(ctx, trial.data(), n_jobs, stream);
            }
            float ms = 0.0f;
            if (rc == VTX_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(VTX_EHIP, "timing the sample batch failed");
            *ms_out = ms / 3.0f;
            return rc;
        };
        // 1. tile size: every size all the sample images accept
        const int sizes[4] = {8, 16, 32, 64};
        float best = 0.0f;
        int rc = VTX_OK;
        for (int k = 0; k < 4 && rc == VTX_OK; ++k) {
            bool ok = true;
            for (const vtx_job& j : trial)
                ok = ok && (int64_t)((j.width + sizes[k] - 1) / sizes[k]) * ((j.height + sizes[k] - 1) / sizes[k]) <=
                               vtx::kMaxLdsTiles;
            if (!ok) continue;
            for (vtx_job& j : trial) j.options.tile_size = sizes[k];
            float ms = 0.0f;
            if ((rc = time_batch(&ms)) != VTX_OK) break;
            t.ms_by_tile[k] = ms;
            if (!t.tile_size || ms < best) {
                best = ms;
                t.tile_size = sizes[k];
            }
        }
        if (rc == VTX_OK && !t.tile_size) rc = fail(VTX_EINVAL, "no tile size fits the sample images");
        if (rc == VTX_OK) {
            t.ms_per_batch = best;
            for (vtx_job& j : trial) j.options.tile_size = t.tile_size;
        }
        // 2. bin capacity: the pairs of each sample job at that size
        std::map<std::string, uint64_t> cap;
        if (rc == VTX_OK) rc = vtx_render_batch(ctx, trial.data(), n_jobs, stream);
        if (rc == VTX_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(VTX_EHIP, "hipStreamSynchronize failed");
        if (rc == VTX_OK) {
            std::lock_guard<std::mutex> lk(g_mu);
            int dev = 0;
            (void)hipGetDevice(&dev);
            auto it = g_ws.find(std::make_pair(dev, st));
            if (it == g_ws.end() || (int)it->second->slots.size() < n_jobs) {
                rc = fail(VTX_EINVAL, "no scratch for the sample batch");
            } else {
                for (int32_t i = 0; i < n_jobs; ++i) {
                    const uint64_t pairs = it->second->slots[(size_t)i]->host_ctr->pairs;
                    uint64_t c = pairs + pairs / 4 + 1024;
                    if (c > kMaxCapacity) c = kMaxCapacity;
                    cap[job_key[(size_t)i]] = std::max(cap[job_key[(size_t)i]], c);
                }
            }
        }
        // 3. SSAO samples of the jobs that leave them to the context
        int ssao = -1;
        if (rc == VTX_OK && want_ssao) {
            static const int counts[9] = {64, 48, 32, 24, 16, 12, 8, 4, 0};
            ssao = kAutoSsaoDefault;
            if (budget > 0.0f) {
                ssao = -1;
                for (int c = 0; c < 9 && rc == VTX_OK && ssao < 0; ++c) {
                    for (int32_t i = 0; i < n_jobs; ++i)
                        if (jobs[i].options.ssao_samples == VTX_SSAO_AUTO) trial[(size_t)i].options.ssao_samples = counts[c];
                    float ms = 0.0f;
                    if ((rc = time_batch(&ms)) != VTX_OK) break;
                    t.ms_by_samples[c] = ms / (float)n_jobs;
                    if (t.ms_by_samples[c] <= budget) ssao = counts[c];
                }
                if (rc == VTX_OK && ssao < 0) ssao = 0;   // the budget is below even no occlusion: the cheapest
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (rc != VTX_OK) return rc;
        t.ssao_samples = ssao;
        t.bin_capacity = cap[key];
        for (const std::string& k : keys) {
            TunedShape ts;
            ts.tile = t.tile_size;
            ts.ssao = ssao >= 0 ? ssao : (cached.count(k) ? cached[k].ssao : -1);
            ts.capacity = cap[k];
            cached[k] = ts;
        }
        if (cache_path && *cache_path) {
            for (const std::string& k : keys) {
                char line[320];
                std::snprintf(line, sizeof(line),
                              "  {\"key\": \"%s\", \"tile_size\": %d, \"ssao_samples\": %d, \"bin_capacity\": %llu, "
                              "\"ms_per_batch\": %.6f}",
                              k.c_str(), cached[k].tile, cached[k].ssao, (unsigned long long)cached[k].capacity,
                              (double)best);
                bool replaced = false;
                for (auto& l : lines)
                    if (l.first == k) {
                        l.second = line;
                        replaced = true;
                    }
                if (!replaced) lines.push_back({k, line});
            }
            FILE* fh = std::fopen(cache_path, "w");
            if (!fh) return fail(VTX_EINVAL, "cannot write the tuning cache %s", cache_path);
            std::fprintf(fh, "{\"vtx_tuning\": [\n");
            for (size_t i = 0; i < lines.size(); ++i)
                std::fprintf(fh, "%s%s\n", lines[i].second.c_str(), i + 1 < lines.size() ? "," : "");
            std::fprintf(fh, "]}\n");
            std::fclose(fh);
        }
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (const std::string& k : keys) ctx->tuned[k] = cached[k];
    }
    if (out) *out = t;
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
    ws->fixed_entries = entries;
    for (Bins* b : ws->slots) {
        b->want_capacity = entries;   // 0: re-derived from the next frame's size
        b->sized.clear();
    }
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
    workspace_free(ws);
    g_ws.erase(it);
    return VTX_OK;
}

const char* vtx_last_error(void) { return g_error.c_str(); }

const char* vtx_version(void) { return "vtx-mi355x 0.2.0 (gfx950)"; }

}  // extern "C"
