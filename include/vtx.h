/*
 * vtx.h - C ABI of the MI355X impostor renderer for massive molecular scenes.
 *
 * The renderer draws the "meshless" representations of VTX (Maria et al.,
 * "VTX: Real-time high-performance molecular structure and dynamics
 * visualization software", Bioinformatics 2025): a molecule is the positions
 * of its atoms, their radii and their connectivity (Methods, "Molecular
 * Graphics Engine"); atoms are spheres and bonds are cylinders, each
 * displayed by ray-casting its implicit surface, which gives pixel-exact
 * images (same section, "Meshless Representations"); a deferred pass then
 * applies screen-space ambient occlusion and shading over the G-buffer
 * (Methods, "High Quality Rendering").
 *
 * Conventions shared by every entry point
 *  - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensor
 *    storage) on the current HIP device.  The caller owns them; the library
 *    never frees or keeps them beyond the call's stream work.
 *  - Work is queued on `stream` (a hipStream_t; NULL = the null stream) and
 *    the call returns without waiting for it, except where stated.
 *  - Return value: VTX_OK (0) or a negative VTX_E* code; vtx_last_error()
 *    then gives a message (per host thread).  On an error nothing has been
 *    queued and the outputs are unchanged.
 *  - Images are row-major, W x H, row 0 is the TOP row, column 0 the left.
 *  - View space: x right, y up, z forward (away from the eye).  Depth is the
 *    view z of the surface point in the length unit of the positions
 *    (angstrom), +inf where no primitive is hit.
 *  - Primitive ids: atom i has id i, bond b has id n_atoms + b; background
 *    is VTX_BACKGROUND_ID.  The visible primitive at a pixel is the one with
 *    the smallest (depth, id), so equal depths go to the smaller id.
 *  - Colours are RGBA8 packed in a uint32, R in the low byte.
 *  - Per-stream scratch memory (tile bins) is owned by the library, grows on
 *    demand and is released by vtx_release_scratch().  Calls queued on the
 *    same stream are ordered; calls on different streams use separate
 *    scratch and may overlap.
 */
#ifndef VTX_H
#define VTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VTX_OK 0
#define VTX_EINVAL (-1)     /* invalid argument */
#define VTX_ENOMEM (-2)     /* device or pinned allocation failed */
#define VTX_EHIP (-3)       /* a HIP runtime call failed */
#define VTX_EOVERFLOW (-4)  /* a size exceeds what the library supports */
#define VTX_EBUSY (-5)      /* admission refused (budget or slots exhausted) */

#define VTX_PERSPECTIVE 0
#define VTX_ORTHOGRAPHIC 1

#define VTX_BACKGROUND_ID 0xFFFFFFFFu
#define VTX_MAX_PIXELS (7680 * 4320)   /* 8K, the paper's largest export size */
#define VTX_MAX_SIDE 16383             /* pixels on either side of a rendered frame */
#define VTX_MAX_SSAO_SAMPLES 64

/* options.flags */
#define VTX_FLAG_STATS 1u        /* count every (primitive, pixel) hit exactly;
                                    disables the depth early-outs */
#define VTX_FLAG_TIMING 2u       /* each kernel of the frame is dispatched with a start
                                    and a stop event of its own (its dispatch's begin
                                    and end), read back by vtx_read_timings */
#define VTX_FLAG_TWO_PASS 8u     /* resident scenes: occlusion pre-pass.  The nearest
                                    eighth of the visible clusters (by depth; rounded
                                    up to the end of its depth class unless that
                                    would pass half of them) is binned and
                                    resolved first; of the rest, only
                                    clusters whose bounding sphere is not behind the
                                    depths of every 16x16-pixel cell under it are
                                    binned, and resolved on top.  The image is the
                                    same as without it.  It pays when near surfaces
                                    close whole cells (a dense slab in front of a
                                    deep scene bins ~10x fewer primitives) and costs
                                    a second binning pass when they do not (sparse
                                    scenes whose cells keep a gap).  Ignored with
                                    VTX_FLAG_STATS, VTX_FLAG_COUNT or
                                    VTX_FLAG_ONE_PASS, with 8-pixel
                                    tiles, for jobs in a batch whose other jobs do
                                    not all set it, and on the first frame of a new
                                    scene or image size in a render slot */
#define VTX_FLAG_ONE_PASS 4u     /* resident scenes: never take the pre-pass */
#define VTX_FLAG_COUNT 16u       /* count the ray tests the frame runs with its depth
                                    early-outs on, and how often each early-out fires
                                    (vtx_stats); the image is the same, the resolve is
                                    the slower counting one; no pre-pass */

/*
 * Camera (paper, "Improved user experience": trackball and free-fly cameras
 * both reduce to a pose and a projection).  The view basis is
 * f = normalize(target - eye), s = normalize(f x up), u = s x f.  Pixel
 * (i, j) has the normalized device coordinates
 * (2 (i + 1/2) / W - 1, 1 - 2 (j + 1/2) / H); a perspective ray leaves the eye
 * through that point of the image plane at tan(fovy/2) (times W/H in x); an
 * orthographic ray is parallel to f from the point eye + ndc_x h (W/H) s +
 * ndc_y h u.  Only surface points with znear <= depth <= zfar are drawn.
 */
typedef struct vtx_camera {
    float eye[3];
    float target[3];
    float up[3];
    float fovy;               /* radians, vertical field of view (perspective) */
    float ortho_half_height;  /* h: half height of the view volume (orthographic) */
    int32_t projection;       /* VTX_PERSPECTIVE or VTX_ORTHOGRAPHIC */
    float znear;              /* > 0 */
    float zfar;               /* > znear */
} vtx_camera;

/*
 * Rendering options (paper, "High Quality Rendering": deferred shading with
 * ambient occlusion computed every frame, custom background with
 * transparency).  Pass NULL for the defaults shown.
 */
typedef struct vtx_options {
    float bond_radius;        /* cylinder radius of every bond (0.15) */
    int32_t ssao_samples;     /* K hemisphere samples, 0 = no ambient occlusion (0);
                                 VTX_SSAO_AUTO: the context's choice (see vtx_autotune) */
    float ssao_radius;        /* hemisphere radius (2.0) */
    float ssao_bias;          /* depth bias of the occlusion test (0.05) */
    uint32_t background;      /* RGBA8 of pixels hit by nothing (0 = transparent black) */
    int32_t tile_size;        /* screen tile edge in pixels: 0 (default 16), 8, 16, 32 or 64;
                                 raised to the next of these while the image has
                                 more than 15360 tiles (VTX_EINVAL if 64 is not
                                 enough: extreme aspect ratios) */
    uint32_t flags;           /* VTX_FLAG_* */
    int32_t representation;   /* VTX_REP_* (VTX_REP_BALL_AND_STICK) */
    float probe_radius;       /* solvent probe of VTX_REP_SAS (1.4) */
    /* deferred post-passes (see below) */
    int32_t shading;          /* VTX_SHADE_* (VTX_SHADE_GLOSSY) */
    uint32_t fog_color;       /* RGBA8 the fog fades to (alpha ignored) */
    float fog_start, fog_end; /* view depths (A) where fog begins and is complete;
                                 fog_end <= fog_start: no fog (0, 0) */
    uint32_t outline_color;   /* RGBA8 of outline pixels (alpha ignored) */
    float outline_depth;      /* relative depth step that makes an outline; 0: none (0) */
    float clip_plane[4];      /* world plane a, b, c, d; a x + b y + c z + d >= 0 is kept;
                                 all zero: no clipping (0, 0, 0, 0) */
    int32_t supersample;      /* S = 1..4 samples per pixel side (0 or 1: none) */
    int32_t ssao_noise;       /* 1: the noise form of the ambient occlusion (see below); 0: none (0) */
} vtx_options;

/*
 * options.ssao_noise (paper, Methods, "High Quality Rendering": screen-space
 * ambient occlusion after Mittring 2007, whose samples are turned per pixel
 * by a tiled noise and the result blurred).  The reading here keeps it
 * deterministic: pixel (x, y) turns its tangent frame about its normal by
 * 2 pi (B[y mod 4][x mod 4] + 1/2) / 16, B the 4x4 ordered-dither (Bayer)
 * matrix, so the 16 pixels of each 4x4 block sample 16 directions; the AO
 * of a hit pixel is then the mean of those values over the hit pixels
 * (x + dx, y + dy), dx, dy in {-2, -1, 0, 1}, inside the image.
 */

/*
 * options.supersample (paper, Methods, "High Quality Rendering": anti-aliasing
 * is one of the deferred post-processes; the reading here is exact
 * supersampling, so that the result stays defined pixel by pixel): the frame
 * is rendered and shaded at (S W) x (S H) in library scratch, with every
 * other option unchanged; output pixel (i, j) then takes, per RGBA channel,
 * the mean of its S x S samples rounded half up (integer arithmetic), and
 * the depth and id of the nearest (depth, id) among them.  Needs
 * (S W) (S H) <= VTX_MAX_PIXELS.  vtx_gbuffer and vtx_shade refuse S > 1.
 */

/*
 * options.clip_plane (paper, Results, the whole-cell figure shown with and
 * without clipping): a primitive's ray hit whose surface point lies on the
 * cut side is dropped, so the primitive draws nothing at that pixel and what
 * lies behind it shows; the cut primitives' interiors are not drawn.  The
 * test is made per pixel in FP32 in view space; the images otherwise obey
 * the same visibility rule.  VTX_EINVAL when (a, b, c) is zero but d is not.
 */

/*
 * Deferred post-passes on the G-buffer (paper, Methods, "High Quality
 * Rendering": shading modes flat, matte, glossy and toon, ambient occlusion,
 * fog and outline, as post-processing of the deferred pass).  The paper gives
 * no formulas; these are this library's readings.  With n.V the facing term,
 * AO the occlusion factor and a the albedo, per hit pixel and channel:
 *   VTX_SHADE_GLOSSY  a (0.2 + 0.8 n.V) AO + 0.25 max(0, 2 (n.V)^2 - 1)^32
 *   VTX_SHADE_MATTE   a (0.2 + 0.8 n.V) AO
 *   VTX_SHADE_FLAT    a AO
 *   VTX_SHADE_TOON    a (0.2 + 0.8 b) AO, b = min(floor(4 n.V), 3) / 3
 * then fog: f = clamp((z - fog_start) / (fog_end - fog_start), 0, 1) and
 * c = (1 - f) c + f fog_color; then outline: a hit pixel whose right, left,
 * lower or upper neighbour inside the image is background or deeper than
 * z (1 + outline_depth) takes outline_color.  Background pixels keep
 * options.background.
 */
#define VTX_SHADE_GLOSSY 0
#define VTX_SHADE_MATTE 1
#define VTX_SHADE_FLAT 2
#define VTX_SHADE_TOON 3

/*
 * options.representation (paper, Methods, "Meshless Representations": the
 * molecular representations are drawn with the same sphere and cylinder
 * impostors).  Ids keep their meaning in every representation.
 *   VTX_REP_BALL_AND_STICK  spheres of the given radii and the bonds
 *   VTX_REP_VAN_DER_WAALS   spheres of the given radii, no bonds
 *   VTX_REP_STICKS          spheres of radius bond_radius and the bonds
 *   VTX_REP_SAS             spheres of radius r + probe_radius (FP32 sum), no bonds
 */
#define VTX_REP_BALL_AND_STICK 0
#define VTX_REP_VAN_DER_WAALS 1
#define VTX_REP_STICKS 2
#define VTX_REP_SAS 3

/* Per-frame counters of the last frame queued on a stream. */
typedef struct vtx_stats {
    uint64_t visible;          /* primitives that survived frustum culling */
    uint64_t pairs;            /* (primitive, tile) bin entries */
    uint64_t fragments_tested; /* (primitive, pixel) ray tests run (VTX_FLAG_STATS: every
                                  footprint pixel; VTX_FLAG_COUNT: those the early-outs left) */
    uint64_t fragments_hit;    /* tests that hit: atom-fragments (VTX_FLAG_STATS) */
    uint64_t fragments_hit_bond; /* of which on bond cylinders (VTX_FLAG_STATS) */
    uint64_t overflow_tiles;   /* tiles resolved by the slow path because the bins were full */
    uint64_t bin_capacity;     /* bin entries available for that frame */
    uint64_t bad_bonds;        /* bonds skipped because an index was >= n_atoms */
    /* VTX_FLAG_STATS or VTX_FLAG_COUNT frames */
    uint64_t fragments_tested_bond; /* of the ray tests, those on bond cylinders */
    /* VTX_FLAG_COUNT frames: the depth early-outs of the resolve */
    uint64_t fragments_skipped; /* footprint pixels not ray-tested: the pixel held a nearer hit */
    uint64_t records_culled;   /* tile-list records dropped whole: behind every 4x4 block under them */
    uint64_t lists_stopped;    /* tile lists ended early: every layer left lay behind the tile */
    uint64_t chunks_stopped;   /* depth-ordered chunks ended early by their depth-bucket bound */
} vtx_stats;

/* Average device time per kernel of the frames rendered with VTX_FLAG_TIMING. */
typedef struct vtx_timings {
    uint64_t frames;        /* frames averaged */
    double ms_clear;        /* clear the tile counters */
    double ms_project;      /* project, cull, count per tile */
    double ms_scan;         /* prefix sum of the tile counts */
    double ms_scatter;      /* fill the tile lists */
    double ms_resolve;      /* per-tile ray casting into the G-buffer */
    double ms_shade;        /* SSAO and shading */
} vtx_timings;

/*
 * vtx_render - one frame: visibility then deferred shading.
 *
 * The paper's statement of the problem (Methods, "Molecular Graphics
 * Engine"): positions, radii and connectivity in, an image out.
 *   positions  n_atoms x 3 float, AoS (x, y, z per atom)
 *   radii      n_atoms float; atoms with radius <= 0 are not drawn
 *   colors     n_atoms RGBA8
 *   bonds      n_bonds x 2 uint32 atom indices (NULL if n_bonds == 0); bonds
 *              whose two atoms coincide are not drawn, bonds with an index
 *              >= n_atoms are skipped and counted in vtx_stats.bad_bonds
 *   cam, opt   host structs, read during the call only (opt may be NULL)
 *   rgba       W x H RGBA8 out (required)
 *   depth      W x H float out (required: the G-buffer the deferred pass reads)
 *   id         W x H uint32 out (required)
 * Requires n_atoms >= 0, n_bonds >= 0, n_atoms + n_bonds < 2^32 - 1,
 * 1 <= W, H <= VTX_MAX_SIDE and W * H <= VTX_MAX_PIXELS (both after
 * supersampling).  Errors: VTX_EINVAL, VTX_ENOMEM, VTX_EHIP.
 */
int vtx_render(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
               const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
               int32_t W, int32_t H, uint32_t* rgba, float* depth, uint32_t* id, void* stream);

/*
 * vtx_render_static - vtx_render for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, same images as vtx_render.  Every
 * scratch buffer of the frame (tile counts and lists, visible-primitive
 * lists, histograms, counters) is carved from one static device array of
 * 64 MiB that each GPU the library runs on holds until the process ends; the
 * call allocates nothing, device or pinned (the array's device address is
 * looked up once per device, on the first call).  The array is shared by
 * every call on a GPU and keeps the last call's contents: each call clears
 * what it needs zeroed with a kernel (no memset node), and calls that overlap
 * on one GPU (different streams, or host threads) race.  The tile lists get
 * the part of the array the other buffers leave; tiles whose lists do not
 * fit are resolved exactly from the visible lists, more slowly.  Frames
 * whose other buffers exceed the array (~ 12 B per primitive plus 4 B per
 * (binning workgroup, tile)) are refused with VTX_EOVERFLOW, stating the
 * bytes needed.  supersample > 1 is refused (VTX_EINVAL); VTX_FLAG_TIMING is
 * ignored; statistics are not read back (vtx_read_stats does not see these
 * frames).
 */
int vtx_render_static(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
                      const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
                      int32_t W, int32_t H, uint32_t* rgba, float* depth, uint32_t* id, void* stream);

/*
 * vtx_gbuffer - visibility only: bin the primitives into screen tiles and
 * ray-cast each pixel against its tile's primitives (Methods, "Meshless
 * Representations": a quad per primitive, then ray-casting of the implicit
 * surface).  Same arguments as vtx_render without rgba; writes depth and id.
 */
int vtx_gbuffer(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
                const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
                int32_t W, int32_t H, float* depth, uint32_t* id, void* stream);

/*
 * vtx_shade - the deferred pass over an existing G-buffer (Methods, "High
 * Quality Rendering": screen-space ambient occlusion recomputed every frame,
 * then lighting).  depth and id are inputs in the layout vtx_gbuffer writes;
 * the surface normal and colour of each pixel are derived from the primitive
 * named by id and the depth.  Optional outputs (NULL to skip), for
 * inspection: normal (W x H x 3 float, view space, unit), albedo (W x H
 * RGBA8), ao (W x H float in [0, 1]).
 */
int vtx_shade(const float* positions, const float* radii, const uint32_t* colors, int64_t n_atoms,
              const uint32_t* bonds, int64_t n_bonds, const vtx_camera* cam, const vtx_options* opt,
              int32_t W, int32_t H, const float* depth, const uint32_t* id, uint32_t* rgba,
              float* normal, uint32_t* albedo, float* ao, void* stream);

/* ---------------------------------------------------------------------------
 * Solvent excluded surface (paper, Methods, "Cartoon and SES
 * representations": the SES is computed by a discrete approach and extracted
 * with marching cubes).  This library's reading, on a grid of spacing h:
 *  - grid point (i, j, k) sits at origin + h (i, j, k); it is inside the
 *    solvent-accessible region when some atom has |p - c| < r + probe (FP64
 *    test); the other points are places a probe centre can be;
 *  - f(p) = min(h sqrt(g), W h) - probe, g the least squared grid distance
 *    from p to such a point (W = ceil(probe / h) + 2: only the sign matters
 *    beyond), in FP32; the surface encloses f >= 0 (every point at least the
 *    probe radius from every probe centre);
 *  - marching cubes over f >= 0: each cube's surface pieces come from its
 *    faces (a face whose inside corners are diagonal keeps them apart), each
 *    closed loop of edge points is a triangle or, with more than three
 *    points, a fan around their mean; a point on edge (a, b) lies at
 *    f_a / (f_a - f_b) of the way from a.
 * The surface is closed when the grid reaches past every atom by the probe
 * radius and one step (the border points are then outside).
 * ------------------------------------------------------------------------- */
typedef struct vtx_ses_grid {
    float origin[3];          /* world position of grid point (0, 0, 0) */
    float spacing;            /* h > 0 */
    int32_t dims[3];          /* points along x, y, z: each >= 2, product < 2^31 */
} vtx_ses_grid;

/*
 * vtx_ses - the solvent excluded surface of the atoms as triangles.
 *   positions  n_atoms x 3 float (device), radii n_atoms float (device)
 *   field      dims[0] x dims[1] x dims[2] float out (device, x fastest), or
 *              NULL: f at every grid point
 *   triangles  capacity x 9 float out (device): v0, v1, v2 (x, y, z each);
 *              counter-clockwise seen from outside.  Triangles are ordered by
 *              cube (x fastest), then by loop and position in the loop.
 *   n_triangles one uint64 out (device): the surface's triangle count; those
 *              past `capacity` are not written (call again with more)
 * Queued on `stream`; library scratch ~ 13 B per grid point.  VTX_EINVAL for
 * bad sizes or pointers, VTX_ENOMEM, VTX_EHIP.
 */
int vtx_ses(const float* positions, const float* radii, int64_t n_atoms, float probe_radius,
            const vtx_ses_grid* grid, float* field, float* triangles, int64_t capacity, uint64_t* n_triangles,
            void* stream);

/* ---------------------------------------------------------------------------
 * Resident scenes.  A context tracks the device memory its scenes hold
 * against a budget; a scene is a library-owned copy of a molecule kept in
 * device memory across frames, laid out for the per-frame passes (atoms
 * reordered along a Morton curve into one xyzr stream, with per-cluster
 * bounding boxes for frustum culling), following the paper's "adapted data
 * structures" for millions of atoms (Methods, "Molecular Graphics Engine").
 * Rendering a scene gives exactly the images vtx_render gives for the same
 * arrays (ids are the original atom and bond indices).
 * ------------------------------------------------------------------------- */
typedef struct vtx_context vtx_context;
typedef struct vtx_scene vtx_scene;

/* vtx_context_create - context on HIP device `device`; scenes created in it
 * may hold at most hbm_budget_bytes of device memory (0 = no limit).
 * VTX_EINVAL for a bad device. */
int vtx_context_create(int device, size_t hbm_budget_bytes, vtx_context** out);
/* vtx_context_destroy - frees the context (its scenes must be destroyed first). */
void vtx_context_destroy(vtx_context* ctx);
/* vtx_context_bytes_in_use - device bytes held by the context's scenes. */
size_t vtx_context_bytes_in_use(const vtx_context* ctx);

/* vtx_scene_footprint_bytes - device bytes a scene of this size holds. */
size_t vtx_scene_footprint_bytes(int64_t n_atoms, int64_t n_bonds);
/* vtx_frame_scratch_bytes - device bytes of per-stream scratch a frame of
 * this size needs at the start (tile bins grow afterwards if needed). */
size_t vtx_frame_scratch_bytes(int32_t W, int32_t H, int64_t n_atoms, int64_t n_bonds);

/*
 * vtx_scene_create - copies the arrays (same meaning as for vtx_render; all
 * device pointers, which the caller may free afterwards) into a new scene of
 * `ctx` on the current device (which must be the context's) and lays them
 * out.  Runs on `stream` and waits for it.  Bonds with an index >= n_atoms
 * are dropped (vtx_scene_info reports how many).  VTX_EBUSY if the scene
 * would exceed the context's budget; VTX_ENOMEM, VTX_EINVAL, VTX_EHIP.
 */
int vtx_scene_create(vtx_context* ctx, const float* positions, const float* radii, const uint32_t* colors,
                     int64_t n_atoms, const uint32_t* bonds, int64_t n_bonds, void* stream, vtx_scene** out);

/*
 * vtx_scene_update_positions - new positions (n_atoms x 3 float, device,
 * original atom order) for the next frames, e.g. a trajectory frame (paper,
 * "High Quality Rendering": dynamic data is re-rendered every frame).  Radii,
 * colours and bonds are kept.  Queued on `stream`; frames queued on that
 * stream afterwards see the new positions.
 */
int vtx_scene_update_positions(vtx_scene* scene, const float* positions, void* stream);

/*
 * vtx_scene_add_frames - stores n_frames more trajectory frames in the scene
 * (paper, "High Quality Rendering" and Results: molecular dynamics
 * trajectories are played back frame by frame, and dynamic data cannot be
 * precomputed).  `positions` is n_frames x n_atoms x 3 float, device, each
 * frame in the original atom order; the caller may free it once the stream
 * has passed this call.  The frames get the indices *first_frame,
 * *first_frame + 1, ... (frame 0 is the positions given at creation or by the
 * last vtx_scene_update_positions) and are selected per job by
 * vtx_render_batch.  Each frame holds vtx_scene_frame_bytes bytes, counted
 * against the context budget (VTX_EBUSY when over).  Queued on `stream`.
 */
int vtx_scene_add_frames(vtx_scene* scene, const float* positions, int32_t n_frames, void* stream,
                         int32_t* first_frame);
/* vtx_scene_frames - number of stored frames, frame 0 included (0 for NULL). */
int32_t vtx_scene_frames(const vtx_scene* scene);
/* vtx_scene_frame_bytes - device bytes of one added trajectory frame. */
size_t vtx_scene_frame_bytes(int64_t n_atoms, int64_t n_bonds);

/* vtx_scene_info - sizes of a scene and how many bonds were dropped; bytes
 * includes its added frames. */
int vtx_scene_info(const vtx_scene* scene, int64_t* n_atoms, int64_t* n_bonds, uint64_t* bad_bonds, size_t* bytes);

/*
 * vtx_scene_order - the scene's stored order: atom_order[i] (device, n_atoms
 * words) gets the original index of stored atom i, bond_order[j] (device,
 * n_bonds - bad_bonds words) the original index of stored bond j.  Atoms are
 * stored by their 30-bit Morton key (10 bits per axis over the bounding box
 * of the positions), bonds by the lower stored index of their two atoms,
 * each sort keeping the original order of equal keys.  Either pointer may be
 * NULL.  Queued on `stream`.  VTX_EINVAL, VTX_EHIP.
 */
int vtx_scene_order(const vtx_scene* scene, uint32_t* atom_order, uint32_t* bond_order, void* stream);

/* vtx_scene_destroy - waits for the device and frees the scene. */
void vtx_scene_destroy(vtx_scene* scene);

/*
 * vtx_render_scene - vtx_render for a resident scene: the frame's visibility
 * pass starts by testing the scene's clusters against the view volume and
 * only bins the atoms and bonds of the clusters that pass.  Outputs as for
 * vtx_render.
 */
int vtx_render_scene(vtx_scene* scene, const vtx_camera* cam, const vtx_options* opt, int32_t W, int32_t H,
                     uint32_t* rgba, float* depth, uint32_t* id, void* stream);

/*
 * One render of a batch: a frame of a resident scene seen by a camera into
 * the job's own device images (each height x width, layouts as for
 * vtx_render).
 */
typedef struct vtx_job {
    vtx_scene* scene;
    int32_t frame;             /* trajectory frame: 0 .. vtx_scene_frames(scene) - 1 */
    vtx_camera camera;
    vtx_options options;
    int32_t width, height;
    uint32_t* rgba;
    float* depth;
    uint32_t* id;
} vtx_job;

/* vtx_check_job - the argument checks vtx_render_batch applies to one job
 * (ctx may be NULL to skip the context check); VTX_OK or VTX_EINVAL with the
 * reason in vtx_last_error. */
int vtx_check_job(const vtx_context* ctx, const vtx_job* job);

/*
 * vtx_render_batch - renders n_jobs (0 .. 4096) independent jobs with one
 * launch per pass for the whole batch (cluster test, count, scatter, one
 * resolve per tile size, shade), so that many small renders (trajectory
 * frames, several viewports, the frames of several clients) fill the device
 * together; the paper's renders are independent frames of the same
 * per-frame method (Methods, "Molecular Graphics Engine" and "High Quality
 * Rendering").  Each job's images equal those vtx_render_scene gives for the
 * same scene frame, camera and options.  Scenes must belong to `ctx`, on the
 * current device; output images must not overlap.  Queued on `stream`
 * (scratch for each job is kept per stream; the first batch of a new shape
 * waits for its counts to size the bins).  vtx_read_stats afterwards sums the
 * counters over the batch's jobs.  VTX_EINVAL names the offending job.
 */
int vtx_render_batch(vtx_context* ctx, const vtx_job* jobs, int32_t n_jobs, void* stream);

/*
 * Batch graphs: a batch of jobs captured once into a hipGraph and replayed
 * with one hipGraphLaunch per call (the trajectory player's case: the same
 * renders re-run every step, e.g. after vtx_scene_update_positions or with
 * new frames written in place).  vtx_batch_graph_create checks the jobs as
 * vtx_render_batch does, renders them once on a private stream to size a
 * private scratch, then captures the launch sequence (no allocation, copy or
 * wait is captured).  Each vtx_batch_graph_launch re-renders exactly those
 * jobs (same scenes, frames, cameras, options and output images), queued on
 * `stream`; the scenes and images must outlive the graph, and launches of one
 * graph must not overlap (queue them on one stream).  VTX_FLAG_TIMING is
 * ignored inside a graph.
 */
typedef struct vtx_batch_graph vtx_batch_graph;
int vtx_batch_graph_create(vtx_context* ctx, const vtx_job* jobs, int32_t n_jobs, vtx_batch_graph** out);
int vtx_batch_graph_launch(vtx_batch_graph* graph, void* stream);
/* vtx_batch_graph_destroy - waits for the device and frees the graph and its scratch. */
void vtx_batch_graph_destroy(vtx_batch_graph* graph);

/* Choices of vtx_autotune for one render shape (all fields are outputs but
 * frame_budget_ms, which the caller sets before the call). */
typedef struct vtx_tuning {
    int32_t tile_size;        /* chosen screen tile edge (8, 16, 32 or 64) */
    int32_t from_cache;       /* 1: read from the cache file, nothing was timed */
    float ms_per_batch;       /* device time of one sample batch at that size */
    float ms_by_tile[4];      /* at 8, 16, 32, 64 (0 = not tried: too many tiles) */
    char key[96];             /* shape it applies to: WxH/p<log2(atoms + bonds)>/<projection> */
    float frame_budget_ms;    /* in: device time per render allowed to sample jobs that ask for
                                 VTX_SSAO_AUTO samples (<= 0: no budget, 16 samples) */
    int32_t ssao_samples;     /* SSAO samples of VTX_SSAO_AUTO renders of this shape
                                 (-1: no sample job asked for them) */
    uint64_t bin_capacity;    /* tile-list entries reserved for a render of this shape:
                                 5/4 of the most (primitive, tile) pairs of a sample
                                 job at the chosen tile size, plus 1024 */
    float ms_by_samples[9];   /* per-render device time with 64, 48, 32, 24, 16, 12, 8, 4, 0
                                 samples (0 = not timed) */
} vtx_tuning;

/* options.ssao_samples value that leaves the count to the context: the one
 * vtx_autotune chose for the render's shape, else 16 (and 16 for renders that
 * have no context: vtx_render, vtx_gbuffer + vtx_shade). */
#define VTX_SSAO_AUTO (-1)

/*
 * vtx_autotune - chooses, for renders shaped like the sample jobs (a shape is
 * image size, log2 of the primitive count and projection), the screen tile
 * size, the tile-list capacity and the SSAO sample count, and keeps them in
 * the context for each shape in the batch:
 *  - tile size: the sample batch (rendered into the jobs' own images, flags
 *    cleared) is timed with HIP events on `stream` at every tile size all its
 *    images accept; the fastest is used by renders of those shapes that leave
 *    options.tile_size at 0 (vtx_render_scene, vtx_render_batch).  Images do
 *    not depend on the tile size.
 *  - bin capacity: the (primitive, tile) pairs of each sample job are read
 *    back at the chosen size; a render of the shape whose scratch is new sizes
 *    its lists from them instead of counting first and waiting for the count.
 *    Images do not depend on it either (a frame that outgrows its lists is
 *    resolved exactly from the visible lists).
 *  - SSAO samples, only when a sample job's options ask for VTX_SSAO_AUTO:
 *    the largest of 64, 48, 32, 24, 16, 12, 8, 4, 0 whose measured device
 *    time per render fits out->frame_budget_ms (set by the caller; <= 0 or
 *    out NULL: 16 without timing).  This one does change the images: fewer
 *    samples, a coarser ambient occlusion.
 * With `cache_path` (NULL: none) the choices are read from that JSON file when
 * it has every shape of the batch, otherwise measured and written to it (other
 * shapes' entries are kept).  Waits for the stream.  `out` (may be NULL)
 * describes the choices for jobs[0]'s shape.  The paper's engine tunes
 * nothing; these are this library's own parameters.
 */
int vtx_autotune(vtx_context* ctx, const vtx_job* jobs, int32_t n_jobs, const char* cache_path, void* stream,
                 vtx_tuning* out);

/* ---------------------------------------------------------------------------
 * Served renders.  A server owns one worker thread that drains a request
 * queue into batches: whenever fewer than max_inflight batches are queued on
 * `stream`, the requests waiting (at most max_batch) are rendered together
 * with vtx_render_batch (continuous batching).  Each request is a vtx_job;
 * its scene and images must stay valid until its completion is reported.
 * Timestamps are seconds of vtx_clock_s (a monotonic host clock); done_s is
 * taken by a host callback queued on the stream after the request's batch,
 * i.e. once the device has finished it.  Residency and admission of scenes
 * are the caller's (vtx_scene_create answers VTX_EBUSY when a scene would
 * exceed the context budget).  The paper renders interactive sessions of
 * frames (Methods; Results, trajectories); a server of many such sessions is
 * this library's own.
 * ------------------------------------------------------------------------- */
typedef struct vtx_server vtx_server;

typedef struct vtx_completion {
    uint64_t ticket;          /* from vtx_server_submit */
    double submit_s;          /* when it was submitted */
    double launch_s;          /* when its batch was handed to the device */
    double done_s;            /* when its batch had finished on the device */
    int32_t batch_size;       /* requests in its batch */
    int32_t status;           /* VTX_OK or the error code of its batch */
} vtx_completion;

typedef struct vtx_server_stats {
    uint64_t submitted, completed, queued;
    uint64_t batches;         /* batches launched */
    uint64_t max_batch_seen;  /* largest batch so far */
    uint64_t failed;          /* requests completed with an error */
} vtx_server_stats;

/* vtx_clock_s - the monotonic host clock of the server's timestamps, seconds. */
double vtx_clock_s(void);
/* vtx_server_create - starts a server rendering in `ctx` on `stream` (current
 * device).  max_batch 1..4096, max_inflight 1..64; VTX_EINVAL otherwise. */
int vtx_server_create(vtx_context* ctx, int32_t max_batch, int32_t max_inflight, void* stream, vtx_server** out);
/* vtx_server_submit - queues one request (thread-safe; returns at once).
 * A job that fails vtx_check_job is refused with its error code. */
int vtx_server_submit(vtx_server* server, const vtx_job* job, uint64_t* ticket);
/* vtx_server_poll - moves up to `max` completions to `out` (*n of them),
 * waiting up to wait_ms for the first when none is ready. */
int vtx_server_poll(vtx_server* server, vtx_completion* out, int32_t max, int32_t wait_ms, int32_t* n);
/* vtx_server_drain - waits until every submitted request has completed. */
int vtx_server_drain(vtx_server* server);
/* vtx_server_stats_read - counters of the server. */
int vtx_server_stats_read(vtx_server* server, vtx_server_stats* out);
/* vtx_server_destroy - renders what is queued, waits for it, stops the worker. */
void vtx_server_destroy(vtx_server* server);

/*
 * vtx_read_stats - waits for `stream` to drain, then returns the counters of
 * the last call queued on it by this library (summed over its jobs for a
 * batch).  VTX_EINVAL if none was.
 */
int vtx_read_stats(void* stream, vtx_stats* out);

/*
 * vtx_set_bin_capacity - fixes the number of tile-bin entries (8 bytes
 * each: a primitive's source index and its footprint in the tile) of the
 * stream's scratch (entries >= 1), or restores automatic sizing
 * (entries = 0: the bins start at max(2^20, (n_atoms + n_bonds) / 2) entries
 * and grow after a frame that needed more).  A frame whose bins overflow is still exact: the
 * tiles that did not fit are resolved from the list of visible primitives,
 * more slowly, and counted in vtx_stats.overflow_tiles.  Waits for the
 * stream.  VTX_EINVAL if entries > 2^28.
 */
int vtx_set_bin_capacity(void* stream, uint64_t entries);

/*
 * vtx_read_timings - waits for `stream`, then returns the per-kernel averages
 * over the frames queued on it with VTX_FLAG_TIMING since the last
 * vtx_reset_timings (frames = 0 if none).
 */
int vtx_read_timings(void* stream, vtx_timings* out);

/* vtx_reset_timings - waits for `stream` and clears its timing averages. */
int vtx_reset_timings(void* stream);

/* vtx_release_scratch - waits for the stream and frees its scratch memory. */
int vtx_release_scratch(void* stream);

/* vtx_last_error - message of the last failed call on this host thread ("" if none). */
const char* vtx_last_error(void);

/* vtx_version - library version string. */
const char* vtx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VTX_H */
