"""Python binding of libvtx (include/vtx.h): argument marshalling only.

Every function of the C ABI is exposed under the same name; all rendering
work runs in the HIP kernels of libvtx.so.  Torch supplies device memory and
streams: array arguments are CUDA (HIP) tensors or raw device addresses.
There is no CPU fallback: importing this module without the built library
raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvtx.so")

VTX_OK = 0
VTX_EINVAL = -1
VTX_ENOMEM = -2
VTX_EHIP = -3
VTX_EOVERFLOW = -4
VTX_EBUSY = -5
VTX_PERSPECTIVE = 0
VTX_ORTHOGRAPHIC = 1
VTX_BACKGROUND_ID = 0xFFFFFFFF
VTX_MAX_PIXELS = 7680 * 4320
VTX_MAX_SIDE = 16383
VTX_MAX_SSAO_SAMPLES = 64
VTX_SSAO_AUTO = -1
VTX_FLAG_STATS = 1
VTX_FLAG_TIMING = 2
VTX_FLAG_ONE_PASS = 4
VTX_FLAG_TWO_PASS = 8
VTX_FLAG_COUNT = 16
VTX_REP_BALL_AND_STICK, VTX_REP_VAN_DER_WAALS, VTX_REP_STICKS, VTX_REP_SAS = 0, 1, 2, 3
VTX_SHADE_GLOSSY, VTX_SHADE_MATTE, VTX_SHADE_FLAT, VTX_SHADE_TOON = 0, 1, 2, 3

# Every symbol include/vtx.h declares.
EXPORTS = ("vtx_render", "vtx_gbuffer", "vtx_shade", "vtx_read_stats", "vtx_set_bin_capacity",
           "vtx_read_timings", "vtx_reset_timings", "vtx_release_scratch", "vtx_last_error", "vtx_version",
           "vtx_context_create", "vtx_context_destroy", "vtx_context_bytes_in_use", "vtx_scene_footprint_bytes",
           "vtx_frame_scratch_bytes", "vtx_scene_create", "vtx_scene_update_positions", "vtx_scene_info",
           "vtx_scene_order", "vtx_scene_destroy", "vtx_render_scene", "vtx_scene_add_frames", "vtx_scene_frames",
           "vtx_scene_frame_bytes", "vtx_render_batch", "vtx_autotune", "vtx_clock_s", "vtx_server_create",
           "vtx_server_submit", "vtx_server_poll", "vtx_server_drain", "vtx_server_stats_read",
           "vtx_server_destroy", "vtx_check_job", "vtx_batch_graph_create",
           "vtx_batch_graph_launch", "vtx_batch_graph_destroy", "vtx_render_static", "vtx_ses")


class vtx_camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("target", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fovy", ctypes.c_float), ("ortho_half_height", ctypes.c_float),
                ("projection", ctypes.c_int32), ("znear", ctypes.c_float), ("zfar", ctypes.c_float)]


class vtx_options(ctypes.Structure):
    _fields_ = [("bond_radius", ctypes.c_float), ("ssao_samples", ctypes.c_int32),
                ("ssao_radius", ctypes.c_float), ("ssao_bias", ctypes.c_float),
                ("background", ctypes.c_uint32), ("tile_size", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("representation", ctypes.c_int32), ("probe_radius", ctypes.c_float),
                ("shading", ctypes.c_int32), ("fog_color", ctypes.c_uint32), ("fog_start", ctypes.c_float),
                ("fog_end", ctypes.c_float), ("outline_color", ctypes.c_uint32), ("outline_depth", ctypes.c_float),
                ("clip_plane", ctypes.c_float * 4), ("supersample", ctypes.c_int32), ("ssao_noise", ctypes.c_int32)]


class vtx_ses_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float), ("dims", ctypes.c_int32 * 3)]


class vtx_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("visible", "pairs", "fragments_tested", "fragments_hit",
                                               "fragments_hit_bond", "overflow_tiles", "bin_capacity",
                                               "bad_bonds", "fragments_tested_bond", "fragments_skipped",
                                               "records_culled", "lists_stopped", "chunks_stopped")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class vtx_timings(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_uint64)] + [(k, ctypes.c_double) for k in (
        "ms_clear", "ms_project", "ms_scan", "ms_scatter", "ms_resolve", "ms_shade")]

    def as_dict(self):
        return {k: (int(getattr(self, k)) if k == "frames" else float(getattr(self, k))) for k, _ in self._fields_}


class vtx_job(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("frame", ctypes.c_int32), ("camera", vtx_camera),
                ("options", vtx_options), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("rgba", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("id", ctypes.c_void_p)]


SSAO_COUNTS = (64, 48, 32, 24, 16, 12, 8, 4, 0)   # the sample counts vtx_autotune tries, in its order


class vtx_tuning(ctypes.Structure):
    _fields_ = [("tile_size", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("ms_per_batch", ctypes.c_float),
                ("ms_by_tile", ctypes.c_float * 4), ("key", ctypes.c_char * 96),
                ("frame_budget_ms", ctypes.c_float), ("ssao_samples", ctypes.c_int32),
                ("bin_capacity", ctypes.c_uint64), ("ms_by_samples", ctypes.c_float * 9)]

    def as_dict(self):
        return {"tile_size": self.tile_size, "from_cache": bool(self.from_cache),
                "ms_per_batch": float(self.ms_per_batch),
                "ms_by_tile": {t: float(v) for t, v in zip((8, 16, 32, 64), self.ms_by_tile) if v > 0},
                "key": self.key.decode(), "frame_budget_ms": float(self.frame_budget_ms),
                "ssao_samples": int(self.ssao_samples), "bin_capacity": int(self.bin_capacity),
                "ms_by_samples": {k: float(v) for k, v in zip(SSAO_COUNTS, self.ms_by_samples) if v > 0}}


class vtx_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("submit_s", ctypes.c_double), ("launch_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("batch_size", ctypes.c_int32), ("status", ctypes.c_int32)]


class vtx_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "queued", "batches", "max_batch_seen",
                                               "failed")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class VtxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vtx error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2501_12750_amd.build` "
                      "(the renderer has no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_CAM = ctypes.POINTER(vtx_camera)
_OPT = ctypes.POINTER(vtx_options)

_lib.vtx_render.restype = ctypes.c_int
_lib.vtx_render.argtypes = [_P, _P, _P, _I64, _P, _I64, _CAM, _OPT, _I32, _I32, _P, _P, _P, _P]
_lib.vtx_ses.restype = ctypes.c_int
_lib.vtx_ses.argtypes = [_P, _P, _I64, ctypes.c_float, ctypes.POINTER(vtx_ses_grid), _P, _P, _I64, _P, _P]
_lib.vtx_render_static.restype = ctypes.c_int
_lib.vtx_render_static.argtypes = [_P, _P, _P, _I64, _P, _I64, _CAM, _OPT, _I32, _I32, _P, _P, _P, _P]
_lib.vtx_gbuffer.restype = ctypes.c_int
_lib.vtx_gbuffer.argtypes = [_P, _P, _P, _I64, _P, _I64, _CAM, _OPT, _I32, _I32, _P, _P, _P]
_lib.vtx_shade.restype = ctypes.c_int
_lib.vtx_shade.argtypes = [_P, _P, _P, _I64, _P, _I64, _CAM, _OPT, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]
_lib.vtx_read_stats.restype = ctypes.c_int
_lib.vtx_read_stats.argtypes = [_P, ctypes.POINTER(vtx_stats)]
_lib.vtx_set_bin_capacity.restype = ctypes.c_int
_lib.vtx_set_bin_capacity.argtypes = [_P, ctypes.c_uint64]
_lib.vtx_read_timings.restype = ctypes.c_int
_lib.vtx_read_timings.argtypes = [_P, ctypes.POINTER(vtx_timings)]
_lib.vtx_reset_timings.restype = ctypes.c_int
_lib.vtx_reset_timings.argtypes = [_P]
_lib.vtx_release_scratch.restype = ctypes.c_int
_lib.vtx_release_scratch.argtypes = [_P]
_lib.vtx_context_create.restype = ctypes.c_int
_lib.vtx_context_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_P)]
_lib.vtx_context_destroy.restype = None
_lib.vtx_context_destroy.argtypes = [_P]
_lib.vtx_context_bytes_in_use.restype = ctypes.c_size_t
_lib.vtx_context_bytes_in_use.argtypes = [_P]
_lib.vtx_scene_footprint_bytes.restype = ctypes.c_size_t
_lib.vtx_scene_footprint_bytes.argtypes = [_I64, _I64]
_lib.vtx_frame_scratch_bytes.restype = ctypes.c_size_t
_lib.vtx_frame_scratch_bytes.argtypes = [_I32, _I32, _I64, _I64]
_lib.vtx_scene_create.restype = ctypes.c_int
_lib.vtx_scene_create.argtypes = [_P, _P, _P, _P, _I64, _P, _I64, _P, ctypes.POINTER(_P)]
_lib.vtx_scene_update_positions.restype = ctypes.c_int
_lib.vtx_scene_update_positions.argtypes = [_P, _P, _P]
_lib.vtx_scene_info.restype = ctypes.c_int
_lib.vtx_scene_info.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(ctypes.c_size_t)]
_lib.vtx_scene_order.restype = ctypes.c_int
_lib.vtx_scene_order.argtypes = [_P, _P, _P, _P]
_lib.vtx_scene_destroy.restype = None
_lib.vtx_scene_destroy.argtypes = [_P]
_lib.vtx_render_scene.restype = ctypes.c_int
_lib.vtx_render_scene.argtypes = [_P, _CAM, _OPT, _I32, _I32, _P, _P, _P, _P]
_lib.vtx_scene_add_frames.restype = ctypes.c_int
_lib.vtx_scene_add_frames.argtypes = [_P, _P, _I32, _P, ctypes.POINTER(_I32)]
_lib.vtx_scene_frames.restype = _I32
_lib.vtx_scene_frames.argtypes = [_P]
_lib.vtx_scene_frame_bytes.restype = ctypes.c_size_t
_lib.vtx_scene_frame_bytes.argtypes = [_I64, _I64]
_lib.vtx_render_batch.restype = ctypes.c_int
_lib.vtx_render_batch.argtypes = [_P, ctypes.POINTER(vtx_job), _I32, _P]
_lib.vtx_autotune.restype = ctypes.c_int
_lib.vtx_autotune.argtypes = [_P, ctypes.POINTER(vtx_job), _I32, ctypes.c_char_p, _P, ctypes.POINTER(vtx_tuning)]
_lib.vtx_batch_graph_create.restype = ctypes.c_int
_lib.vtx_batch_graph_create.argtypes = [_P, ctypes.POINTER(vtx_job), _I32, ctypes.POINTER(_P)]
_lib.vtx_batch_graph_launch.restype = ctypes.c_int
_lib.vtx_batch_graph_launch.argtypes = [_P, _P]
_lib.vtx_batch_graph_destroy.restype = None
_lib.vtx_batch_graph_destroy.argtypes = [_P]
_lib.vtx_check_job.restype = ctypes.c_int
_lib.vtx_check_job.argtypes = [_P, ctypes.POINTER(vtx_job)]
_lib.vtx_clock_s.restype = ctypes.c_double
_lib.vtx_clock_s.argtypes = []
_lib.vtx_server_create.restype = ctypes.c_int
_lib.vtx_server_create.argtypes = [_P, _I32, _I32, _P, ctypes.POINTER(_P)]
_lib.vtx_server_submit.restype = ctypes.c_int
_lib.vtx_server_submit.argtypes = [_P, ctypes.POINTER(vtx_job), ctypes.POINTER(ctypes.c_uint64)]
_lib.vtx_server_poll.restype = ctypes.c_int
_lib.vtx_server_poll.argtypes = [_P, ctypes.POINTER(vtx_completion), _I32, _I32, ctypes.POINTER(_I32)]
_lib.vtx_server_drain.restype = ctypes.c_int
_lib.vtx_server_drain.argtypes = [_P]
_lib.vtx_server_stats_read.restype = ctypes.c_int
_lib.vtx_server_stats_read.argtypes = [_P, ctypes.POINTER(vtx_server_stats)]
_lib.vtx_server_destroy.restype = None
_lib.vtx_server_destroy.argtypes = [_P]
_lib.vtx_last_error.restype = ctypes.c_char_p
_lib.vtx_last_error.argtypes = []
_lib.vtx_version.restype = ctypes.c_char_p
_lib.vtx_version.argtypes = []


def _addr(x):
    """Device address of a tensor (or an int address, or None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc):
    if rc != VTX_OK:
        raise VtxError(rc, vtx_last_error())


def camera_struct(cam) -> vtx_camera:
    c = vtx_camera()
    c.eye[:] = list(cam.eye)
    c.target[:] = list(cam.target)
    c.up[:] = list(cam.up)
    c.fovy = cam.fovy
    c.ortho_half_height = cam.ortho_half_height
    c.projection = int(cam.projection)
    c.znear = cam.znear
    c.zfar = cam.zfar
    return c


def options_struct(opts) -> vtx_options:
    o = vtx_options()
    o.bond_radius = opts.bond_radius
    o.ssao_samples = int(opts.ssao_samples)
    o.ssao_radius = opts.ssao_radius
    o.ssao_bias = opts.ssao_bias
    o.background = int(opts.background) & 0xFFFFFFFF
    o.tile_size = int(getattr(opts, "tile_size", 0))
    o.flags = int(getattr(opts, "flags", 0))
    o.representation = int(getattr(opts, "representation", 0))
    o.probe_radius = float(getattr(opts, "probe_radius", 1.4))
    o.shading = int(getattr(opts, "shading", 0))
    o.fog_color = int(getattr(opts, "fog_color", 0)) & 0xFFFFFFFF
    o.fog_start = float(getattr(opts, "fog_start", 0.0))
    o.fog_end = float(getattr(opts, "fog_end", 0.0))
    o.outline_color = int(getattr(opts, "outline_color", 0)) & 0xFFFFFFFF
    o.outline_depth = float(getattr(opts, "outline_depth", 0.0))
    o.clip_plane[:] = [float(v) for v in getattr(opts, "clip_plane", (0.0, 0.0, 0.0, 0.0))]
    o.supersample = int(getattr(opts, "supersample", 1))
    o.ssao_noise = int(getattr(opts, "ssao_noise", 0))
    return o


def _cam_opt(cam, opts):
    c = cam if isinstance(cam, vtx_camera) else camera_struct(cam)
    o = None if opts is None else (opts if isinstance(opts, vtx_options) else options_struct(opts))
    return ctypes.byref(c), (ctypes.byref(o) if o is not None else None), (c, o)


def vtx_render(positions, radii, colors, n_atoms, bonds, n_bonds, cam, opts, W, H, rgba, depth, id,
               stream=None):
    cp, op, _keep = _cam_opt(cam, opts)
    _check(_lib.vtx_render(_addr(positions), _addr(radii), _addr(colors), n_atoms, _addr(bonds), n_bonds,
                           cp, op, W, H, _addr(rgba), _addr(depth), _addr(id), _stream(stream)))


def vtx_render_static(positions, radii, colors, n_atoms, bonds, n_bonds, cam, opts, W, H, rgba, depth, id,
                      stream=None):
    cp, op, _keep = _cam_opt(cam, opts)
    _check(_lib.vtx_render_static(_addr(positions), _addr(radii), _addr(colors), n_atoms, _addr(bonds), n_bonds,
                                  cp, op, W, H, _addr(rgba), _addr(depth), _addr(id), _stream(stream)))


def vtx_ses(positions, radii, n_atoms, probe_radius, origin, spacing, dims, field, triangles, capacity, n_triangles,
            stream=None):
    g = vtx_ses_grid()
    for k in range(3):
        g.origin[k] = float(origin[k])
        g.dims[k] = int(dims[k])
    g.spacing = float(spacing)
    _check(_lib.vtx_ses(_addr(positions), _addr(radii), n_atoms, float(probe_radius), ctypes.byref(g), _addr(field),
                        _addr(triangles), int(capacity), _addr(n_triangles), _stream(stream)))


def vtx_gbuffer(positions, radii, colors, n_atoms, bonds, n_bonds, cam, opts, W, H, depth, id, stream=None):
    cp, op, _keep = _cam_opt(cam, opts)
    _check(_lib.vtx_gbuffer(_addr(positions), _addr(radii), _addr(colors), n_atoms, _addr(bonds), n_bonds,
                            cp, op, W, H, _addr(depth), _addr(id), _stream(stream)))


def vtx_shade(positions, radii, colors, n_atoms, bonds, n_bonds, cam, opts, W, H, depth, id, rgba,
              normal=None, albedo=None, ao=None, stream=None):
    cp, op, _keep = _cam_opt(cam, opts)
    _check(_lib.vtx_shade(_addr(positions), _addr(radii), _addr(colors), n_atoms, _addr(bonds), n_bonds,
                          cp, op, W, H, _addr(depth), _addr(id), _addr(rgba), _addr(normal), _addr(albedo),
                          _addr(ao), _stream(stream)))


def vtx_read_stats(stream=None) -> dict:
    st = vtx_stats()
    _check(_lib.vtx_read_stats(_stream(stream), ctypes.byref(st)))
    return st.as_dict()


def vtx_set_bin_capacity(entries, stream=None):
    _check(_lib.vtx_set_bin_capacity(_stream(stream), int(entries)))


def vtx_read_timings(stream=None) -> dict:
    t = vtx_timings()
    _check(_lib.vtx_read_timings(_stream(stream), ctypes.byref(t)))
    return t.as_dict()


def vtx_reset_timings(stream=None):
    _check(_lib.vtx_reset_timings(_stream(stream)))


def vtx_release_scratch(stream=None):
    _check(_lib.vtx_release_scratch(_stream(stream)))


def vtx_context_create(device=0, hbm_budget_bytes=0) -> int:
    h = _P()
    _check(_lib.vtx_context_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
    return h.value


def vtx_context_destroy(ctx):
    _lib.vtx_context_destroy(ctx)


def vtx_context_bytes_in_use(ctx) -> int:
    return int(_lib.vtx_context_bytes_in_use(ctx))


def vtx_scene_footprint_bytes(n_atoms, n_bonds) -> int:
    return int(_lib.vtx_scene_footprint_bytes(int(n_atoms), int(n_bonds)))


def vtx_frame_scratch_bytes(W, H, n_atoms, n_bonds) -> int:
    return int(_lib.vtx_frame_scratch_bytes(int(W), int(H), int(n_atoms), int(n_bonds)))


def vtx_scene_create(ctx, positions, radii, colors, n_atoms, bonds, n_bonds, stream=None) -> int:
    h = _P()
    _check(_lib.vtx_scene_create(ctx, _addr(positions), _addr(radii), _addr(colors), n_atoms, _addr(bonds),
                                 n_bonds, _stream(stream), ctypes.byref(h)))
    return h.value


def vtx_scene_update_positions(scene, positions, stream=None):
    _check(_lib.vtx_scene_update_positions(scene, _addr(positions), _stream(stream)))


def vtx_scene_info(scene) -> dict:
    n, m, bad, nbytes = _I64(), _I64(), ctypes.c_uint64(), ctypes.c_size_t()
    _check(_lib.vtx_scene_info(scene, ctypes.byref(n), ctypes.byref(m), ctypes.byref(bad), ctypes.byref(nbytes)))
    return {"n_atoms": n.value, "n_bonds": m.value, "bad_bonds": bad.value, "bytes": nbytes.value}


def vtx_scene_order(scene, atom_order, bond_order, stream=None):
    """Original index of each stored atom / stored bond into device arrays
    (either may be None)."""
    _check(_lib.vtx_scene_order(scene, _addr(atom_order), _addr(bond_order), _stream(stream)))


def vtx_scene_destroy(scene):
    _lib.vtx_scene_destroy(scene)


def vtx_render_scene(scene, cam, opts, W, H, rgba, depth, id, stream=None):
    cp, op, _keep = _cam_opt(cam, opts)
    _check(_lib.vtx_render_scene(scene, cp, op, W, H, _addr(rgba), _addr(depth), _addr(id), _stream(stream)))


def vtx_scene_add_frames(scene, positions, n_frames, stream=None) -> int:
    """Stores n_frames trajectory frames (n_frames x n_atoms x 3 on the device);
    returns the index of the first."""
    first = _I32()
    _check(_lib.vtx_scene_add_frames(scene, _addr(positions), int(n_frames), _stream(stream), ctypes.byref(first)))
    return first.value


def vtx_scene_frames(scene) -> int:
    return int(_lib.vtx_scene_frames(scene))


def vtx_scene_frame_bytes(n_atoms, n_bonds) -> int:
    return int(_lib.vtx_scene_frame_bytes(int(n_atoms), int(n_bonds)))


def make_job(scene, frame, cam, opts, W, H, rgba, depth, id) -> vtx_job:
    j = vtx_job()
    j.scene = scene
    j.frame = int(frame)
    j.camera = cam if isinstance(cam, vtx_camera) else camera_struct(cam)
    j.options = opts if isinstance(opts, vtx_options) else options_struct(opts)
    j.width, j.height = int(W), int(H)
    j.rgba, j.depth, j.id = _addr(rgba), _addr(depth), _addr(id)
    return j


def vtx_render_batch(ctx, jobs, stream=None):
    """jobs: a sequence of vtx_job (see make_job) or a ctypes array of them."""
    if not isinstance(jobs, ctypes.Array):
        arr = (vtx_job * len(jobs))(*jobs)
    else:
        arr = jobs
    _check(_lib.vtx_render_batch(ctx, arr, len(arr), _stream(stream)))


def vtx_autotune(ctx, jobs, cache_path=None, stream=None, frame_budget_ms=0.0) -> dict:
    arr = jobs if isinstance(jobs, ctypes.Array) else (vtx_job * len(jobs))(*jobs)
    t = vtx_tuning()
    t.frame_budget_ms = float(frame_budget_ms)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(_lib.vtx_autotune(ctx, arr, len(arr), path, _stream(stream), ctypes.byref(t)))
    return t.as_dict()


def vtx_clock_s() -> float:
    return float(_lib.vtx_clock_s())


def vtx_server_create(ctx, max_batch=64, max_inflight=2, stream=None) -> int:
    h = _P()
    rc = _lib.vtx_server_create(ctx, int(max_batch), int(max_inflight), _stream(stream), ctypes.byref(h))
    if rc != VTX_OK:
        raise VtxError(rc, "vtx_server_create: bad arguments")
    return h.value


def vtx_batch_graph_create(ctx, jobs) -> int:
    arr = jobs if isinstance(jobs, ctypes.Array) else (vtx_job * len(jobs))(*jobs)
    h = _P()
    _check(_lib.vtx_batch_graph_create(ctx, arr, len(arr), ctypes.byref(h)))
    return h.value


def vtx_batch_graph_launch(graph, stream=None):
    _check(_lib.vtx_batch_graph_launch(graph, _stream(stream)))


def vtx_batch_graph_destroy(graph):
    _lib.vtx_batch_graph_destroy(graph)


def vtx_check_job(ctx, job):
    _check(_lib.vtx_check_job(ctx, ctypes.byref(job)))


def vtx_server_submit(server, job) -> int:
    t = ctypes.c_uint64()
    _check(_lib.vtx_server_submit(server, ctypes.byref(job), ctypes.byref(t)))
    return t.value


def vtx_server_poll(server, max_items=256, wait_ms=0) -> list:
    buf = (vtx_completion * max(1, max_items))()
    n = _I32()
    _check(_lib.vtx_server_poll(server, buf, int(max_items), int(wait_ms), ctypes.byref(n)))
    return [{"ticket": c.ticket, "submit_s": c.submit_s, "launch_s": c.launch_s, "done_s": c.done_s,
             "batch_size": c.batch_size, "status": c.status} for c in buf[:n.value]]


def vtx_server_drain(server):
    _check(_lib.vtx_server_drain(server))


def vtx_server_stats_read(server) -> dict:
    st = vtx_server_stats()
    _check(_lib.vtx_server_stats_read(server, ctypes.byref(st)))
    return st.as_dict()


def vtx_server_destroy(server):
    _lib.vtx_server_destroy(server)


def vtx_last_error() -> str:
    return (_lib.vtx_last_error() or b"").decode()


def vtx_version() -> str:
    return (_lib.vtx_version() or b"").decode()


# ---------------------------------------------------------------------------
# convenience: scenes resident in device memory, outputs allocated by torch
# ---------------------------------------------------------------------------
class DeviceScene:
    """Device copies (torch tensors) of a scene's arrays."""

    def __init__(self, scene, device="cuda"):
        import torch
        self.n_atoms = int(scene.n_atoms)
        self.n_bonds = int(scene.n_bonds)
        self.positions = torch.from_numpy(np.ascontiguousarray(scene.positions, dtype=np.float32)).to(device)
        self.radii = torch.from_numpy(np.ascontiguousarray(scene.radii, dtype=np.float32)).to(device)
        self.colors = torch.from_numpy(np.ascontiguousarray(scene.colors, dtype=np.uint32).view(np.int32)).to(device)
        b = np.ascontiguousarray(scene.bonds, dtype=np.uint32).reshape(-1, 2)
        self.bonds = torch.from_numpy(b.view(np.int32)).to(device) if self.n_bonds else None

    def args(self):
        return (self.positions, self.radii, self.colors, self.n_atoms, self.bonds, self.n_bonds)


class Frame:
    """Output buffers of one W x H frame (torch tensors on the device)."""

    def __init__(self, W, H, device="cuda", aux=False):
        import torch
        self.W, self.H = W, H
        self.rgba = torch.empty((H, W), dtype=torch.int32, device=device)
        self.depth = torch.empty((H, W), dtype=torch.float32, device=device)
        self.id = torch.empty((H, W), dtype=torch.int32, device=device)
        if aux:
            self.normal = torch.empty((H, W, 3), dtype=torch.float32, device=device)
            self.albedo = torch.empty((H, W), dtype=torch.int32, device=device)
            self.ao = torch.empty((H, W), dtype=torch.float32, device=device)

    def numpy(self):
        out = {"rgba": self.rgba.cpu().numpy().view(np.uint32), "depth": self.depth.cpu().numpy(),
               "id": self.id.cpu().numpy().view(np.uint32)}
        if hasattr(self, "normal"):
            out["normal"] = self.normal.cpu().numpy()
            out["albedo"] = self.albedo.cpu().numpy().view(np.uint32)
            out["ao"] = self.ao.cpu().numpy()
        return out


def render(dscene, cam, opts, W, H, frame=None, stream=None) -> Frame:
    fr = frame if frame is not None else Frame(W, H)
    vtx_render(*dscene.args(), cam, opts, W, H, fr.rgba, fr.depth, fr.id, stream)
    return fr


def gbuffer(dscene, cam, opts, W, H, frame=None, stream=None) -> Frame:
    fr = frame if frame is not None else Frame(W, H)
    vtx_gbuffer(*dscene.args(), cam, opts, W, H, fr.depth, fr.id, stream)
    return fr


def shade(dscene, cam, opts, W, H, frame, stream=None) -> Frame:
    vtx_shade(*dscene.args(), cam, opts, W, H, frame.depth, frame.id, frame.rgba,
              getattr(frame, "normal", None), getattr(frame, "albedo", None), getattr(frame, "ao", None), stream)
    return frame


class ResidentScene:
    """A scene kept in device memory by the library (vtx_scene_create)."""

    def __init__(self, ctx, dscene, stream=None):
        self.ctx = ctx
        self.n_atoms, self.n_bonds = dscene.n_atoms, dscene.n_bonds
        self.handle = vtx_scene_create(ctx, *dscene.args(), stream=stream)

    def update_positions(self, positions, stream=None):
        vtx_scene_update_positions(self.handle, positions, stream)

    def render(self, cam, opts, W, H, frame=None, stream=None) -> Frame:
        fr = frame if frame is not None else Frame(W, H)
        vtx_render_scene(self.handle, cam, opts, W, H, fr.rgba, fr.depth, fr.id, stream)
        return fr

    def add_frames(self, positions, n_frames, stream=None) -> int:
        return vtx_scene_add_frames(self.handle, positions, n_frames, stream)

    def frames(self) -> int:
        return vtx_scene_frames(self.handle)

    def info(self):
        return vtx_scene_info(self.handle)

    def order(self, stream=None):
        """(atom_order, bond_order) as int64 host arrays: the original index
        of each stored atom and of each stored bond."""
        import torch
        info = self.info()
        a = torch.empty(max(1, info["n_atoms"]), dtype=torch.int32, device="cuda")
        b = torch.empty(max(1, info["n_bonds"] - info["bad_bonds"]), dtype=torch.int32, device="cuda")
        vtx_scene_order(self.handle, a, b, stream)
        torch.cuda.synchronize()
        mask = 0xFFFFFFFF
        return ((a.cpu().numpy().astype("int64") & mask)[:info["n_atoms"]],
                (b.cpu().numpy().astype("int64") & mask)[:info["n_bonds"] - info["bad_bonds"]])

    def close(self):
        if self.handle:
            vtx_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
