"""Python side of O-splat, the footprint-restricted FP64 C reference renderer.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product.  Returns the same
per-pixel dict layout as ``ofull.gbuffer`` / ``ofull.render``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "osplat.c")
LIB = os.path.join(HERE, "libosplat.so")
MAX_ACCEPT = 8
BACKGROUND_ID = 0xFFFFFFFF

_lib = None


def build(force: bool = True) -> str:
    """Compile osplat.c with gcc (plain IEEE FP64, no fast-math) into libosplat.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.osplat_gbuffer.restype = ctypes.c_int
        L.osplat_gbuffer.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int64, P, ctypes.c_double, P,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     P, P, P, P, P, P, P, P, P, P, P]
        L.osplat_shade.restype = ctypes.c_int
        L.osplat_shade.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, P, P, P, P, P,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_uint32,
                                   ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                   ctypes.c_double, ctypes.c_uint32, P,
                                   ctypes.c_int, P, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def cam_array(cam, opts=None) -> np.ndarray:
    clip = [float(v) for v in getattr(opts, "clip_plane", (0.0, 0.0, 0.0, 0.0))] if opts is not None else [0.0] * 4
    return np.array(list(cam.eye) + list(cam.target) + list(cam.up)
                    + [cam.fovy, cam.ortho_half_height, float(cam.projection), cam.znear, cam.zfar] + clip,
                    dtype=np.float64)


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def gbuffer(scene, cam, opts, W, H, window=None, nthreads=None):
    from oracle.ofull import representation_scene
    if window is None:
        window = (0, 0, W, H)
    scene = representation_scene(scene, opts)
    x0, y0, w, h = window
    P = w * h
    pos = np.ascontiguousarray(scene.positions, dtype=np.float32)
    rad = np.ascontiguousarray(scene.radii, dtype=np.float32)
    col = np.ascontiguousarray(scene.colors, dtype=np.uint32)
    bonds = np.ascontiguousarray(scene.bonds, dtype=np.uint32).reshape(-1, 2)
    if bonds.size == 0:
        bonds = np.zeros((1, 2), dtype=np.uint32)
    nb = scene.n_bonds
    out = dict(z=np.empty(P), id=np.empty(P, dtype=np.uint32), normal_view=np.empty((P, 3)),
               albedo=np.empty(P, dtype=np.uint32), unstable=np.empty(P, dtype=np.uint8),
               nv=np.empty(P), acc_n=np.empty(P, dtype=np.int32),
               acc_id=np.empty((P, MAX_ACCEPT), dtype=np.uint32), acc_z=np.empty((P, MAX_ACCEPT)),
               acc_bg=np.empty(P, dtype=np.uint8))
    frag = np.zeros(1, dtype=np.int64)
    ca = cam_array(cam, opts)
    rc = lib().osplat_gbuffer(scene.n_atoms, _ptr(pos), _ptr(rad), _ptr(col), nb, _ptr(bonds),
                              float(opts.bond_radius), _ptr(ca), W, H, x0, y0, w, h,
                              nthreads or default_threads(),
                              _ptr(out["z"]), _ptr(out["id"]), _ptr(out["normal_view"]),
                              _ptr(out["albedo"]), _ptr(out["unstable"]), _ptr(out["nv"]),
                              _ptr(out["acc_n"]), _ptr(out["acc_id"]), _ptr(out["acc_z"]),
                              _ptr(out["acc_bg"]), _ptr(frag))
    if rc != 0:
        raise RuntimeError(f"osplat_gbuffer failed: {rc}")
    res = {}
    for k, v in out.items():
        if k in ("normal_view",):
            res[k] = v.reshape(h, w, 3)
        elif k in ("acc_id", "acc_z"):
            res[k] = v.reshape(h, w, MAX_ACCEPT)
        else:
            res[k] = v.reshape(h, w)
    res["id"] = res["id"].astype(np.int64)
    res["acc_id"] = res["acc_id"].astype(np.int64)
    res["unstable"] = res["unstable"].astype(bool)
    res["acc_bg"] = res["acc_bg"].astype(bool)
    res["fragments"] = int(frag[0])
    res["view"] = (cam, W, H, window)
    return res


def shade_gbuffer(cam, opts, W, H, window, z, normal_view, albedo, depth_buf=None, depth_win=None,
                  nthreads=None, edge_px=1e-3, depth_rel=1e-5, ambiguous=None, normal_buf=None):
    """Deferred pass over the window (see ofull.shade_gbuffer, same arguments)."""
    x0, y0, w, h = window
    if depth_buf is None:
        depth_buf, depth_win = z, window
        normal_buf = normal_view
    if normal_buf is None:
        normal_buf = normal_view if tuple(depth_win) == tuple(window) else None
    noise = int(getattr(opts, "ssao_noise", 0))
    if noise and normal_buf is None:
        raise ValueError("SSAO noise needs the normals over the depth buffer (normal_buf)")
    nb = None if normal_buf is None else np.ascontiguousarray(normal_buf, dtype=np.float64)
    amb = None if ambiguous is None else np.ascontiguousarray(ambiguous, dtype=np.uint8)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    nn = np.ascontiguousarray(normal_view, dtype=np.float64)
    al = np.ascontiguousarray(albedo, dtype=np.uint32)
    db = np.ascontiguousarray(depth_buf, dtype=np.float64)
    bx0, by0, bw, bh = depth_win
    P = w * h
    rgba = np.empty(P, dtype=np.uint32)
    ao = np.empty(P)
    uns = np.empty(P, dtype=np.int32)
    outside = np.empty(P, dtype=np.int32)
    ca = cam_array(cam)
    rc = lib().osplat_shade(_ptr(ca), W, H, x0, y0, w, h, _ptr(zz), _ptr(nn), _ptr(al), _ptr(db),
                            None if nb is None else _ptr(nb),
                            bx0, by0, bw, bh, int(opts.ssao_samples), float(opts.ssao_radius),
                            float(opts.ssao_bias), noise, int(opts.background) & 0xFFFFFFFF,
                            float(edge_px), float(depth_rel), int(getattr(opts, "shading", 0)),
                            float(getattr(opts, "fog_start", 0.0)), float(getattr(opts, "fog_end", 0.0)),
                            int(getattr(opts, "fog_color", 0)) & 0xFFFFFFFF,
                            float(getattr(opts, "outline_depth", 0.0)),
                            int(getattr(opts, "outline_color", 0)) & 0xFFFFFFFF,
                            None if amb is None else _ptr(amb), nthreads or default_threads(),
                            _ptr(rgba), _ptr(ao), _ptr(uns), _ptr(outside))
    if rc != 0:
        raise RuntimeError(f"osplat_shade failed: {rc}")
    return dict(rgba=rgba.reshape(h, w), ao=ao.reshape(h, w), ssao_unstable=uns.reshape(h, w),
                ssao_outside=outside.reshape(h, w))


def render(scene, cam, opts, W, H, window=None, halo=0, nthreads=None, edge_px=1e-3, depth_rel=1e-5):
    """G-buffer over the window grown by ``halo`` pixels, then SSAO + shading of the window."""
    if window is None:
        window = (0, 0, W, H)
    x0, y0, w, h = window
    gx0, gy0 = max(0, x0 - halo), max(0, y0 - halo)
    gx1, gy1 = min(W, x0 + w + halo), min(H, y0 + h + halo)
    gwin = (gx0, gy0, gx1 - gx0, gy1 - gy0)
    g = gbuffer(scene, cam, opts, W, H, gwin, nthreads)
    sl = (slice(y0 - gy0, y0 - gy0 + h), slice(x0 - gx0, x0 - gx0 + w))
    inner = {k: (np.ascontiguousarray(v[sl]) if isinstance(v, np.ndarray) and v.ndim >= 2 else v)
             for k, v in g.items()}
    from oracle.ofull import ambiguous_pixels
    sh = shade_gbuffer(cam, opts, W, H, window, inner["z"], inner["normal_view"], inner["albedo"],
                       depth_buf=g["z"], depth_win=gwin, nthreads=nthreads, edge_px=edge_px,
                       depth_rel=depth_rel, ambiguous=ambiguous_pixels(g), normal_buf=g["normal_view"])
    inner.update(sh)
    inner["view"] = (cam, W, H, window)
    return inner
