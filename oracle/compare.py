"""Parity rules between a device frame and the oracle (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's parity sample.  The device results enter as plain NumPy arrays.

Rules:
  id      bit-exact where the oracle's accept set is a single answer; a member
          of the accept set elsewhere (depth ties within TAU z, grazing hits).
  depth   |z_dev - z_ref(id_dev)| <= 1e-5 z_ref wherever the device reports
          a hit.
  albedo  bit-exact at strict pixels whose winner's shading is stable.
  normal  angle <= 1e-3 + normal_fp32_bound at strict, stable pixels.  The
          bound is that of the deferred pass's reconstruction: it takes the
          surface point z D on the pixel's ray in FP64 from the stored FP32
          depth (off by at most u z, u = 2^-24, so the point by u t, t the
          hit's distance along the unit ray), subtracts the primitive's FP64
          position and rounds the difference (u r) before normalising in FP32
          (a few u of direction): the angle is at most u (t / r + 3), taken
          twice over.  r is the sphere or cylinder radius.
  rgb     each channel within 1/255 at strict, stable pixels whose SSAO
          samples are all stable; end to end, the edge band and depth band
          within which a sample counts as unstable come from e2e_bands.
"""
from __future__ import annotations

import numpy as np

from . import ofull

BG = 0xFFFFFFFF
DEPTH_RTOL = 1e-5
EPS32 = 2.0 ** -24


def _u32(a):
    a = np.asarray(a)
    if a.dtype == np.int32:
        a = a.view(np.uint32)
    return a.astype(np.int64)


def check_gbuffer(dev_depth, dev_id, ref):
    """Visibility parity over a window: returns a report dict (counts)."""
    gid = _u32(dev_id)
    gz = np.asarray(dev_depth, dtype=np.float64)
    n = ref["acc_n"]
    slots = np.arange(ref["acc_id"].shape[-1])[None, None, :] < np.minimum(n, ref["acc_id"].shape[-1])[..., None]
    match = (ref["acc_id"] == gid[..., None]) & slots
    member = match.any(axis=-1)
    is_bg = gid == BG
    overflow = n > ref["acc_id"].shape[-1]
    ok_id = np.where(is_bg, ref["acc_bg"], member) | overflow
    strict = ((n == 1) & ~ref["acc_bg"]) | ((n == 0) & ref["acc_bg"])
    strict_bad = strict & (gid != ref["id"])
    zref = np.where(match, ref["acc_z"], np.inf).min(axis=-1)
    hit = ~is_bg & member
    zerr = np.zeros_like(gz)
    zerr[hit] = np.abs(gz[hit] - zref[hit]) / zref[hit]
    depth_bad = hit & (zerr > DEPTH_RTOL)
    bg_depth_bad = is_bg & np.isfinite(gz)
    return dict(pixels=int(gid.size), strict=int(strict.sum()), exempt=int((~strict).sum()),
                id_bad=int((~ok_id).sum()), strict_id_bad=int(strict_bad.sum()),
                depth_bad=int(depth_bad.sum()) + int(bg_depth_bad.sum()),
                max_depth_rel=float(zerr.max()) if zerr.size else 0.0,
                accept_overflow=int(overflow.sum()), hits=int((~is_bg).sum()))


def primitive_radius(scene, opts, ids):
    from oracle.ofull import representation_scene
    scene = representation_scene(scene, opts)
    ids = np.asarray(ids, dtype=np.int64)
    r = np.full(ids.shape, float(opts.bond_radius))
    atom = ids < scene.n_atoms
    r[atom] = scene.radii[ids[atom]]
    return r


def ray_distance(ref):
    """Distance along the unit pixel ray from its origin to depth ref["z"]
    (perspective: z |D| with D = (ndx tx, ndy ty, 1); orthographic: z)."""
    cam, W, H, window = ref["view"]
    x0, y0, w, h = window
    z = np.where(np.isfinite(ref["z"]), ref["z"], 0.0)
    if cam.projection != 0:
        return z
    th = np.tan(cam.fovy / 2.0)
    nx = 2.0 * (np.arange(x0, x0 + w) + 0.5) / W - 1.0
    ny = 1.0 - 2.0 * (np.arange(y0, y0 + h) + 0.5) / H
    D = np.sqrt(1.0 + (nx[None, :] * th * W / H) ** 2 + (ny[:, None] * th) ** 2)
    return z * D


def normal_fp32_bound(ref, r):
    """Largest angle (radians) between the device's normal and the exact one
    that the FP32 depth and normal rounding allow at each pixel (see the rules
    above): 2 u (t / r + 3)."""
    return 2.0 * EPS32 * (ray_distance(ref) / r + 3.0)


def check_surface(dev_normal, dev_albedo, ref, scene, opts):
    """Normal and albedo parity at strict, shading-stable pixels."""
    strict = (ref["acc_n"] == 1) & ~ref["acc_bg"] & ~ref["unstable"]
    gn = np.asarray(dev_normal, dtype=np.float64)
    rn = ref["normal_view"]
    cosang = np.clip(np.einsum("...k,...k->...", gn, rn) /
                     np.maximum(np.linalg.norm(gn, axis=-1) * np.linalg.norm(rn, axis=-1), 1e-300), -1.0, 1.0)
    ang = np.arccos(cosang)
    r = primitive_radius(scene, opts, np.where(strict, ref["id"], 0))
    tol = 1e-3 + normal_fp32_bound(ref, r)
    normal_bad = strict & (ang > tol)
    alb_bad = strict & (_u32(dev_albedo) != ref["albedo"].astype(np.int64))
    return dict(surface_checked=int(strict.sum()), normal_bad=int(normal_bad.sum()),
                max_normal_angle=float(ang[strict].max()) if strict.any() else 0.0,
                albedo_bad=int(alb_bad.sum()))


def e2e_bands(cam, opts, W, H, r_min, z_min, z_max=None):
    """(edge_px, depth_rel): the bands within which an SSAO sample of the
    end-to-end check counts as unstable, from the FP32 error of the device's
    sample position against the oracle's.

    r_min is the smallest sphere or cylinder radius drawn, z_min the nearest
    hit depth (z_max the farthest, orthographic views only).  The device
    builds a sample from the pixel's point P in FP32 (ndx, its product with
    tan and with z each rounded: |dP| <= 8 u z (tx + ty)) and from its FP32
    normal, off by at most dn = 2 u (t / r + 3) (normal_fp32_bound, t <= z
    |D|max), through the normal's branchless basis: with a = 1 / (1 - |n_z|)
    in [1/2, 1] the derivatives of T and B are at most 3, so the offset
    direction h.x T + h.y B + h.z n moves by at most 5 dn, and the sample by
    5 R dn.  Projected with focal length f pixels at depth Sz >= z - R, a
    move dS shifts the sample's pixel coordinates by at most
    (1 + tx) f |dS| / Sz.  Orthographic views project with f = (H/2)/h,
    independent of depth, so the normal term takes z_max.  The depth band
    adds the stored depths' own rounding (u each side) to the sample's move
    along z.  Both bands are at least the stated ones (1e-3 px, 1e-5)."""
    u = EPS32
    R = float(opts.ssao_radius)
    if cam.projection == 0:
        th = float(np.tan(cam.fovy / 2.0))
        tx, ty = th * W / H, th
        Dmax = float(np.sqrt(1.0 + tx * tx + ty * ty))
        f = (H / 2.0) / th
        # z / Sz: a sample at most R nearer than its pixel (samples at or
        # behind the near plane are not tested)
        near = 1.0 + R / max(z_min - R, float(cam.znear))
        dn_per_z = 2.0 * u * (Dmax / r_min + 3.0 / z_min)     # dn / z
        pos_px = (1.0 + tx) * f * near * 8.0 * u * (tx + ty)
        nrm_px = (1.0 + tx) * f * near * 5.0 * R * dn_per_z
        nrm_rel = 5.0 * R * dn_per_z * near
    else:
        f = (H / 2.0) / float(cam.ortho_half_height)
        dn = 2.0 * u * (float(z_max) / r_min + 3.0)
        pos_px = 8.0 * u * (W + H) / 2.0
        nrm_px = f * 5.0 * R * dn
        nrm_rel = 5.0 * R * dn / z_min
    edge_px = 1e-3 + pos_px + nrm_px
    depth_rel = 1e-5 + 4.0 * u + nrm_rel
    return edge_px, depth_rel


def e2e_bands_for(scene, cam, opts, W, H):
    """e2e_bands for a scene: the smallest radius the representation draws and
    the depth range of its primitives in front of the camera."""
    from oracle.ofull import camera_frame, representation_scene
    sc = representation_scene(scene, opts)
    radii = sc.radii.astype(np.float64)
    r_min = float(radii[radii > 0].min()) if sc.n_atoms else 1.0
    if sc.n_bonds:
        r_min = min(r_min, float(opts.bond_radius))
    e, s, u, f = camera_frame(cam)
    # depth range of the atoms whose sphere can reach the view volume (its
    # half-widths grown by the radius times the slant of its planes); a
    # bound for the bands only, so FP32 and 1e-3 of slack are enough
    z_min, z_max = np.inf, -np.inf
    basis = np.stack([s, u, f], axis=1).astype(np.float32)
    step = 1 << 24
    for k in range(0, sc.n_atoms, step):
        rel = sc.positions[k:k + step].astype(np.float32) - e.astype(np.float32)[None, :]
        v = rel @ basis
        x, y, z = v[:, 0], v[:, 1], v[:, 2]
        rr = radii[k:k + step].astype(np.float32) * np.float32(1.001)
        if cam.projection == 0:
            th = float(np.tan(cam.fovy / 2.0))
            tx, ty = th * W / H, th
            inside = ((np.abs(x) <= tx * z + rr * np.sqrt(1 + tx * tx) + 1e-3 * np.abs(z)) &
                      (np.abs(y) <= ty * z + rr * np.sqrt(1 + ty * ty) + 1e-3 * np.abs(z)))
        else:
            hh = float(cam.ortho_half_height)
            inside = (np.abs(x) <= hh * W / H + rr + 1e-3) & (np.abs(y) <= hh + rr + 1e-3)
        inside &= (z + rr >= float(cam.znear)) & (z - rr <= float(cam.zfar))
        if inside.any():
            z_min = min(z_min, float((z - rr)[inside].min()) * (1 - 1e-3))
            z_max = max(z_max, float((z + rr)[inside].max()) * (1 + 1e-3))
    z_min = max(float(cam.znear), z_min if np.isfinite(z_min) else 0.0)
    z_max = max(z_min, z_max if np.isfinite(z_max) else 0.0)
    return e2e_bands(cam, opts, W, H, r_min, z_min, z_max)


def rgb_diff(a, b):
    a = _u32(a)
    b = _u32(b)
    return np.max(np.stack([np.abs(((a >> s) & 255) - ((b >> s) & 255)) for s in (0, 8, 16, 24)]), axis=0)


def check_shading_crossfed(cam, opts, W, H, dev, oracle_mod=None, nthreads=None):
    """SSAO + shading parity on the device's own G-buffer (full frame).

    dev: dict with depth, id, normal, albedo, rgba, ao as full W x H arrays.
    The oracle recomputes AO and colour from the device depth, normals and
    albedo, which isolates the deferred pass from visibility differences.
    """
    from . import osplat
    mod = oracle_mod or osplat
    z = np.asarray(dev["depth"], dtype=np.float64)
    win = (0, 0, W, H)
    kw = {"nthreads": nthreads} if mod is osplat else {}
    ref = mod.shade_gbuffer(cam, opts, W, H, win, z, np.asarray(dev["normal"], dtype=np.float64),
                            _u32(dev["albedo"]).astype(np.uint32), **kw)
    stable = ref["ssao_unstable"] == 0
    d = rgb_diff(dev["rgba"], ref["rgba"])
    bad = stable & (d > 1)
    ao_err = np.abs(np.asarray(dev["ao"], dtype=np.float64) - ref["ao"])
    return dict(shade_checked=int(stable.sum()), shade_exempt=int((~stable).sum()), rgb_bad=int(bad.sum()),
                max_rgb_diff_stable=int(d[stable].max()) if stable.any() else 0,
                max_ao_err_stable=float(ao_err[stable].max()) if stable.any() else 0.0)


def check_end_to_end(dev_rgba, ref):
    """RGB parity against the oracle's own end-to-end image over a window."""
    strict = (((ref["acc_n"] == 1) & ~ref["acc_bg"] & ~ref["unstable"]) | ((ref["acc_n"] == 0) & ref["acc_bg"]))
    stable = strict & (ref["ssao_unstable"] == 0) & (ref["ssao_outside"] == 0)
    d = rgb_diff(dev_rgba, ref["rgba"])
    bad = stable & (d > 1)
    return dict(e2e_checked=int(stable.sum()), e2e_exempt=int((~stable).sum()), e2e_bad=int(bad.sum()),
                max_rgb_diff=int(d[stable].max()) if stable.any() else 0)
