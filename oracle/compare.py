"""Parity rules between a device frame and the oracle (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's parity sample.  The device results enter as plain NumPy arrays.

Rules (the tolerances and why they are what they are are stated in the design
notes):
  id      bit-exact where the oracle's accept set is a single answer; a member
          of the accept set elsewhere (depth ties within TAU z, grazing hits).
  depth   |z_dev - z_ref(id_dev)| <= DEPTH_RTOL z_ref + 16 eps32 z_ref / n.V
          wherever the device reports a hit.  The second term is the FP32
          conditioning of a ray-surface hit: a perturbation of a few ulps of
          the distance moves the hit along the ray by that much divided by
          the cosine n.V, which grows without bound at a silhouette.  It is
          below the first term wherever n.V > 0.1; the number of pixels where
          it is larger is reported as depth_conditioned.
  albedo  bit-exact at strict pixels whose winner's shading is stable.
  normal  angle <= 1e-3 + 64 eps32 z / (r n.V) at strict, stable pixels,
          where r is the primitive radius: the FP32 error of a hit point is
          a few ulps of its depth and it is amplified by 1 / (n.V) towards
          the silhouette.
  rgb     each channel within 1/255 at strict, stable pixels whose SSAO
          samples are all stable.
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
    cond = 16 * EPS32 / np.maximum(np.abs(ref["nv"]), 1e-3)
    depth_bad = hit & (zerr > DEPTH_RTOL + cond)
    conditioned = hit & (zerr > DEPTH_RTOL)
    bg_depth_bad = is_bg & np.isfinite(gz)
    return dict(pixels=int(gid.size), strict=int(strict.sum()), exempt=int((~strict).sum()),
                id_bad=int((~ok_id).sum()), strict_id_bad=int(strict_bad.sum()),
                depth_bad=int(depth_bad.sum()) + int(bg_depth_bad.sum()),
                max_depth_rel=float(zerr.max()) if zerr.size else 0.0,
                depth_conditioned=int(conditioned.sum()),
                accept_overflow=int(overflow.sum()), hits=int((~is_bg).sum()))


def primitive_radius(scene, opts, ids):
    from oracle.ofull import representation_scene
    scene = representation_scene(scene, opts)
    ids = np.asarray(ids, dtype=np.int64)
    r = np.full(ids.shape, float(opts.bond_radius))
    atom = ids < scene.n_atoms
    r[atom] = scene.radii[ids[atom]]
    return r


def check_surface(dev_normal, dev_albedo, ref, scene, opts):
    """Normal and albedo parity at strict, shading-stable pixels."""
    strict = (ref["acc_n"] == 1) & ~ref["acc_bg"] & ~ref["unstable"]
    gn = np.asarray(dev_normal, dtype=np.float64)
    rn = ref["normal_view"]
    cosang = np.clip(np.einsum("...k,...k->...", gn, rn) /
                     np.maximum(np.linalg.norm(gn, axis=-1) * np.linalg.norm(rn, axis=-1), 1e-300), -1.0, 1.0)
    ang = np.arccos(cosang)
    r = primitive_radius(scene, opts, np.where(strict, ref["id"], 0))
    tol = 1e-3 + 64 * EPS32 * np.where(np.isfinite(ref["z"]), ref["z"], 0.0) / (r * np.maximum(ref["nv"], 1e-6))
    normal_bad = strict & (ang > tol)
    alb_bad = strict & (_u32(dev_albedo) != ref["albedo"].astype(np.int64))
    return dict(surface_checked=int(strict.sum()), normal_bad=int(normal_bad.sum()),
                max_normal_angle=float(ang[strict].max()) if strict.any() else 0.0,
                albedo_bad=int(alb_bad.sum()))


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
