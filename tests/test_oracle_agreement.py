"""The two oracle implementations agree.

O-full evaluates every pixel against every primitive; O-splat restricts each
primitive to a conservative screen rectangle.  Equal results on the plain
small scene, on crops of ball-and-stick scenes and on adversarial footprints
(close-up spheres, primitives crossing the eye plane, off-axis wide-angle
views) show the rectangle is conservative and the two codes compute the same
definition.
"""
import math

import numpy as np
import pytest

from oracle import ofull, osplat
from paper_2501_12750_amd import scenes

BG = 0xFFFFFFFF


def assert_same(a, b, shading=False):
    assert a["fragments"] == b["fragments"]
    assert np.array_equal(a["acc_n"], b["acc_n"])
    assert np.array_equal(a["acc_bg"], b["acc_bg"])
    assert np.array_equal(a["id"], b["id"])
    fin = np.isfinite(a["z"])
    assert np.array_equal(fin, np.isfinite(b["z"]))
    assert np.all(np.abs(a["z"][fin] - b["z"][fin]) <= 1e-13 * a["z"][fin])
    assert np.allclose(a["normal_view"], b["normal_view"], rtol=0, atol=1e-11)
    assert np.array_equal(a["albedo"], b["albedo"])
    assert np.array_equal(a["unstable"], b["unstable"])
    # accept sets as sets
    sa = np.sort(np.where(np.arange(8)[None, None, :] < a["acc_n"][..., None], a["acc_id"], -1), axis=-1)
    sb = np.sort(np.where(np.arange(8)[None, None, :] < b["acc_n"][..., None], b["acc_id"], -1), axis=-1)
    assert np.array_equal(sa, sb)
    if shading:
        assert np.array_equal(a["rgba"], b["rgba"])
        assert np.allclose(a["ao"], b["ao"], rtol=0, atol=1e-12)
        assert np.array_equal(a["ssao_unstable"], b["ssao_unstable"])


@pytest.mark.slow
def test_plain_small_full_frame():
    wl = scenes.plain_small()
    a = ofull.gbuffer(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    b = osplat.gbuffer(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    assert_same(a, b)
    assert a["fragments"] > 100_000


def test_ball_and_stick_with_ssao():
    wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=200, sigma=4.0, pitch=6.0,
                               width=100, height=90, ssao_samples=16)
    a = ofull.render(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    b = osplat.render(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    assert_same(a, b, shading=True)
    assert np.any(a["id"] >= wl.scene.n_atoms) and np.any(a["id"] < wl.scene.n_atoms)
    assert np.any(a["ao"] < 1.0)


def test_crop_with_halo_equals_full_frame_region():
    wl = scenes.ball_and_stick(n_globules=27, atoms_per_globule=120, sigma=4.0, pitch=7.0,
                               width=160, height=120, ssao_samples=16)
    win = (57, 31, 40, 36)
    full = osplat.render(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    crop_o = ofull.render(wl.scene, wl.camera, wl.options, wl.width, wl.height, window=win, halo=24)
    crop_s = osplat.render(wl.scene, wl.camera, wl.options, wl.width, wl.height, window=win, halo=24)
    sl = (slice(win[1], win[1] + win[3]), slice(win[0], win[0] + win[2]))
    assert np.all(crop_s["ssao_outside"] == 0)
    for k in ("id", "acc_n", "albedo", "rgba", "ssao_unstable"):
        assert np.array_equal(crop_s[k], full[k][sl]), k
        assert np.array_equal(crop_o[k], full[k][sl]), k


def _adversarial(kind):
    rng = np.random.default_rng({"near": 11, "eyeplane": 12, "wide": 13}[kind])
    if kind == "near":
        # large spheres just in front of the camera, mostly off-axis
        c = rng.uniform([-6, -6, 2], [6, 6, 9], size=(40, 3))
        r = rng.uniform(0.5, 3.0, size=40)
        cam = scenes.Camera(eye=(0, 0, 12.0), target=(0, 0, 0), fovy=math.radians(70), znear=0.5)
    elif kind == "eyeplane":
        # primitives crossing the eye plane and the near plane
        c = rng.uniform([-8, -8, 6], [8, 8, 16], size=(40, 3))
        r = rng.uniform(0.5, 4.0, size=40)
        cam = scenes.Camera(eye=(0, 0, 12.0), target=(0, 0, 0), fovy=math.radians(60), znear=1.5)
    else:
        c = rng.uniform(-30, 30, size=(60, 3))
        r = rng.uniform(0.5, 2.5, size=60)
        cam = scenes.Camera(eye=(0, 0, 25.0), target=(5, -3, 0), fovy=math.radians(100), znear=0.5)
    n = c.shape[0]
    bonds = np.stack([np.arange(0, n - 1, 2), np.arange(1, n, 2)], axis=1).astype(np.uint32)
    sc = scenes.Scene(c.astype(np.float32), r.astype(np.float32),
                      scenes.ELEMENT_COLOR[rng.integers(0, 5, n)].astype(np.uint32), bonds)
    return sc, cam, scenes.Options(bond_radius=0.7, ssao_samples=8)


@pytest.mark.parametrize("kind", ["near", "eyeplane", "wide"])
def test_adversarial_footprints(kind):
    sc, cam, opts = _adversarial(kind)
    W, H = 72, 54
    a = ofull.render(sc, cam, opts, W, H)
    b = osplat.render(sc, cam, opts, W, H)
    assert_same(a, b, shading=True)
    assert np.count_nonzero(a["id"] != BG) > 200


def test_orthographic_scene():
    wl = scenes.ball_and_stick(n_globules=2, atoms_per_globule=150, sigma=3.0, pitch=5.0,
                               width=64, height=48, ssao_samples=8)
    c = np.asarray(wl.camera.target)
    cam = scenes.Camera(eye=(c[0] + 3.0, c[1] + 40.0, c[2] + 5.0), target=tuple(c), up=(0, 0, 1),
                        projection=scenes.ORTHOGRAPHIC, ortho_half_height=9.0)
    a = ofull.render(wl.scene, cam, wl.options, wl.width, wl.height)
    b = osplat.render(wl.scene, cam, wl.options, wl.width, wl.height)
    assert_same(a, b, shading=True)


@pytest.mark.parametrize("shading", [0, 1, 2, 3])
def test_post_passes_agree(shading):
    """Both oracles give the same image and the same unstable counts with a
    shading mode, fog and outline on, over a crop with a halo (the outline
    and SSAO read depths across the crop's edge)."""
    import dataclasses
    wl = scenes.ball_and_stick(n_globules=6, atoms_per_globule=200, sigma=4.0, pitch=6.0,
                               width=90, height=80, ssao_samples=8)
    c = np.asarray(wl.camera.eye, dtype=np.float64)
    t = np.asarray(wl.camera.target, dtype=np.float64)
    dist = float(np.linalg.norm(c - t))
    opts = dataclasses.replace(wl.options, representation=1, shading=shading, fog_color=scenes.pack_rgba(30, 60, 90),
                               fog_start=dist - 10.0, fog_end=dist + 10.0, outline_color=scenes.pack_rgba(5, 5, 5),
                               outline_depth=0.2)
    win = (20, 15, 40, 35)
    a = ofull.render(wl.scene, wl.camera, opts, wl.width, wl.height, window=win, halo=12)
    b = osplat.render(wl.scene, wl.camera, opts, wl.width, wl.height, window=win, halo=12)
    assert_same(a, b, shading=True)
    outline = a["rgba"] == (scenes.pack_rgba(5, 5, 5) | (255 << 24))
    assert outline.sum() > 10 and (~outline & (a["id"] != BG)).sum() > 30


def test_clip_plane_agrees():
    """Both oracles clip the same (primitive, pixel) hits, bonds included,
    with the same accept sets where a hit lies within rounding of the plane."""
    import dataclasses
    wl = scenes.ball_and_stick(n_globules=6, atoms_per_globule=200, sigma=4.0, pitch=6.0,
                               width=90, height=80, ssao_samples=8)
    c = np.asarray(wl.camera.target, dtype=np.float64)
    n = np.array([0.6, -0.3, 0.74])
    opts = dataclasses.replace(wl.options, clip_plane=(float(n[0]), float(n[1]), float(n[2]), float(-n @ c)))
    a = ofull.render(wl.scene, wl.camera, opts, wl.width, wl.height)
    b = osplat.render(wl.scene, wl.camera, opts, wl.width, wl.height)
    assert_same(a, b, shading=True)
    full = osplat.render(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    assert np.count_nonzero(a["id"] != full["id"]) > 200
    assert np.any(a["id"] >= wl.scene.n_atoms) and np.any((a["id"] < wl.scene.n_atoms))


def test_ssao_noise_agrees_full_frame_and_crop():
    """The noise form of SSAO (rotation and 4x4 blur): both oracles give the
    same AO, colours and unstable counts on a full frame, and a crop with a
    halo gives the full frame's values where its blur footprint is covered."""
    wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=200, sigma=4.0, pitch=6.0,
                               width=100, height=90, ssao_samples=16)
    opts = scenes.Options(**{**wl.options.__dict__, "ssao_noise": 1})
    a = ofull.render(wl.scene, wl.camera, opts, wl.width, wl.height)
    b = osplat.render(wl.scene, wl.camera, opts, wl.width, wl.height)
    assert_same(a, b, shading=True)
    plain = osplat.render(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    assert not np.array_equal(plain["ao"], b["ao"])
    win = (31, 22, 30, 28)
    crop = osplat.render(wl.scene, wl.camera, opts, wl.width, wl.height, window=win, halo=24)
    sl = (slice(win[1], win[1] + win[3]), slice(win[0], win[0] + win[2]))
    ok = crop["ssao_outside"] == 0
    assert ok.mean() > 0.9
    assert np.array_equal(crop["rgba"][ok], b["rgba"][sl][ok])
    assert np.allclose(crop["ao"][ok], b["ao"][sl][ok], rtol=0, atol=1e-12)
