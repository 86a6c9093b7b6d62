"""Device renderer vs the CPU oracle, through the C ABI (needs an MI355X).

Visibility (depth, id) is compared on every pixel with the accept-set rules;
normals and albedo at strict pixels; the deferred pass both cross-fed (oracle
SSAO + shading on the device's own G-buffer) and end to end.
"""
import math

import numpy as np
import pytest

from oracle import compare, osplat
from paper_2501_12750_amd import scenes
from tests.gpu_util import assert_clean, crop, run_device, run_render, windows, with_opts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vtx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2501_12750_amd import vtx as v
    return v


def full_parity(vtx, wl, check_shading=True, name=""):
    sc, cam, opts, W, H = wl.scene, wl.camera, wl.options, wl.width, wl.height
    ds = vtx.DeviceScene(sc)
    dev = run_device(vtx, ds, cam, opts, W, H)
    edge, drel = compare.e2e_bands_for(sc, cam, opts, W, H)
    ref = osplat.render(sc, cam, opts, W, H, edge_px=edge, depth_rel=drel)
    rep = compare.check_gbuffer(dev["depth"], dev["id"], ref)
    rep.update(compare.check_surface(dev["normal"], dev["albedo"], ref, sc, opts))
    if check_shading:
        rep.update(compare.check_shading_crossfed(cam, opts, W, H, dev))
        rep.update(compare.check_end_to_end(dev["rgba"], ref))
    print(name, f"bands {edge:.2e} px {drel:.2e}", rep, flush=True)
    assert_clean(rep, name)
    assert rep["strict"] > 0.9 * rep["pixels"]
    return dev, ref, rep


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_plain_small(vtx, tile):
    wl = scenes.plain_small()
    wl.options = with_opts(wl.options, tile_size=tile)
    dev, ref, rep = full_parity(vtx, wl, name=f"plain_small tile={tile}")
    assert rep["hits"] > 10000


def test_ball_and_stick_small_ragged(vtx):
    # 333 x 221: neither side a multiple of any tile size
    wl = scenes.ball_and_stick(n_globules=27, atoms_per_globule=300, sigma=5.0, pitch=8.0,
                               width=333, height=221, ssao_samples=16)
    dev, ref, rep = full_parity(vtx, wl, name="ball_and_stick_small")
    ids = dev["id"]
    assert np.any((ids >= wl.scene.n_atoms) & (ids != 0xFFFFFFFF)), "no bond visible"
    assert rep["shade_checked"] > 0.9 * rep["pixels"]


def test_orthographic(vtx):
    wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=300, sigma=4.0, pitch=6.0,
                               width=200, height=150, ssao_samples=8)
    c = wl.camera.target
    wl.camera = scenes.Camera(eye=(c[0] + 5.0, c[1] + 60.0, c[2] + 7.0), target=c, up=(0, 0, 1),
                              projection=scenes.ORTHOGRAPHIC, ortho_half_height=14.0)
    full_parity(vtx, wl, name="orthographic")


def _adversarial(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "near":
        c = rng.uniform([-6, -6, 2], [6, 6, 9], size=(60, 3))
        r = rng.uniform(0.5, 3.0, size=60)
        cam = scenes.Camera(eye=(0, 0, 12.0), target=(0, 0, 0), fovy=math.radians(70), znear=0.5)
    elif kind == "eyeplane":
        c = rng.uniform([-8, -8, 6], [8, 8, 16], size=(60, 3))
        r = rng.uniform(0.5, 4.0, size=60)
        cam = scenes.Camera(eye=(0, 0, 12.0), target=(0, 0, 0), fovy=math.radians(60), znear=1.5)
    else:
        c = rng.uniform(-30, 30, size=(400, 3))
        r = rng.uniform(0.5, 2.5, size=400)
        cam = scenes.Camera(eye=(0, 0, 25.0), target=(5, -3, 0), fovy=math.radians(100), znear=0.5)
    n = c.shape[0]
    bonds = np.stack([np.arange(0, n - 1, 2), np.arange(1, n, 2)], axis=1).astype(np.uint32)
    sc = scenes.Scene(c.astype(np.float32), r.astype(np.float32),
                      scenes.ELEMENT_COLOR[rng.integers(0, 5, n)].astype(np.uint32), bonds)
    return scenes.Workload(kind, sc, cam, scenes.Options(bond_radius=0.7, ssao_samples=8), 240, 180)


@pytest.mark.parametrize("kind", ["near", "eyeplane", "wide"])
def test_adversarial_footprints(vtx, kind):
    full_parity(vtx, _adversarial(kind, 21), name=kind)


def test_bin_overflow_is_exact(vtx):
    import torch
    wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=300, sigma=4.0, pitch=6.0,
                               width=256, height=192, ssao_samples=0)
    ds = vtx.DeviceScene(wl.scene)
    s = torch.cuda.Stream()
    base = run_device(vtx, ds, wl.camera, wl.options, wl.width, wl.height, aux=False, stream=s)
    st0 = vtx.vtx_read_stats(s)
    assert st0["overflow_tiles"] == 0
    vtx.vtx_set_bin_capacity(64, s)
    small = run_device(vtx, ds, wl.camera, wl.options, wl.width, wl.height, aux=False, stream=s)
    st1 = vtx.vtx_read_stats(s)
    vtx.vtx_set_bin_capacity(0, s)
    assert st1["overflow_tiles"] > 0 and st1["bin_capacity"] == 64
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(base[k], small[k]), k
    again = run_device(vtx, ds, wl.camera, wl.options, wl.width, wl.height, aux=False, stream=s)
    assert vtx.vtx_read_stats(s)["overflow_tiles"] == 0
    assert np.array_equal(base["id"], again["id"])


def test_permutation_and_determinism(vtx):
    wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=300, sigma=4.0, pitch=6.0,
                               width=300, height=200, ssao_samples=16)
    sc = wl.scene
    ds = vtx.DeviceScene(sc)
    a = run_render(vtx, ds, wl.camera, wl.options, wl.width, wl.height)
    b = run_render(vtx, ds, wl.camera, wl.options, wl.width, wl.height)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    rng = np.random.default_rng(5)
    pa, pb = rng.permutation(sc.n_atoms), rng.permutation(sc.n_bonds)
    sp = sc.permuted(pa, pb)
    c = run_render(vtx, vtx.DeviceScene(sp), wl.camera, wl.options, wl.width, wl.height)
    assert np.array_equal(a["depth"], c["depth"])
    N = sc.n_atoms
    ids = c["id"].astype(np.int64)
    mapped = np.where(ids == 0xFFFFFFFF, 0xFFFFFFFF,
                      np.where(ids < N, pa[np.minimum(ids, N - 1)], N + pb[np.clip(ids - N, 0, pb.size - 1)]))
    same = mapped == a["id"].astype(np.int64)
    # only exact depth ties may map differently
    assert same.mean() > 0.999


def test_edge_cases(vtx):
    import torch
    cam = scenes.Camera(eye=(0, 0, 30.0), target=(0, 0, 0))
    opts = scenes.Options(ssao_samples=4, background=scenes.pack_rgba(1, 2, 3, 4))
    # empty scene
    empty = scenes.Scene(np.zeros((0, 3), np.float32), np.zeros(0, np.float32), np.zeros(0, np.uint32),
                         np.zeros((0, 2), np.uint32))
    d = run_render(vtx, vtx.DeviceScene(empty), cam, opts, 37, 23)
    assert np.all(d["id"] == 0xFFFFFFFF) and np.all(np.isinf(d["depth"])) and np.all(d["rgba"] == opts.background)
    # 1 x 1 image, a single atom on the axis
    one = scenes.Scene(np.zeros((1, 3), np.float32), np.ones(1, np.float32),
                       np.array([scenes.ELEMENT_COLOR[0]], np.uint32), np.zeros((0, 2), np.uint32))
    d = run_render(vtx, vtx.DeviceScene(one), cam, opts, 1, 1)
    assert d["id"][0, 0] == 0 and abs(d["depth"][0, 0] - 29.0) <= 29.0 * 1e-5
    # every atom at one point: all tie, smallest id wins
    pile = scenes.Scene(np.full((5000, 3), 0.25, np.float32), np.full(5000, 2.0, np.float32),
                        np.full(5000, scenes.ELEMENT_COLOR[1], np.uint32), np.zeros((0, 2), np.uint32))
    d = run_render(vtx, vtx.DeviceScene(pile), cam, opts, 64, 64)
    hit = d["id"] != 0xFFFFFFFF
    assert hit.sum() > 20 and np.all(d["id"][hit] == 0)
    # bad and degenerate bonds: skipped, counted
    pos = np.array([[0, 0.1, 0], [0, 0.1, 0], [3, 0.1, 0]], np.float32)
    bonds = np.array([[0, 1], [1, 1], [0, 7], [0, 2]], np.uint32)
    sc = scenes.Scene(pos, np.full(3, 0.2, np.float32), np.full(3, scenes.ELEMENT_COLOR[2], np.uint32), bonds)
    s = torch.cuda.Stream()
    ds = vtx.DeviceScene(sc)
    fr = vtx.Frame(96, 64)
    vtx.vtx_render(*ds.args(), cam, with_opts(opts, bond_radius=0.5), 96, 64, fr.rgba, fr.depth, fr.id, s)
    st = vtx.vtx_read_stats(s)
    assert st["bad_bonds"] == 1
    ids = fr.numpy()["id"]
    assert np.any(ids == 3 + 3) and not np.any((ids >= 3) & (ids < 3 + 3))
    # camera inside a huge sphere sees through it
    inside = scenes.Scene(np.array([[0, 0, 30.0], [0, 0, 0]], np.float32), np.array([50.0, 1.0], np.float32),
                          np.full(2, scenes.ELEMENT_COLOR[0], np.uint32), np.zeros((0, 2), np.uint32))
    d = run_render(vtx, vtx.DeviceScene(inside), cam, opts, 48, 48)
    assert not np.any(d["id"] == 0) and np.any(d["id"] == 1)


def test_invalid_arguments_raise(vtx):
    wl = scenes.plain_small(n_atoms=10, width=8, height=8)
    ds = vtx.DeviceScene(wl.scene)
    fr = vtx.Frame(8, 8)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_render(*ds.args(), wl.camera, wl.options, 0, 8, fr.rgba, fr.depth, fr.id)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_render(*ds.args(), wl.camera, with_opts(wl.options, tile_size=12), 8, 8, fr.rgba, fr.depth, fr.id)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_render(*ds.args(), wl.camera, wl.options, 8, 8, None, fr.depth, fr.id)
    # a side above VTX_MAX_SIDE (16383) is refused even when the pixel count fits
    wide = vtx.Frame(16384, 2)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_render(*ds.args(), wl.camera, wl.options, 16384, 2, wide.rgba, wide.depth, wide.id)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_render(*ds.args(), wl.camera, with_opts(wl.options, supersample=2), 8192, 2, wide.rgba, wide.depth,
                       wide.id)


def test_fragment_count_matches_oracle(vtx):
    import torch
    wl = scenes.plain_small()
    opts = with_opts(wl.options, flags=vtx.VTX_FLAG_STATS)
    s = torch.cuda.Stream()
    ds = vtx.DeviceScene(wl.scene)
    fr = vtx.Frame(wl.width, wl.height)
    vtx.vtx_render(*ds.args(), wl.camera, opts, wl.width, wl.height, fr.rgba, fr.depth, fr.id, s)
    st = vtx.vtx_read_stats(s)
    ref = osplat.gbuffer(wl.scene, wl.camera, wl.options, wl.width, wl.height)
    assert abs(st["fragments_hit"] - ref["fragments"]) <= max(10, 1e-4 * ref["fragments"])
    assert st["fragments_tested"] >= st["fragments_hit"]
    # the early-outs do not change the image
    plain = run_render(vtx, ds, wl.camera, wl.options, wl.width, wl.height)
    assert np.array_equal(plain["id"], fr.numpy()["id"])


def test_ball_and_stick_full_size_sampled(vtx):
    """1M atoms + ~1.05M bonds at 1920x1080 with SSAO 16, in the benchmark's
    launch configuration; windows of the frame against the oracle's crops."""
    wl = scenes.ball_and_stick()
    sc, cam, opts, W, H = wl.scene, wl.camera, wl.options, wl.width, wl.height
    ds = vtx.DeviceScene(sc)
    dev = run_device(vtx, ds, cam, opts, W, H)
    rep_x = compare.check_shading_crossfed(cam, opts, W, H, dev)
    print("crossfed", rep_x, flush=True)
    assert_clean(rep_x, "crossfed")
    edge, drel = compare.e2e_bands_for(sc, cam, opts, W, H)
    for win in windows(W, H, 64, 6, seed=1) + [(W // 2 - 32, H // 2 - 32, 64, 64)]:
        ref = osplat.render(sc, cam, opts, W, H, window=win, halo=24, edge_px=edge, depth_rel=drel)
        dv = crop(dev, win)
        rep = compare.check_gbuffer(dv["depth"], dv["id"], ref)
        rep.update(compare.check_surface(dv["normal"], dv["albedo"], ref, sc, opts))
        rep.update(compare.check_end_to_end(dv["rgba"], ref))
        print(win, rep, flush=True)
        assert_clean(rep, str(win))


def test_whole_cell_100m(vtx):
    """The whole-cell scene the benchmark times: 10^8 atoms, 3840x2160, SSAO
    16, rendered through vtx_render_scene (a resident scene: the benchmark's
    launch form, at the tile size the library takes for 4K).  Checked:
      - bit-equal to vtx_render on the caller's arrays;
      - SSAO and shading of the whole frame cross-fed against the oracle;
      - eight 64^2 windows centred on hit pixels (G-buffer with a 64-pixel
        SSAO halo) against the oracle: ids, depth, normals, albedo, colours."""
    import torch
    wl = scenes.whole_cell()
    sc, cam, opts, W, H = wl.scene, wl.camera, wl.options, wl.width, wl.height
    print("whole cell:", sc.n_atoms, "atoms", flush=True)
    ds = vtx.DeviceScene(sc)
    ctx = vtx.vtx_context_create(0, 0)
    rs = vtx.ResidentScene(ctx, ds)
    fr = rs.render(cam, opts, W, H)
    torch.cuda.synchronize()
    dev = fr.numpy()
    plain = run_render(vtx, ds, cam, opts, W, H)
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(dev[k], plain[k]), k
    del plain
    # the deferred pass again on the scene's G-buffer, with its normals,
    # albedo and AO written out: the same colours
    aux = vtx.Frame(W, H, aux=True)
    aux.depth.copy_(fr.depth)
    aux.id.copy_(fr.id)
    vtx.vtx_shade(*ds.args(), cam, opts, W, H, aux.depth, aux.id, aux.rgba, aux.normal, aux.albedo, aux.ao)
    torch.cuda.synchronize()
    full = aux.numpy()
    assert np.array_equal(full["rgba"], dev["rgba"])
    rs.close()
    vtx.vtx_context_destroy(ctx)
    del ds, fr, aux
    hit = dev["id"] != 0xFFFFFFFF
    print("hit fraction", float(hit.mean()), flush=True)
    assert hit.mean() > 0.05
    rep_x = compare.check_shading_crossfed(cam, opts, W, H, full)
    print("crossfed", rep_x, "exempt fraction", rep_x["shade_exempt"] / (W * H), flush=True)
    assert_clean(rep_x, "crossfed")
    edge, drel = compare.e2e_bands_for(sc, cam, opts, W, H)
    print(f"e2e bands {edge:.3e} px, {drel:.3e}", flush=True)
    rng = np.random.default_rng(8)
    ys, xs = np.nonzero(hit)
    for k in rng.choice(ys.size, 8, replace=False):
        x0 = int(min(max(xs[k] - 32, 0), W - 64))
        y0 = int(min(max(ys[k] - 32, 0), H - 64))
        win = (x0, y0, 64, 64)
        ref = osplat.render(sc, cam, opts, W, H, window=win, halo=64, edge_px=edge, depth_rel=drel)
        dv = crop(full, win)
        rep = compare.check_gbuffer(dv["depth"], dv["id"], ref)
        rep.update(compare.check_surface(dv["normal"], dv["albedo"], ref, sc, opts))
        rep.update(compare.check_end_to_end(dv["rgba"], ref))
        print(win, rep, "exempt", rep["exempt"] / rep["pixels"], "e2e exempt",
              rep["e2e_exempt"] / rep["pixels"], flush=True)
        assert_clean(rep, str(win))
        assert rep["hits"] > 0


def test_max_image_8k(vtx):
    """7680 x 4320, the largest image the library accepts (the tile size is
    raised to 64 so the tile grid fits the binner); windows against the oracle."""
    wl = scenes.plain_small(n_atoms=20000, width=7680, height=4320)
    sc, cam, opts, W, H = wl.scene, wl.camera, wl.options, wl.width, wl.height
    dev = run_device(vtx, vtx.DeviceScene(sc), cam, opts, W, H)
    for win in windows(W, H, 64, 4, seed=3) + [(W // 2 - 40, H // 2 - 40, 80, 80), (W - 30, H - 20, 30, 20)]:
        ref = osplat.render(sc, cam, opts, W, H, window=win, halo=0)
        dv = crop(dev, win)
        rep = compare.check_gbuffer(dv["depth"], dv["id"], ref)
        rep.update(compare.check_surface(dv["normal"], dv["albedo"], ref, sc, opts))
        rep.update(compare.check_end_to_end(dv["rgba"], ref))
        assert_clean(rep, str(win))
    assert np.count_nonzero(dev["id"] != 0xFFFFFFFF) > 1e6


def test_tile_grid_past_8192_tiles(vtx):
    """2560 x 1440 at 16-pixel tiles: 14,400 tiles, so the list offsets scan
    every one of its 15 rows of 1024 tiles (the benchmark frames have 8,160);
    windows, the last tiles among them, against the oracle, and the resident
    scene's frame equal to vtx_render's."""
    import torch
    wl = scenes.plain_small(n_atoms=20000, width=2560, height=1440)
    sc, cam, W, H = wl.scene, wl.camera, wl.width, wl.height
    opts = with_opts(wl.options, tile_size=16)
    assert ((W + 15) // 16) * ((H + 15) // 16) == 14400
    ds = vtx.DeviceScene(sc)
    dev = run_device(vtx, ds, cam, opts, W, H)
    # windows on hits in the tiles past the first 8192 (tile rows 52 on)
    ys, xs = np.nonzero(dev["id"] != 0xFFFFFFFF)
    late = np.flatnonzero((ys // 16) * ((W + 15) // 16) + xs // 16 >= 8192)
    assert late.size > 1000
    picks = [late[0], late[late.size // 2], late[-1]]
    on_late = [(int(min(max(xs[k] - 32, 0), W - 64)), int(min(max(ys[k] - 32, 0), H - 64)), 64, 64) for k in picks]
    for win in windows(W, H, 64, 4, seed=5) + [(W // 2 - 32, H // 2 - 32, 64, 64), (W - 48, H - 40, 48, 40)] + on_late:
        ref = osplat.render(sc, cam, opts, W, H, window=win, halo=0)
        dv = crop(dev, win)
        rep = compare.check_gbuffer(dv["depth"], dv["id"], ref)
        rep.update(compare.check_surface(dv["normal"], dv["albedo"], ref, sc, opts))
        rep.update(compare.check_end_to_end(dv["rgba"], ref))
        print(win, {k: rep[k] for k in ("pixels", "hits", "id_bad", "depth_bad")}, flush=True)
        assert_clean(rep, str(win))
    assert np.count_nonzero(dev["id"] != 0xFFFFFFFF) > 1e5
    plain = run_render(vtx, ds, cam, opts, W, H)
    ctx = vtx.vtx_context_create(0, 0)
    try:
        rs = vtx.ResidentScene(ctx, ds)
        fr = rs.render(cam, opts, W, H)
        torch.cuda.synchronize()
        got = fr.numpy()
        rs.close()
    finally:
        vtx.vtx_context_destroy(ctx)
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(got[k], plain[k]), f"resident scene: {k} differs at {np.count_nonzero(got[k] != plain[k])} px"


def test_many_consecutive_frames_identical(vtx):
    """Back-to-back frames on one stream reuse the tile counts each frame
    re-arms for the next; 300 frames without synchronization must all
    reproduce the first frame bit for bit (tiles with several chunks)."""
    import torch
    wl = scenes.ball_and_stick(n_globules=64, atoms_per_globule=400, sigma=5.0, pitch=7.0,
                               width=640, height=480, ssao_samples=8)
    ds = vtx.DeviceScene(wl.scene)
    ref = run_render(vtx, ds, wl.camera, wl.options, wl.width, wl.height)
    frames = [vtx.Frame(wl.width, wl.height) for _ in range(4)]
    for i in range(300):
        fr = frames[i % 4]
        vtx.vtx_render(*ds.args(), wl.camera, wl.options, wl.width, wl.height, fr.rgba, fr.depth, fr.id)
    torch.cuda.synchronize()
    for fr in frames:
        d = fr.numpy()
        for k in ("rgba", "depth", "id"):
            assert np.array_equal(d[k], ref[k]), k


@pytest.mark.parametrize("rep", [1, 2, 3])
def test_representations(vtx, rep):
    """Van der Waals, sticks and solvent-accessible surface: the same kernels
    with other sphere radii and with or without the bonds."""
    wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=300, sigma=4.0, pitch=6.0,
                               width=240, height=160, ssao_samples=16)
    if rep != 2:
        # van der Waals radii for the spheres, so the representations differ
        el = np.random.default_rng(5).choice(5, size=wl.scene.n_atoms, p=scenes.ELEMENT_MIX)
        wl.scene = scenes.Scene(wl.scene.positions, np.ascontiguousarray(scenes.ELEMENT_VDW[el]),
                                wl.scene.colors, wl.scene.bonds)
    wl.options = with_opts(wl.options, representation=rep, probe_radius=1.4)
    dev, ref, rep_ = full_parity(vtx, wl, name=f"representation {rep}")
    ids = dev["id"]
    has_bonds = np.any((ids >= wl.scene.n_atoms) & (ids != 0xFFFFFFFF))
    assert has_bonds == (rep == 2)
    # the resident-scene path draws the same images
    ctx = vtx.vtx_context_create(0, 0)
    rs = vtx.ResidentScene(ctx, vtx.DeviceScene(wl.scene))
    import torch
    got = rs.render(wl.camera, wl.options, wl.width, wl.height).numpy()
    torch.cuda.synchronize()
    plain = run_render(vtx, vtx.DeviceScene(wl.scene), wl.camera, wl.options, wl.width, wl.height)
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(got[k], plain[k]), k
    rs.close()
    vtx.vtx_context_destroy(ctx)


@pytest.mark.parametrize("shading", [0, 1, 2, 3])
def test_post_passes(vtx, shading):
    """Shading modes, fog and outline (the deferred post-passes): the oracle
    shades the device's own G-buffer with the same options (cross-fed), and
    end to end without the outline (whose decision also reads neighbouring
    pixels' visibility)."""
    wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=300, sigma=4.0, pitch=6.0,
                               width=240, height=160, ssao_samples=16)
    el = np.random.default_rng(5).choice(5, size=wl.scene.n_atoms, p=scenes.ELEMENT_MIX)
    wl.scene = scenes.Scene(wl.scene.positions, np.ascontiguousarray(scenes.ELEMENT_VDW[el]),
                            wl.scene.colors, wl.scene.bonds)
    dist = float(np.linalg.norm(np.asarray(wl.camera.eye) - np.asarray(wl.camera.target)))
    fog = dict(fog_color=scenes.pack_rgba(40, 80, 160), fog_start=dist - 15.0, fog_end=dist + 15.0)
    wl.options = with_opts(wl.options, representation=1, shading=shading, **fog)
    dev, ref, rep = full_parity(vtx, wl, name=f"post shading={shading} fog")
    assert rep["shade_checked"] > 0.9 * rep["pixels"]
    # with the outline: cross-fed
    oc = scenes.pack_rgba(250, 250, 0)
    opts = with_opts(wl.options, outline_color=oc, outline_depth=0.2)
    dev = run_device(vtx, vtx.DeviceScene(wl.scene), wl.camera, opts, wl.width, wl.height)
    rx = compare.check_shading_crossfed(wl.camera, opts, wl.width, wl.height, dev)
    print("outline", rx, flush=True)
    assert rx["rgb_bad"] == 0 and rx["shade_checked"] > 0.9 * wl.width * wl.height
    drawn = np.asarray(dev["rgba"]) == (oc | (255 << 24))
    assert drawn.sum() > 100 and (~drawn & (np.asarray(dev["id"]) != 0xFFFFFFFF)).sum() > 1000


@pytest.mark.parametrize("proj", ["persp", "ortho"])
def test_clip_plane(vtx, proj):
    """A clip plane through the scene (bonds included): visibility against the
    oracle's accept sets, which admit either outcome within rounding of the
    plane, and the shading on top."""
    wl = scenes.ball_and_stick(n_globules=27, atoms_per_globule=300, sigma=5.0, pitch=8.0,
                               width=333, height=221, ssao_samples=16)
    c = np.asarray(wl.camera.target, dtype=np.float64)
    if proj == "ortho":
        e = np.asarray(wl.camera.eye, dtype=np.float64)
        wl.camera = scenes.Camera(eye=tuple(e), target=tuple(c), projection=scenes.ORTHOGRAPHIC,
                                  ortho_half_height=25.0)
    n = np.array([0.6, -0.3, 0.74])
    wl.options = with_opts(wl.options, clip_plane=(float(n[0]), float(n[1]), float(n[2]), float(-n @ c + 3.0)))
    dev, ref, rep = full_parity(vtx, wl, name=f"clip plane {proj}")
    base = run_render(vtx, vtx.DeviceScene(wl.scene), wl.camera, with_opts(wl.options, clip_plane=(0.0, 0.0, 0.0, 0.0)),
                      wl.width, wl.height)
    assert np.count_nonzero(dev["id"] != base["id"]) > 1000


@pytest.mark.parametrize("proj", ["persp", "ortho"])
def test_ssao_noise(vtx, proj):
    """The noise form of the ambient occlusion (per-pixel rotation from the
    4x4 Bayer table, 4x4 blur): cross-fed over the whole frame and end to end
    against the oracle; it differs from the plain form's image."""
    wl = scenes.ball_and_stick(n_globules=27, atoms_per_globule=300, sigma=5.0, pitch=8.0,
                               width=333, height=221, ssao_samples=16)
    if proj == "ortho":
        c = wl.camera.target
        wl.camera = scenes.Camera(eye=(c[0] + 5.0, c[1] + 60.0, c[2] + 7.0), target=c, up=(0, 0, 1),
                                  projection=scenes.ORTHOGRAPHIC, ortho_half_height=25.0)
    plain = run_render(vtx, vtx.DeviceScene(wl.scene), wl.camera, wl.options, wl.width, wl.height)
    wl.options = with_opts(wl.options, ssao_noise=1)
    dev, ref, rep = full_parity(vtx, wl, name=f"ssao noise {proj}")
    assert rep["shade_checked"] > 0.8 * rep["pixels"] and rep["e2e_checked"] > 0.7 * rep["pixels"]
    assert np.array_equal(plain["id"], dev["id"])
    assert np.count_nonzero(plain["rgba"] != dev["rgba"]) > 1000
