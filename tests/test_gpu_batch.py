"""Batched renders (vtx_render_batch): many jobs, one launch per pass.

Every job of a batch must give exactly the images the single-render entry
point gives for the same scene frame, camera and options, whatever else is in
the batch (needs an MI355X).
"""
import math

import numpy as np
import pytest

from oracle import compare, osplat
from paper_2501_12750_amd import scenes
from tests.gpu_util import assert_clean, run_render, with_opts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vtx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2501_12750_amd import vtx as v
    return v


@pytest.fixture(scope="module")
def ctx(vtx):
    c = vtx.vtx_context_create(0, 0)
    yield c
    vtx.vtx_context_destroy(c)


def run_batch(vtx, ctx, specs, stream=None):
    """specs: (scene handle, frame, camera, options, W, H); returns numpy images per job."""
    import torch
    frames = [vtx.Frame(W, H) for (_, _, _, _, W, H) in specs]
    jobs = [vtx.make_job(h, f, cam, opts, W, H, fr.rgba, fr.depth, fr.id)
            for (h, f, cam, opts, W, H), fr in zip(specs, frames)]
    vtx.vtx_render_batch(ctx, jobs, stream)
    torch.cuda.synchronize()
    return [fr.numpy() for fr in frames]


def assert_identical(a, b, what):
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs at {np.count_nonzero(a[k] != b[k])} pixels"


VIEWPORTS_SMALL = [(320, 180), (333, 221), (400, 225), (256, 144)]


def trajectory_scene(vtx, ctx, n_atoms, n_frames):
    import torch
    scene0, frames, cams, opts, _ = scenes.trajectory(n_atoms=n_atoms, n_frames=n_frames)
    rs = vtx.ResidentScene(ctx, vtx.DeviceScene(scene0))
    if n_frames > 1:
        first = rs.add_frames(torch.from_numpy(np.ascontiguousarray(frames[1:])).to("cuda"), n_frames - 1)
        assert first == 1
    assert rs.frames() == n_frames
    return scene0, frames, cams, opts, rs


def test_batch_trajectory_equals_single_renders(vtx, ctx):
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 5000, 6)
    specs = []
    for f in range(6):
        for k in range(4):
            W, H = VIEWPORTS_SMALL[(f + k) % 4]
            specs.append((rs.handle, f, cams[k], opts, W, H))
    got = run_batch(vtx, ctx, specs)
    for i, (_, f, cam, o, W, H) in enumerate(specs):
        sc_f = scenes.Scene(frames[f], scene0.radii, scene0.colors, scene0.bonds)
        ref = run_render(vtx, vtx.DeviceScene(sc_f), cam, o, W, H)
        assert_identical(got[i], ref, f"job {i} (frame {f})")
        assert np.count_nonzero(ref["id"] != 0xFFFFFFFF) > 1000
    rs.close()


def test_batch_refine_across_job_boundaries(vtx, ctx):
    """Jobs of one or two by two shade blocks, so that every refine workgroup
    (eight blocks) spans several jobs, with every pixel covered by atoms, so
    that marked winners fall on that path of the refine pass."""
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 5000, 3)
    c = frames[0].mean(axis=0)
    sizes = [(24, 24), (20, 28), (32, 16)]
    specs = []
    for f in range(3):
        for k in range(6):
            ang = 2.0 * math.pi * k / 6.0
            cam = scenes.Camera(eye=(c[0] + 40.0 * math.sin(ang), c[1] + 6.0, c[2] + 40.0 * math.cos(ang)),
                                target=tuple(c), fovy=math.radians(20.0))
            W, H = sizes[(f + k) % 3]
            specs.append((rs.handle, f, cam, opts, W, H))
    got = run_batch(vtx, ctx, specs)
    for i, (_, f, cam, o, W, H) in enumerate(specs):
        sc_f = scenes.Scene(frames[f], scene0.radii, scene0.colors, scene0.bonds)
        ref = run_render(vtx, vtx.DeviceScene(sc_f), cam, o, W, H)
        assert_identical(got[i], ref, f"job {i} (frame {f})")
        assert np.count_nonzero(ref["id"] == 0xFFFFFFFF) == 0, f"job {i}: background pixels"
    rs.close()


def _mixed_specs(vtx, ctx):
    bas = scenes.ball_and_stick(n_globules=27, atoms_per_globule=300, sigma=5.0, pitch=8.0,
                                width=333, height=221, ssao_samples=16)
    small = scenes.plain_small()
    ds_b, ds_s = vtx.DeviceScene(bas.scene), vtx.DeviceScene(small.scene)
    rs_b, rs_s = vtx.ResidentScene(ctx, ds_b), vtx.ResidentScene(ctx, ds_s)
    c = bas.camera.target
    ortho = scenes.Camera(eye=(c[0] + 5.0, c[1] + 60.0, c[2] + 7.0), target=c, up=(0, 0, 1),
                          projection=scenes.ORTHOGRAPHIC, ortho_half_height=14.0)
    specs = [
        (rs_b, ds_b, bas.camera, with_opts(bas.options, tile_size=8), 333, 221),
        (rs_s, ds_s, small.camera, small.options, 256, 256),
        (rs_b, ds_b, ortho, with_opts(bas.options, ssao_samples=8, tile_size=32), 200, 150),
        (rs_s, ds_s, small.camera, with_opts(small.options, ssao_samples=16, tile_size=32), 300, 200),
        (rs_b, ds_b, bas.camera, bas.options, 640, 360),
        (rs_b, ds_b, bas.camera, with_opts(bas.options, tile_size=64), 97, 61),
        (rs_s, ds_s, small.camera, with_opts(small.options, tile_size=8), 1, 1),
    ]
    return specs, (rs_b, rs_s)


def test_batch_mixed_scenes_tile_sizes_and_repeat(vtx, ctx):
    specs, keep = _mixed_specs(vtx, ctx)
    bspecs = [(rs.handle, 0, cam, o, W, H) for (rs, _, cam, o, W, H) in specs]
    refs = [run_render(vtx, ds, cam, o, W, H) for (_, ds, cam, o, W, H) in specs]
    for rep in range(2):                      # the second batch reuses the sized scratch
        got = run_batch(vtx, ctx, bspecs)
        for i in range(len(specs)):
            assert_identical(got[i], refs[i], f"round {rep} job {i}")
    # a smaller batch on the same stream, in another order
    order = [4, 0, 2]
    got = run_batch(vtx, ctx, [bspecs[i] for i in order])
    for j, i in enumerate(order):
        assert_identical(got[j], refs[i], f"reordered job {i}")
    for rs in keep:
        rs.close()


def test_batch_jobs_match_the_oracle(vtx, ctx):
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 3000, 3)
    specs = [(rs.handle, 2, cams[1], opts, 200, 150), (rs.handle, 0, cams[3], with_opts(opts, tile_size=8), 160, 120)]
    got = run_batch(vtx, ctx, specs)
    for i, (_, f, cam, o, W, H) in enumerate(specs):
        sc_f = scenes.Scene(frames[f], scene0.radii, scene0.colors, scene0.bonds)
        edge, drel = compare.e2e_bands_for(sc_f, cam, o, W, H)
        ref = osplat.render(sc_f, cam, o, W, H, edge_px=edge, depth_rel=drel)
        rep = compare.check_gbuffer(got[i]["depth"], got[i]["id"], ref)
        rep.update(compare.check_end_to_end(got[i]["rgba"], ref))
        print(f"job {i}", rep, flush=True)
        assert_clean(rep, f"job {i}")
        assert rep["hits"] > 1000
    rs.close()


def test_batch_overflowing_bins_stay_exact(vtx, ctx):
    import torch
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 4000, 2)
    specs = [(rs.handle, f, cams[k], opts, 320, 180) for f in range(2) for k in range(2)]
    ref = run_batch(vtx, ctx, specs)
    stream = torch.cuda.current_stream()
    vtx.vtx_set_bin_capacity(500, stream)
    try:
        got = run_batch(vtx, ctx, specs)
        st = vtx.vtx_read_stats(stream)
        assert st["overflow_tiles"] > 0
    finally:
        vtx.vtx_set_bin_capacity(0, stream)
    for i in range(len(specs)):
        assert_identical(got[i], ref[i], f"overflow job {i}")
    rs.close()


def test_batch_invalid_jobs(vtx, ctx):
    import torch
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 500, 2)
    fr = vtx.Frame(64, 64)
    good = vtx.make_job(rs.handle, 1, cams[0], opts, 64, 64, fr.rgba, fr.depth, fr.id)
    vtx.vtx_render_batch(ctx, [])                               # nothing to do
    cases = {
        "frame out of range": vtx.make_job(rs.handle, 2, cams[0], opts, 64, 64, fr.rgba, fr.depth, fr.id),
        "null output": vtx.make_job(rs.handle, 0, cams[0], opts, 64, 64, fr.rgba, None, fr.id),
        "null scene": vtx.make_job(None, 0, cams[0], opts, 64, 64, fr.rgba, fr.depth, fr.id),
        "bad size": vtx.make_job(rs.handle, 0, cams[0], opts, 0, 64, fr.rgba, fr.depth, fr.id),
    }
    for what, bad in cases.items():
        with pytest.raises(vtx.VtxError) as e:
            vtx.vtx_render_batch(ctx, [good, bad])
        assert e.value.code == vtx.VTX_EINVAL, what
        assert "job 1" in str(e.value), what
    other = vtx.vtx_context_create(0, 0)
    with pytest.raises(vtx.VtxError) as e:
        vtx.vtx_render_batch(other, [good])
    assert e.value.code == vtx.VTX_EINVAL
    vtx.vtx_context_destroy(other)
    # frames count against the context budget
    per = vtx.vtx_scene_frame_bytes(500, 0)
    used = vtx.vtx_context_bytes_in_use(ctx)
    tight = vtx.vtx_context_create(0, 0)
    rs2 = vtx.ResidentScene(tight, vtx.DeviceScene(scene0))
    base = rs2.info()["bytes"]
    assert base + per == rs.info()["bytes"]
    rs2.close()
    vtx.vtx_context_destroy(tight)
    small = vtx.vtx_context_create(0, base + per - 1)
    rs3 = vtx.ResidentScene(small, vtx.DeviceScene(scene0))
    pos = torch.from_numpy(np.ascontiguousarray(frames[1:2])).to("cuda")
    with pytest.raises(vtx.VtxError) as e:
        rs3.add_frames(pos, 1)
    assert e.value.code == vtx.VTX_EBUSY
    assert vtx.vtx_context_bytes_in_use(small) == base
    rs3.close()
    vtx.vtx_context_destroy(small)
    assert vtx.vtx_context_bytes_in_use(ctx) == used
    vtx.vtx_render_batch(ctx, [good])
    rs.close()


def test_batch_full_trajectory_sampled(vtx, ctx):
    """50,000 atoms x 64 frames x 4 orbit viewports (720p..1440p) = 256 jobs in
    one batch; a sample of jobs is compared with single renders."""
    import torch
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 50_000, 64)
    viewports = scenes.TRAJECTORY_VIEWPORTS
    specs = [(rs.handle, f, cams[k], opts) + tuple(viewports[k]) for f in range(64) for k in range(4)]
    imgs = [vtx.Frame(W, H) for (_, _, _, _, W, H) in specs]
    jobs = [vtx.make_job(h, f, cam, o, W, H, fr.rgba, fr.depth, fr.id)
            for (h, f, cam, o, W, H), fr in zip(specs, imgs)]
    vtx.vtx_render_batch(ctx, jobs)
    torch.cuda.synchronize()
    for i in (0, 1, 2, 3, 97, 130, 255):
        _, f, cam, o, W, H = specs[i]
        sc_f = scenes.Scene(frames[f], scene0.radii, scene0.colors, scene0.bonds)
        ref = run_render(vtx, vtx.DeviceScene(sc_f), cam, o, W, H)
        assert_identical(imgs[i].numpy(), ref, f"job {i}")
    rs.close()


def test_batch_graph_replays_match_eager_renders(vtx, ctx):
    """A captured batch replayed several times, with other eager work on the
    same stream between replays, gives the eager batch's images every time;
    replays follow updated trajectory positions written in place."""
    import torch
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 5000, 4)
    specs = [(rs.handle, f, cams[k], opts, *VIEWPORTS_SMALL[(f + k) % 4]) for f in range(4) for k in range(4)]
    ref = run_batch(vtx, ctx, specs)
    imgs = [vtx.Frame(W, H) for (_, _, _, _, W, H) in specs]
    jobs = [vtx.make_job(h, f, cam, o, W, H, fr.rgba, fr.depth, fr.id)
            for (h, f, cam, o, W, H), fr in zip(specs, imgs)]
    graph = vtx.vtx_batch_graph_create(ctx, jobs)
    other = scenes.plain_small()
    ds_other = vtx.DeviceScene(other.scene)
    try:
        for rep in range(4):
            for fr in imgs:
                fr.rgba.zero_()
                fr.depth.zero_()
                fr.id.zero_()
            vtx.vtx_batch_graph_launch(graph)
            run_render(vtx, ds_other, other.camera, other.options, 256, 256)   # eager work between replays
            torch.cuda.synchronize()
            for i, fr in enumerate(imgs):
                assert_identical(fr.numpy(), ref[i], f"replay {rep} job {i}")
        # frame 0 moved in place: the replay renders the new positions
        moved = np.ascontiguousarray(frames[3])
        rs.update_positions(torch.from_numpy(moved).to("cuda"))
        torch.cuda.synchronize()
        vtx.vtx_batch_graph_launch(graph)
        torch.cuda.synchronize()
        sc_moved = scenes.Scene(moved, scene0.radii, scene0.colors, scene0.bonds)
        for i, (_, f, cam, o, W, H) in enumerate(specs):
            if f == 0:
                assert_identical(imgs[i].numpy(), run_render(vtx, vtx.DeviceScene(sc_moved), cam, o, W, H),
                                 f"moved job {i}")
            else:
                assert_identical(imgs[i].numpy(), ref[i], f"unmoved job {i}")
    finally:
        vtx.vtx_batch_graph_destroy(graph)
    # a one-job graph (the job travels in the kernel arguments)
    _, f0, cam0, o0, W0, H0 = specs[0]
    assert f0 == 0
    imgs[0].id.zero_()
    single = vtx.vtx_batch_graph_create(ctx, jobs[:1])
    imgs[0].id.zero_()
    vtx.vtx_batch_graph_launch(single)
    torch.cuda.synchronize()
    assert_identical(imgs[0].numpy(), run_render(vtx, vtx.DeviceScene(sc_moved), cam0, o0, W0, H0), "one-job graph")
    vtx.vtx_batch_graph_destroy(single)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_batch_graph_create(ctx, [])
    rs.close()


def test_batch_graph_with_post_passes_clip_and_supersampling(vtx, ctx):
    """A captured batch whose jobs mix shading modes, fog, outline, a clip
    plane and supersampling (its full-size scratch sized by the eager render
    before capture) replays the eager batch's images, every replay."""
    import dataclasses
    import torch
    scene0, frames, cams, opts, rs = trajectory_scene(vtx, ctx, 5000, 2)
    c = np.zeros(3)
    variants = [dataclasses.replace(opts, shading=3, outline_color=scenes.pack_rgba(0, 0, 0), outline_depth=0.05),
                dataclasses.replace(opts, clip_plane=(1.0, 0.2, 0.0, 0.5)),
                dataclasses.replace(opts, supersample=2, fog_color=scenes.pack_rgba(200, 200, 220), fog_start=120.0,
                                    fog_end=170.0),
                dataclasses.replace(opts, shading=2, supersample=3)]
    specs = [(rs.handle, k % 2, cams[k % 4], variants[k], *VIEWPORTS_SMALL[k]) for k in range(4)]
    ref = run_batch(vtx, ctx, specs)
    # each job alone (single-render launches) draws the same image
    for i, (h, f, cam, o, W, H) in enumerate(specs):
        assert_identical(run_batch(vtx, ctx, [specs[i]])[0], ref[i], f"alone {i}")
    imgs = [vtx.Frame(W, H) for (_, _, _, _, W, H) in specs]
    jobs = [vtx.make_job(h, f, cam, o, W, H, fr.rgba, fr.depth, fr.id)
            for (h, f, cam, o, W, H), fr in zip(specs, imgs)]
    graph = vtx.vtx_batch_graph_create(ctx, jobs)
    try:
        for rep in range(3):
            for fr in imgs:
                fr.rgba.zero_()
                fr.id.zero_()
            vtx.vtx_batch_graph_launch(graph)
            torch.cuda.synchronize()
            for i, fr in enumerate(imgs):
                assert_identical(fr.numpy(), ref[i], f"replay {rep} job {i}")
    finally:
        vtx.vtx_batch_graph_destroy(graph)
