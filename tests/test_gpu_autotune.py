"""vtx_autotune: the tile-size tuner and its cache (needs an MI355X)."""
import json

import numpy as np
import pytest

from paper_2501_12750_amd import scenes
from tests.gpu_util import with_opts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vtx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2501_12750_amd import vtx as v
    return v


def _setup(vtx, ctx, n_atoms=4000):
    import torch
    scene0, frames, cams, opts, _ = scenes.trajectory(n_atoms=n_atoms, n_frames=3)
    rs = vtx.ResidentScene(ctx, vtx.DeviceScene(scene0))
    rs.add_frames(torch.from_numpy(np.ascontiguousarray(frames[1:])).to("cuda"), 2)
    return rs, cams, opts


def _batch(vtx, ctx, rs, cams, opts, tile, W=480, H=270):
    import torch
    imgs = [vtx.Frame(W, H) for _ in range(6)]
    jobs = [vtx.make_job(rs.handle, i % 3, cams[i % 4], with_opts(opts, tile_size=tile), W, H,
                         fr.rgba, fr.depth, fr.id) for i, fr in enumerate(imgs)]
    vtx.vtx_render_batch(ctx, jobs)
    torch.cuda.synchronize()
    return jobs, [fr.numpy() for fr in imgs]


def test_autotune_chooses_caches_and_applies(vtx, tmp_path):
    ctx = vtx.vtx_context_create(0, 0)
    rs, cams, opts = _setup(vtx, ctx)
    jobs, ref = _batch(vtx, ctx, rs, cams, opts, 16)
    cache = tmp_path / "tuning.json"
    t = vtx.vtx_autotune(ctx, jobs, cache)
    print(t)
    assert t["tile_size"] in (8, 16, 32, 64) and not t["from_cache"]
    assert set(t["ms_by_tile"]) == {8, 16, 32, 64} and min(t["ms_by_tile"].values()) > 0
    assert t["ms_by_tile"][t["tile_size"]] == min(t["ms_by_tile"].values())
    entries = json.loads(cache.read_text())["vtx_tuning"]
    assert [e["tile_size"] for e in entries if e["key"] == t["key"]] == [t["tile_size"]]
    # the images do not depend on the tile size, tuned or explicit
    for tile in (0, 8, 32, 64):
        _, got = _batch(vtx, ctx, rs, cams, opts, tile)
        for a, b in zip(got, ref):
            for k in ("depth", "id", "rgba"):
                assert np.array_equal(a[k], b[k]), f"tile {tile}: {k}"
    # a second context reads the choice back without timing anything
    ctx2 = vtx.vtx_context_create(0, 0)
    t2 = vtx.vtx_autotune(ctx2, jobs, cache)
    assert t2["from_cache"] and t2["tile_size"] == t["tile_size"] and t2["key"] == t["key"]
    # another shape is added to the same file, the first entry kept
    jobs3, _ = _batch(vtx, ctx, rs, cams, opts, 16, W=200, H=120)
    t3 = vtx.vtx_autotune(ctx, jobs3, cache)
    assert not t3["from_cache"] and t3["key"] != t["key"]
    keys = {e["key"]: e["tile_size"] for e in json.loads(cache.read_text())["vtx_tuning"]}
    assert keys == {t["key"]: t["tile_size"], t3["key"]: t3["tile_size"]}
    rs.close()
    vtx.vtx_context_destroy(ctx)
    vtx.vtx_context_destroy(ctx2)


def test_autotune_rejects_bad_arguments(vtx):
    ctx = vtx.vtx_context_create(0, 0)
    with pytest.raises(vtx.VtxError) as e:
        vtx.vtx_autotune(ctx, [])
    assert e.value.code == vtx.VTX_EINVAL
    vtx.vtx_context_destroy(ctx)


def test_autotune_sizes_the_bins(vtx, tmp_path):
    """The tuner reserves 5/4 of a sample job's pairs (+1024) at the chosen
    tile size; renders of that shape then fit their lists."""
    import torch
    ctx = vtx.vtx_context_create(0, 0)
    rs, cams, opts = _setup(vtx, ctx)
    jobs, ref = _batch(vtx, ctx, rs, cams, opts, 16)
    t = vtx.vtx_autotune(ctx, jobs, tmp_path / "t.json")
    assert t["bin_capacity"] > 1024
    # the same batch at the tuned size, with statistics, on a fresh stream
    stream = torch.cuda.Stream()
    for j in jobs:
        j.options.tile_size = 0
        j.options.flags = vtx.VTX_FLAG_STATS
    with torch.cuda.stream(stream):
        vtx.vtx_render_batch(ctx, jobs, stream)
    stream.synchronize()
    st = vtx.vtx_read_stats(stream)
    print(t, st)
    assert st["overflow_tiles"] == 0
    assert st["pairs"] <= len(jobs) * (t["bin_capacity"] - 1024) * 4 // 5 + len(jobs)
    assert st["bin_capacity"] >= st["pairs"]
    entries = json.loads((tmp_path / "t.json").read_text())["vtx_tuning"]
    assert [e["bin_capacity"] for e in entries if e["key"] == t["key"]] == [t["bin_capacity"]]
    rs.close()
    vtx.vtx_context_destroy(ctx)


def test_autotune_picks_ssao_samples_within_a_budget(vtx, tmp_path):
    """Jobs that ask for VTX_SSAO_AUTO get the largest tried count whose
    time per render fits the budget; renders asking for it afterwards equal
    renders with that count given explicitly."""
    import torch
    ctx = vtx.vtx_context_create(0, 0)
    rs, cams, opts = _setup(vtx, ctx)
    auto = with_opts(opts, ssao_samples=vtx.VTX_SSAO_AUTO)
    jobs, _ = _batch(vtx, ctx, rs, cams, auto, 0)
    # no budget: 16 samples, nothing timed for them
    t0 = vtx.vtx_autotune(ctx, jobs)
    assert t0["ssao_samples"] == 16 and t0["ms_by_samples"] == {}
    # a generous budget: the most samples
    t1 = vtx.vtx_autotune(ctx, jobs, frame_budget_ms=1e6)
    assert t1["ssao_samples"] == 64 and list(t1["ms_by_samples"]) == [64]
    # a budget between the times of two counts: the larger count that fits
    t2 = vtx.vtx_autotune(ctx, jobs, frame_budget_ms=1e-6)
    assert t2["ssao_samples"] == 0 and set(t2["ms_by_samples"]) == set(vtx.SSAO_COUNTS)
    times = t2["ms_by_samples"]
    assert times[64] > times[0]
    # the budget as the tuner holds it (FP32), so that both sides compare the same value
    mid = float(np.float32(0.5 * (times[64] + times[0])))
    t3 = vtx.vtx_autotune(ctx, jobs, tmp_path / "s.json", frame_budget_ms=mid)
    fits = [k for k in vtx.SSAO_COUNTS if times[k] <= mid]
    print(times, t3)
    assert t3["ssao_samples"] in vtx.SSAO_COUNTS and t3["ms_by_samples"][t3["ssao_samples"]] <= mid
    assert all(t3["ms_by_samples"].get(k, 1e9) > mid for k in vtx.SSAO_COUNTS if k > t3["ssao_samples"])
    assert fits  # the cheapest count fits a budget above its own time
    # renders asking for the context's count equal explicit ones
    _, got = _batch(vtx, ctx, rs, cams, auto, 0)
    _, ref = _batch(vtx, ctx, rs, cams, with_opts(opts, ssao_samples=t3["ssao_samples"]), 0)
    for a, b in zip(got, ref):
        for k in ("depth", "id", "rgba"):
            assert np.array_equal(a[k], b[k]), k
    # the cache keeps the count; a second context reads it back untimed
    ctx2 = vtx.vtx_context_create(0, 0)
    t4 = vtx.vtx_autotune(ctx2, jobs, tmp_path / "s.json", frame_budget_ms=mid)
    assert t4["from_cache"] and t4["ssao_samples"] == t3["ssao_samples"] and t4["bin_capacity"] == t3["bin_capacity"]
    rs.close()
    vtx.vtx_context_destroy(ctx)
    vtx.vtx_context_destroy(ctx2)
