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
