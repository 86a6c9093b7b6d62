"""The resolve's depth early-outs on resident scenes (needs an MI355X).

A VTX_FLAG_STATS frame tests every (primitive, pixel) pair of every tile
list: no chunk cull, no early end of a layered list, no front-to-back
sub-chunks.  Its images are the plain z-buffer's, so a normal frame of the
same scene and camera (which culls, stops layered lists early and ends
front-to-back chunks at the depth-bucket bound) must match it bit for bit.
"""

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


@pytest.fixture(scope="module")
def ctx(vtx):
    c = vtx.vtx_context_create(0, 0)
    yield c
    vtx.vtx_context_destroy(c)


def workload(name):
    if name.startswith("cell"):
        wl = scenes.whole_cell(n_atoms=2_000_000, n_compartments=6, box=1500.0, r_min=250.0, r_max=400.0,
                               width=960, height=540, seed=5)
        tile = {"cell": 32, "cell_t16": 16, "cell_t64": 64, "cell_two_pass": 32}[name]
        wl.options = with_opts(wl.options, tile_size=tile)
        return wl
    if name == "globule":
        # large atoms, dozens deep per pixel: front-to-back sub-chunks
        scene0, _, cams, opts, _ = scenes.trajectory(n_atoms=50_000, n_frames=1)
        return scenes.Workload("globule", scene0, cams[1], with_opts(opts, tile_size=32), 2560, 1440)
    if name == "ball_and_stick":
        return scenes.ball_and_stick(n_globules=64, atoms_per_globule=400, sigma=6.0, pitch=14.0,
                                     width=640, height=360, ssao_samples=8)
    raise ValueError(name)


@pytest.mark.parametrize("name", ["cell", "cell_t16", "cell_t64", "cell_two_pass", "globule", "ball_and_stick"])
def test_early_outs_do_not_change_the_image(vtx, ctx, name):
    import torch
    wl = workload(name)
    ds = vtx.DeviceScene(wl.scene)
    rs = vtx.ResidentScene(ctx, ds)
    flags = vtx.VTX_FLAG_TWO_PASS if name == "cell_two_pass" else 0
    rs.render(wl.camera, wl.options, wl.width, wl.height)            # sizes the lists
    fast = rs.render(wl.camera, with_opts(wl.options, flags=flags), wl.width, wl.height)
    torch.cuda.synchronize()
    fast = fast.numpy()
    full = rs.render(wl.camera, with_opts(wl.options, flags=vtx.VTX_FLAG_STATS), wl.width, wl.height)
    torch.cuda.synchronize()
    st = vtx.vtx_read_stats()
    full = full.numpy()
    rs.close()
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(fast[k], full[k]), f"{name}: {k} differs at {np.count_nonzero(fast[k] != full[k])} pixels"
    hits = np.count_nonzero(full["id"] != 0xFFFFFFFF)
    depth_complexity = st["fragments_hit"] / max(1, hits)
    print(name, "hit pixels", hits, "fragments per hit pixel", round(depth_complexity, 2), flush=True)
    assert hits > 1000
    assert depth_complexity > 1.5      # enough overlap for the early-outs to have work


@pytest.mark.parametrize("name", ["cell", "globule"])
def test_early_outs_fire(vtx, ctx, name):
    """A VTX_FLAG_COUNT frame runs the same early-outs as a normal one and
    counts them: on the layered cell some tile lists end early, on the deep
    globule some depth-ordered chunks end at their bucket bound, and on both
    records are culled whole and covered pixels skip ray tests.  It draws the
    normal frame's image, and tests fewer fragments than a statistics frame."""
    import torch
    wl = workload(name)
    rs = vtx.ResidentScene(ctx, vtx.DeviceScene(wl.scene))
    normal = rs.render(wl.camera, wl.options, wl.width, wl.height)
    torch.cuda.synchronize()
    normal = normal.numpy()
    counted = rs.render(wl.camera, with_opts(wl.options, flags=vtx.VTX_FLAG_COUNT), wl.width, wl.height)
    torch.cuda.synchronize()
    st = vtx.vtx_read_stats()
    counted = counted.numpy()
    rs.render(wl.camera, with_opts(wl.options, flags=vtx.VTX_FLAG_STATS), wl.width, wl.height)
    torch.cuda.synchronize()
    full = vtx.vtx_read_stats()
    rs.close()
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(normal[k], counted[k]), k
    print(name, {k: st[k] for k in ("fragments_tested", "fragments_skipped", "records_culled", "lists_stopped",
                                    "chunks_stopped")}, "all", full["fragments_tested"], flush=True)
    assert 0 < st["fragments_tested"] < full["fragments_tested"]
    assert st["fragments_skipped"] > 0 and st["records_culled"] > 0
    if name == "cell":
        assert st["lists_stopped"] > 0
    else:
        assert st["chunks_stopped"] > 0
