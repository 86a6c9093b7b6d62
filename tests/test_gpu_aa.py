"""Anti-aliasing by exact supersampling (options.supersample): the reduced
image equals the full-size render reduced, on every launch form, and matches
the oracle's supersampled render where all samples are decided (needs an
MI355X)."""
import numpy as np
import pytest

from oracle import compare, ofull, osplat
from paper_2501_12750_amd import scenes
from tests.gpu_util import run_render, with_opts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vtx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2501_12750_amd import vtx as v
    return v


def reduce(full, S):
    """Per output pixel: channel means rounded half up, nearest (depth, id)."""
    H, W = full["depth"].shape[0] // S, full["depth"].shape[1] // S
    blk = lambda a: a.reshape(H, S, W, S).transpose(0, 2, 1, 3).reshape(H, W, S * S)
    key = (blk(full["depth"].astype(np.float32).view(np.uint32)).astype(np.uint64) << np.uint64(32)) | \
        blk(full["id"].astype(np.uint32)).astype(np.uint64)
    best = key.min(axis=-1)
    n = S * S
    rgba = np.zeros((H, W), dtype=np.uint64)
    c = blk(full["rgba"].astype(np.uint64))
    for ch in range(4):
        rgba |= ((((c >> np.uint64(8 * ch)) & np.uint64(255)).sum(axis=-1) + np.uint64(n // 2)) // np.uint64(n)) \
            << np.uint64(8 * ch)
    return dict(depth=(best >> np.uint64(32)).astype(np.uint32).view(np.float32),
                id=(best & np.uint64(0xFFFFFFFF)).astype(np.uint32), rgba=rgba.astype(np.uint32))


def _scene():
    wl = scenes.ball_and_stick(n_globules=27, atoms_per_globule=300, sigma=5.0, pitch=8.0,
                               width=213, height=141, ssao_samples=16)
    return wl


@pytest.mark.parametrize("S", [2, 3])
def test_supersample_equals_the_reduced_full_size_render(vtx, S):
    import torch
    wl = _scene()
    ds = vtx.DeviceScene(wl.scene)
    W, H = wl.width, wl.height
    aa = run_render(vtx, ds, wl.camera, with_opts(wl.options, supersample=S), W, H)
    full = run_render(vtx, ds, wl.camera, wl.options, S * W, S * H)
    ref = reduce(full, S)
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(aa[k].view(np.uint32) if k == "depth" else aa[k],
                              ref[k].view(np.uint32) if k == "depth" else ref[k]), k
    # edges are blended: the image has colours the plain render lacks
    assert len(np.unique(aa["rgba"])) > len(np.unique(run_render(vtx, ds, wl.camera, wl.options, W, H)["rgba"]))
    # the resident-scene and batch forms, with a supersampled and a plain job
    ctx = vtx.vtx_context_create(0, 0)
    rs = vtx.ResidentScene(ctx, vtx.DeviceScene(wl.scene))
    got = rs.render(wl.camera, with_opts(wl.options, supersample=S), W, H).numpy()
    torch.cuda.synchronize()
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(got[k], aa[k]), k
    fa, fb = vtx.Frame(W, H), vtx.Frame(W, H)
    jobs = [vtx.make_job(rs.handle, 0, wl.camera, with_opts(wl.options, supersample=S), W, H, fa.rgba, fa.depth,
                         fa.id),
            vtx.make_job(rs.handle, 0, wl.camera, wl.options, W, H, fb.rgba, fb.depth, fb.id)]
    vtx.vtx_render_batch(ctx, jobs)
    torch.cuda.synchronize()
    plain = run_render(vtx, ds, wl.camera, wl.options, W, H)
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(fa.numpy()[k], aa[k]), k
        assert np.array_equal(fb.numpy()[k], plain[k]), k
    rs.close()
    vtx.vtx_context_destroy(ctx)


def test_supersample_matches_the_oracle(vtx):
    S = 2
    wl = _scene()
    W, H = wl.width, wl.height
    aa = run_render(vtx, vtx.DeviceScene(wl.scene), wl.camera, with_opts(wl.options, supersample=S), W, H)
    edge, drel = compare.e2e_bands_for(wl.scene, wl.camera, wl.options, S * W, S * H)
    hi = osplat.render(wl.scene, wl.camera, wl.options, S * W, S * H, edge_px=edge, depth_rel=drel)
    ref = ofull.supersample_reduce(hi, S)
    st = ref["stable"]
    assert st.sum() > 0.6 * W * H
    assert np.array_equal(aa["id"][st].astype(np.int64), ref["id"][st])
    fin = st & np.isfinite(ref["z"])
    assert np.all(np.abs(aa["depth"][fin] - ref["z"][fin]) <= 1e-5 * ref["z"][fin] + 1e-6)
    d = np.max(np.stack([np.abs(((aa["rgba"].astype(np.int64) >> s) & 255) - ((ref["rgba"].astype(np.int64) >> s) & 255))
                         for s in (0, 8, 16, 24)]), axis=0)
    print("supersample parity: stable", int(st.sum()), "max rgb diff", int(d[st].max()), flush=True)
    assert d[st].max() <= 1


def test_supersample_argument_checks(vtx):
    wl = _scene()
    ds = vtx.DeviceScene(wl.scene)
    with pytest.raises(vtx.VtxError):
        run_render(vtx, ds, wl.camera, with_opts(wl.options, supersample=5), 64, 64)
    with pytest.raises(vtx.VtxError):
        run_render(vtx, ds, wl.camera, with_opts(wl.options, supersample=2), 7680, 4320)
    fr = vtx.Frame(32, 32)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_gbuffer(*ds.args(), wl.camera, with_opts(wl.options, supersample=2), 32, 32, fr.depth, fr.id)
