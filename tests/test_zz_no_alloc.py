"""vtx_render_static, the entry point that allocates nothing, against
vtx_render (needs an MI355X).

Both run the same kernels; vtx_render_static takes every scratch buffer from
one static device array.  Two calls in a row, the second with a smaller
input on the same array, must each give vtx_render's images bit for bit (the
integer outputs exactly; depth and colour too, since the arithmetic is the
same).  A frame whose scratch would not fit the array is refused, and a
frame whose tile lists outgrow it is still exact (resolved from the visible
lists).
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


def _pair(vtx, wl, opts=None):
    import torch
    opts = opts or wl.options
    ds = vtx.DeviceScene(wl.scene)
    ref = vtx.Frame(wl.width, wl.height)
    vtx.vtx_render(*ds.args(), wl.camera, opts, wl.width, wl.height, ref.rgba, ref.depth, ref.id)
    got = vtx.Frame(wl.width, wl.height)
    got.rgba.fill_(7)
    got.depth.fill_(-1.0)
    got.id.fill_(7)
    vtx.vtx_render_static(*ds.args(), wl.camera, opts, wl.width, wl.height, got.rgba, got.depth, got.id)
    torch.cuda.synchronize()
    return ref.numpy(), got.numpy()


def _same(ref, got, name):
    for k in ("id", "depth", "rgba"):
        assert np.array_equal(ref[k], got[k]), f"{name}: {k} differs at {np.count_nonzero(ref[k] != got[k])} pixels"


def test_static_equals_render_twice_then_smaller(vtx):
    big = scenes.ball_and_stick(n_globules=64, atoms_per_globule=400, sigma=6.0, pitch=14.0,
                                width=800, height=600, ssao_samples=16)
    small = scenes.plain_small(n_atoms=2000, width=333, height=221)
    for name, wl in (("big", big), ("big again", big), ("small", small)):
        ref, got = _pair(vtx, wl)
        _same(ref, got, name)
        assert np.count_nonzero(ref["id"] != 0xFFFFFFFF) > 1000, name


def test_static_full_size_ball_and_stick(vtx):
    """The 1M-atom, 1.04M-bond ball-and-stick frame at 1920x1080 fits the
    array and matches vtx_render."""
    wl = scenes.ball_and_stick()
    ref, got = _pair(vtx, wl)
    _same(ref, got, "ball_and_stick 1080p")


def test_static_refuses_frames_too_large(vtx):
    import torch
    wl = scenes.plain_small(n_atoms=8_000_000, width=64, height=64)
    ds = vtx.DeviceScene(wl.scene)
    fr = vtx.Frame(64, 64)
    with pytest.raises(vtx.VtxError) as e:
        vtx.vtx_render_static(*ds.args(), wl.camera, wl.options, 64, 64, fr.rgba, fr.depth, fr.id)
    assert e.value.code == vtx.VTX_EOVERFLOW and "static scratch" in str(e.value)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_render_static(*ds.args(), wl.camera, with_opts(wl.options, supersample=2), 64, 64,
                              fr.rgba, fr.depth, fr.id)
    torch.cuda.synchronize()
    # the array still works afterwards
    small = scenes.plain_small(n_atoms=500, width=64, height=48)
    ref, got = _pair(vtx, small)
    _same(ref, got, "after refusals")
