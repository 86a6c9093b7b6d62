"""Resident scenes (vtx_scene_*): the Morton-ordered, cluster-culled path must
render exactly what vtx_render renders for the same arrays (needs an MI355X)."""
import numpy as np
import pytest

from paper_2501_12750_amd import scenes
from tests.gpu_util import run_render
from tests.test_gpu_parity import _adversarial

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


def scene_render(vtx, ctx, wl):
    import torch
    ds = vtx.DeviceScene(wl.scene)
    rs = vtx.ResidentScene(ctx, ds)
    fr = rs.render(wl.camera, wl.options, wl.width, wl.height)
    torch.cuda.synchronize()
    out = fr.numpy()
    rs.close()
    return out, ds


def assert_identical(a, b, what):
    for k in ("depth", "id", "rgba"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs at {np.count_nonzero(a[k] != b[k])} pixels"


def _without_bonds(wl):
    """The same workload with its bonds dropped: a scene without bonds takes
    the count kernel's atom-only instantiation."""
    sc = wl.scene
    wl.scene = scenes.Scene(sc.positions, sc.radii, sc.colors, np.zeros((0, 2), np.uint32))
    return wl


@pytest.mark.parametrize("name", ["plain_small", "ball_and_stick_small", "orthographic", "near", "eyeplane", "wide",
                                  "orthographic_atoms", "near_atoms", "eyeplane_atoms", "wide_atoms"])
def test_scene_equals_plain_render(vtx, ctx, name):
    atoms_only = name.endswith("_atoms")
    name = name[:-len("_atoms")] if atoms_only else name
    if name == "plain_small":
        wl = scenes.plain_small()
    elif name == "ball_and_stick_small":
        wl = scenes.ball_and_stick(n_globules=27, atoms_per_globule=300, sigma=5.0, pitch=8.0,
                                   width=333, height=221, ssao_samples=16)
    elif name == "orthographic":
        wl = scenes.ball_and_stick(n_globules=8, atoms_per_globule=300, sigma=4.0, pitch=6.0,
                                   width=200, height=150, ssao_samples=8)
        c = wl.camera.target
        wl.camera = scenes.Camera(eye=(c[0] + 5.0, c[1] + 60.0, c[2] + 7.0), target=c, up=(0, 0, 1),
                                  projection=scenes.ORTHOGRAPHIC, ortho_half_height=14.0)
    else:
        wl = _adversarial(name, 21)
    if atoms_only:
        wl = _without_bonds(wl)
        assert wl.scene.n_bonds == 0
    print(name, "atoms only" if atoms_only else "", "atoms", wl.scene.n_atoms, "bonds", wl.scene.n_bonds, flush=True)
    got, ds = scene_render(vtx, ctx, wl)
    ref = run_render(vtx, ds, wl.camera, wl.options, wl.width, wl.height)
    assert_identical(got, ref, name)
    assert np.count_nonzero(ref["id"] != 0xFFFFFFFF) > 100


def test_scene_equals_plain_full_size(vtx, ctx):
    """1M atoms + ~1.05M bonds at 1080p with SSAO 16."""
    wl = scenes.ball_and_stick()
    got, ds = scene_render(vtx, ctx, wl)
    ref = run_render(vtx, ds, wl.camera, wl.options, wl.width, wl.height)
    assert_identical(got, ref, "ball_and_stick 1M")


def test_scene_equals_plain_whole_cell_10m(vtx, ctx):
    wl = scenes.whole_cell(n_atoms=10_000_000)
    got, ds = scene_render(vtx, ctx, wl)
    ref = run_render(vtx, ds, wl.camera, wl.options, wl.width, wl.height)
    assert_identical(got, ref, "whole cell 10M")


def test_scene_trajectory_updates(vtx, ctx):
    import torch
    scene0, frames, cams, opts, viewports = scenes.trajectory(n_atoms=5000, n_frames=4)
    ds = vtx.DeviceScene(scene0)
    rs = vtx.ResidentScene(ctx, ds)
    W, H = viewports[0]
    for t in (1, 3):
        pos = torch.from_numpy(frames[t]).to("cuda")
        rs.update_positions(pos)
        got = rs.render(cams[t % 4], opts, W, H).numpy()
        sc_t = scenes.Scene(frames[t], scene0.radii, scene0.colors, scene0.bonds)
        ref = run_render(vtx, vtx.DeviceScene(sc_t), cams[t % 4], opts, W, H)
        torch.cuda.synchronize()
        assert_identical(got, ref, f"trajectory frame {t}")
    rs.close()


def test_scene_budget_and_bad_bonds(vtx):
    wl = scenes.ball_and_stick(n_globules=2, atoms_per_globule=200, sigma=3.0, pitch=5.0, width=64, height=64)
    need = vtx.vtx_scene_footprint_bytes(wl.scene.n_atoms, wl.scene.n_bonds)
    assert need > 0
    small = vtx.vtx_context_create(0, need - 1)
    ds = vtx.DeviceScene(wl.scene)
    with pytest.raises(vtx.VtxError) as e:
        vtx.ResidentScene(small, ds)
    assert e.value.code == vtx.VTX_EBUSY
    assert vtx.vtx_context_bytes_in_use(small) == 0
    vtx.vtx_context_destroy(small)
    fits = vtx.vtx_context_create(0, need)
    bonds = wl.scene.bonds.copy()
    bonds[0, 1] = wl.scene.n_atoms + 5            # out of range: dropped
    sc = scenes.Scene(wl.scene.positions, wl.scene.radii, wl.scene.colors, bonds)
    rs = vtx.ResidentScene(fits, vtx.DeviceScene(sc))
    info = rs.info()
    assert info["bad_bonds"] == 1 and info["bytes"] == need
    assert vtx.vtx_context_bytes_in_use(fits) == need
    rs.close()
    assert vtx.vtx_context_bytes_in_use(fits) == 0
    vtx.vtx_context_destroy(fits)
