"""The C-ABI library loads and exports every entry point include/vtx.h
declares, and its host-side argument checks reject bad calls before any
device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vtx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vtx_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def vtx():
    from paper_2501_12750_amd import vtx as v
    return v


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("vtx_render", "vtx_gbuffer", "vtx_shade", "vtx_read_stats", "vtx_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(vtx):
    lib = ctypes.CDLL(vtx.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(vtx.EXPORTS)


def test_library_is_built_for_gfx950(vtx):
    data = open(vtx.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_version(vtx):
    assert "gfx950" in vtx.vtx_version()


def _cam():
    from paper_2501_12750_amd import scenes, vtx as v
    return v.camera_struct(scenes.Camera(eye=(0, 0, 10.0), target=(0, 0, 0)))


@pytest.mark.parametrize("case", ["W0", "toolarge", "nullpos", "nullout", "badtile", "badproj", "znear",
                                  "eye_eq_target", "up_parallel", "ssao", "negn"])
def test_host_argument_checks(vtx, case):
    from paper_2501_12750_amd import scenes
    cam = _cam()
    opt = vtx.options_struct(scenes.Options())
    W, H, n, pos, out = 16, 16, 4, 0x1000, 0x2000
    if case == "W0":
        W = 0
    elif case == "toolarge":
        W, H = 8000, 5000
    elif case == "nullpos":
        pos = None
    elif case == "nullout":
        out = None
    elif case == "badtile":
        opt.tile_size = 12
    elif case == "badproj":
        cam.projection = 7
    elif case == "znear":
        cam.znear = 0.0
    elif case == "eye_eq_target":
        cam.target[:] = list(cam.eye)
    elif case == "up_parallel":
        cam.up[:] = [0.0, 0.0, 1.0]
    elif case == "ssao":
        opt.ssao_samples = 65
    elif case == "negn":
        n = -1
    with pytest.raises(vtx.VtxError) as e:
        vtx.vtx_render(pos, 0x3000, 0x4000, n, None, 0, cam, opt, W, H, out, 0x5000, 0x6000, stream=0)
    assert e.value.code == vtx.VTX_EINVAL
    assert vtx.vtx_last_error()
