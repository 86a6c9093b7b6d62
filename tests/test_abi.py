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


def test_struct_layouts_match_the_header(vtx, tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct of the same name."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [vtx.vtx_camera, vtx.vtx_options, vtx.vtx_stats, vtx.vtx_job, vtx.vtx_tuning, vtx.vtx_completion,
               vtx.vtx_server_stats]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "vtx.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, f"{name}.{f}"


def test_ssao_auto_is_accepted_without_a_context(vtx):
    """VTX_SSAO_AUTO passes the host checks of the plain entry point (it
    means 16 samples there); a count above the maximum does not."""
    from paper_2501_12750_amd import scenes
    cam = _cam()
    opt = vtx.options_struct(scenes.Options())
    opt.ssao_samples = vtx.VTX_SSAO_AUTO
    # a null position array is reported after the option checks pass
    rc = vtx._lib.vtx_render(None, None, None, 4, None, 0, ctypes.byref(cam), ctypes.byref(opt), 16, 16,
                             ctypes.c_void_p(0x2000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x2000), None)
    assert rc == vtx.VTX_EINVAL and "NULL" in vtx.vtx_last_error()
    opt.ssao_samples = -2
    rc = vtx._lib.vtx_render(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), None, 4, None, 0, ctypes.byref(cam),
                             ctypes.byref(opt), 16, 16, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x2000),
                             ctypes.c_void_p(0x2000), None)
    assert rc == vtx.VTX_EINVAL and "ssao_samples" in vtx.vtx_last_error()


def test_constants_match_the_header(vtx, tmp_path):
    """Every integer constant the header #defines has the same value in the
    binding (the C compiler evaluates the header's side)."""
    import re
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = re.findall(r"^#define (VTX_[A-Z0-9_]+) ", open(os.path.join(ROOT, "include", "vtx.h")).read(), re.M)
    assert {"VTX_FLAG_ONE_PASS", "VTX_FLAG_TWO_PASS", "VTX_SSAO_AUTO"} <= set(names)
    lines = ['#include <stdio.h>', '#include "vtx.h"', "int main(void) {"]
    lines += [f'printf("{n} %lld\\n", (long long)({n}));' for n in names]
    lines.append("return 0; }")
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "consts"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = {out[i]: int(out[i + 1]) for i in range(0, len(out), 2)}
    missing = [n for n in names if not hasattr(vtx, n)]
    assert not missing, f"constants missing from the binding: {missing}"
    for n in names:
        want = got[n] & 0xFFFFFFFF if getattr(vtx, n) >= 0 else got[n]
        assert getattr(vtx, n) == want, n
