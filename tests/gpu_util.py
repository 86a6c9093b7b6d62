"""Shared helpers of the GPU tests: run the device renderer through the C ABI
and bring its outputs back as NumPy arrays."""
import numpy as np

from paper_2501_12750_amd import scenes


def run_device(vtx, dscene, cam, opts, W, H, aux=True, stream=None):
    """G-buffer then deferred pass; returns numpy dict (depth, id, rgba[, normal, albedo, ao])."""
    import torch
    fr = vtx.Frame(W, H, aux=aux)
    vtx.vtx_gbuffer(*dscene.args(), cam, opts, W, H, fr.depth, fr.id, stream)
    vtx.vtx_shade(*dscene.args(), cam, opts, W, H, fr.depth, fr.id, fr.rgba,
                  fr.normal if aux else None, fr.albedo if aux else None, fr.ao if aux else None, stream)
    torch.cuda.synchronize()
    return fr.numpy()


def run_render(vtx, dscene, cam, opts, W, H, stream=None):
    import torch
    fr = vtx.render(dscene, cam, opts, W, H, stream=stream)
    torch.cuda.synchronize()
    return fr.numpy()


def crop(d, win):
    x0, y0, w, h = win
    return {k: v[y0:y0 + h, x0:x0 + w] for k, v in d.items()}


def with_opts(opts, **kw):
    import dataclasses
    return dataclasses.replace(opts, **kw)


def windows(W, H, size, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        x0 = int(rng.integers(0, max(1, W - size)))
        y0 = int(rng.integers(0, max(1, H - size)))
        out.append((x0, y0, min(size, W - x0), min(size, H - y0)))
    return out


def assert_clean(rep, name=""):
    bad = {k: v for k, v in rep.items() if k.endswith("_bad") and v}
    assert not bad, f"{name}: {bad} / {rep}"


__all__ = ["run_device", "run_render", "crop", "with_opts", "windows", "assert_clean", "scenes"]
