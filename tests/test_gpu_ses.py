"""The solvent excluded surface through the C ABI (vtx_ses) against the SES
oracle (needs an MI355X): the grid field bit for bit, and the triangles
(same count, same cubes and order, vertices within FP32 rounding)."""
import math

import numpy as np
import pytest

from oracle import oses
from paper_2501_12750_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vtx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2501_12750_amd import vtx as v
    return v


def grid_for(pos, rad, probe, h, pad=2):
    lo = np.min(pos - rad[:, None], axis=0) - probe - pad * h
    hi = np.max(pos + rad[:, None], axis=0) + probe + pad * h
    dims = tuple(int(d) for d in np.ceil((hi - lo) / h).astype(int) + 1)
    return lo.astype(np.float32), np.float32(h), dims


def run_ses(vtx, pos, rad, probe, origin, h, dims, capacity=None):
    import torch
    dp = torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float32)).cuda()
    dr = torch.from_numpy(np.ascontiguousarray(rad, dtype=np.float32)).cuda()
    field = torch.empty(dims[::-1], dtype=torch.float32, device="cuda")
    cap = capacity if capacity is not None else 4 * int(np.prod(dims))
    tri = torch.empty((max(cap, 1), 9), dtype=torch.float32, device="cuda")
    ntri = torch.zeros(1, dtype=torch.int64, device="cuda")
    vtx.vtx_ses(dp, dr, pos.shape[0], probe, origin, h, dims, field, tri, cap, ntri)
    torch.cuda.synchronize()
    n = int(ntri.item())
    return field.cpu().numpy(), tri[:min(n, cap)].cpu().numpy().reshape(-1, 3, 3), n


def check(vtx, pos, rad, probe, h, name):
    origin, hh, dims = grid_for(pos, rad, probe, h)
    ref = oses.ses_field(pos, rad, probe, origin, hh, dims)
    f, tri, n = run_ses(vtx, pos, rad, probe, origin, hh, dims)
    same = f == ref["f"]
    print(name, "grid", dims, "field equal", int(same.sum()), "of", f.size, flush=True)
    assert same.all(), f"{name}: field differs at {np.count_nonzero(~same)} points"
    mc = oses.marching_cubes(ref["f"], origin, hh)
    assert n == mc["vertices"].shape[0], (n, mc["vertices"].shape[0])
    err = np.abs(tri.astype(np.float64) - mc["vertices"])
    tol = 1e-5 * (np.abs(mc["vertices"]) + float(hh))
    print(name, "triangles", n, "max vertex error", float(err.max()) if n else 0.0, flush=True)
    assert np.all(err <= tol)
    return n


def test_ses_small_scenes(vtx):
    rng = np.random.default_rng(4)
    pos = rng.uniform(-3, 3, size=(12, 3)).astype(np.float32)
    rad = rng.uniform(1.0, 1.8, size=12).astype(np.float32)
    assert check(vtx, pos, rad, 1.4, 0.4, "random 12") > 100
    two = np.array([[-2.0, 0.0, 0.0], [2.0, 0.0, 0.0]], dtype=np.float32)
    assert check(vtx, two, np.array([1.5, 1.5], np.float32), 1.4, 0.1, "two-atom neck") > 1000
    one = np.array([[0.3, -0.2, 0.1]], dtype=np.float32)
    check(vtx, one, np.array([1.7], np.float32), 1.4, 0.25, "one atom")


def test_ses_protein_like_globule(vtx):
    scene0, _, _, _, _ = scenes.trajectory(n_atoms=6000, n_frames=1)
    n = check(vtx, scene0.positions, scene0.radii, 1.4, 0.5, "globule 6k")
    assert n > 10000


def test_ses_slab_many_atoms_per_plane(vtx):
    """A thin slab of 8k atoms on a 318 x 178 x 23 grid: thousands of atoms
    reach every z plane, and most grid points lie in several atoms' spheres."""
    rng = np.random.default_rng(7)
    n = 8000
    pos = np.stack([rng.uniform(-75, 75, n), rng.uniform(-40, 40, n), rng.uniform(-1, 1, n)], 1).astype(np.float32)
    rad = rng.uniform(1.2, 1.9, n).astype(np.float32)
    assert check(vtx, pos, rad, 1.4, 0.5, "slab 8k") > 10000


def test_ses_capacity_and_arguments(vtx):
    import torch
    one = np.array([[0.0, 0.0, 0.0]], dtype=np.float32)
    rad = np.array([2.0], np.float32)
    origin, h, dims = grid_for(one, rad, 1.4, 0.3)
    f, tri_all, n = run_ses(vtx, one, rad, 1.4, origin, h, dims)
    f2, tri_few, n2 = run_ses(vtx, one, rad, 1.4, origin, h, dims, capacity=10)
    assert n2 == n and tri_few.shape[0] == 10 and np.array_equal(tri_few, tri_all[:10])
    dp = torch.zeros((1, 3), dtype=torch.float32, device="cuda")
    dr = torch.ones(1, dtype=torch.float32, device="cuda")
    nt = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(vtx.VtxError):
        vtx.vtx_ses(dp, dr, 1, 1.4, (0, 0, 0), 0.0, (8, 8, 8), None, None, 0, nt)
    with pytest.raises(vtx.VtxError):
        vtx.vtx_ses(dp, dr, 1, 1.4, (0, 0, 0), 0.5, (1, 8, 8), None, None, 0, nt)
    # no atoms: every point outside, no triangles
    vtx.vtx_ses(None, None, 0, 1.4, (0, 0, 0), 0.5, (6, 6, 6), None, None, 0, nt)
    torch.cuda.synchronize()
    assert int(nt.item()) == 0
