"""Pins of the SES oracle (solvent excluded surface on a grid + marching
cubes) against geometry and brute force, not against itself:
  * the case table: empty and full cubes, complement symmetry, closed and
    consistently oriented meshes on random fields;
  * marching cubes of an analytic sphere field: volume and outward normals;
  * the distance field: exact against brute force on a small scene; every
    grid point inside an atom is inside the SES, every probe-centre point is
    at -rp;
  * an isolated atom's SES is its sphere, within the grid's error bound;
  * two atoms closer than the probe can pass between: the neck radius of the
    toroidal patch, sqrt((r + rp)^2 - (d/2)^2) - rp, within the bound; two
    atoms the probe separates: no surface between them.
"""
import math
from collections import Counter

import numpy as np
import pytest

from oracle import oses

H_SQRT3 = math.sqrt(3.0)


def grid_for(centres, radii, probe, h, pad=2):
    lo = np.min(np.asarray(centres) - np.asarray(radii)[:, None], axis=0) - probe - pad * h
    hi = np.max(np.asarray(centres) + np.asarray(radii)[:, None], axis=0) + probe + pad * h
    dims = np.ceil((hi - lo) / h).astype(int) + 1
    return lo.astype(np.float32), np.float32(h), tuple(int(d) for d in dims)


def closed_and_oriented(verts):
    """Every undirected edge of the mesh is used twice, once per direction."""
    key = lambda p: tuple(np.round(p, 9))
    directed = Counter()
    for tri in verts:
        k = [key(p) for p in tri]
        for a, b in ((0, 1), (1, 2), (2, 0)):
            directed[(k[a], k[b])] += 1
    for (a, b), c in directed.items():
        if c != 1 or directed.get((b, a), 0) != 1:
            return False
    return True


def test_case_table_basics():
    t = oses.mc_table()
    assert len(t) == 256 and t[0] == [] and t[255] == []
    for m in range(256):
        crossing = {e for e, (a, b) in enumerate(oses.EDGES) if ((m >> a) & 1) != ((m >> b) & 1)}
        used = [e for lp in t[m] for e in lp]
        assert sorted(used) == sorted(crossing), m        # every crossing edge in exactly one loop
        assert sorted(e for lp in t[255 - m] for e in lp) == sorted(used), m
        assert all(len(lp) >= 3 for lp in t[m])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_fields_give_closed_oriented_meshes(seed):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(7, 8, 9)).astype(np.float32)
    f[0], f[-1], f[:, 0], f[:, -1], f[:, :, 0], f[:, :, -1] = -1, -1, -1, -1, -1, -1   # closed surfaces
    mc = oses.marching_cubes(f, (0.0, 0.0, 0.0), 1.0)
    assert mc["vertices"].shape[0] > 20
    assert closed_and_oriented(mc["vertices"])


def test_sphere_field_volume_and_normals():
    r, h = 5.0, 0.5
    c = np.array([0.13, -0.21, 0.07])
    n = int(2 * (r + 2) / h) + 1
    o = -np.array([r + 2, r + 2, r + 2])
    ax = [o[k] + h * np.arange(n) for k in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    f = (r - np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)).astype(np.float32)
    mc = oses.marching_cubes(f, o.astype(np.float32), h)
    v = mc["vertices"]
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    cen = v.mean(axis=1) - c
    assert np.all(np.einsum("ij,ij->i", nrm, cen) > 0)           # outward
    vol = np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])).sum() / 6.0
    assert abs(vol / (4.0 / 3.0 * math.pi * r ** 3) - 1.0) < 0.01
    assert closed_and_oriented(v)


def test_field_matches_brute_force_and_contains_vdw():
    rng = np.random.default_rng(4)
    pos = rng.uniform(-3, 3, size=(12, 3)).astype(np.float32)
    rad = rng.uniform(1.0, 1.8, size=12).astype(np.float32)
    probe, h = 1.4, 0.4
    o, h, dims = grid_for(pos, rad, probe, h)
    res = oses.ses_field(pos, rad, probe, o, h, dims)
    nx, ny, nz = dims
    kk, jj, ii = np.mgrid[0:nz, 0:ny, 0:nx]
    P = np.stack([o[0].astype(np.float64) + float(h) * ii, o[1].astype(np.float64) + float(h) * jj,
                  o[2].astype(np.float64) + float(h) * kk], axis=-1)
    d = np.linalg.norm(P[..., None, :] - pos.astype(np.float64)[None, None, None], axis=-1)
    R = rad.astype(np.float64) + float(np.float32(probe))
    exterior = np.all(d >= R, axis=-1)
    # the oracle's exterior may differ only on points within rounding of a sphere
    near = np.any(np.abs(d - R) < 1e-9, axis=-1)
    assert np.array_equal(res["exterior"][~near], exterior[~near])
    ext_idx = np.argwhere(res["exterior"])
    W = res["W"]
    for q in np.argwhere(~res["exterior"])[::7]:
        g = ((ext_idx - q) ** 2).sum(axis=1).min() if ext_idx.size else 10 ** 9
        want = g if g <= W * W else -1
        assert res["g"][tuple(q)] == want, q
    inside_vdw = np.any(d < rad.astype(np.float64), axis=-1)
    assert np.all(res["f"][inside_vdw] > 0)
    assert np.all(res["f"][res["exterior"]] == np.float32(-np.float32(probe)))


@pytest.mark.parametrize("h", [0.25, 0.5])
def test_isolated_atom_ses_is_its_sphere(h):
    c = np.array([[0.3, -0.2, 0.1]], dtype=np.float32)
    r = np.array([1.7], dtype=np.float32)
    o, hh, dims = grid_for(c, r, 1.4, h)
    res = oses.ses_field(c, r, 1.4, o, hh, dims)
    mc = oses.marching_cubes(res["f"], o, hh)
    rho = np.linalg.norm(mc["vertices"].reshape(-1, 3) - c.astype(np.float64)[0], axis=1)
    assert rho.size > 100
    assert rho.min() >= 1.7 - h - 1e-9 and rho.max() <= 1.7 + (H_SQRT3 + 1) * h + 1e-9
    assert closed_and_oriented(mc["vertices"])


def test_two_atom_neck_radius():
    r, rp, d, h = 1.5, 1.4, 4.0, 0.1
    c = np.array([[-d / 2, 0.0, 0.0], [d / 2, 0.0, 0.0]], dtype=np.float32)
    rad = np.array([r, r], dtype=np.float32)
    o, hh, dims = grid_for(c, rad, rp, h)
    res = oses.ses_field(c, rad, rp, o, hh, dims)
    mc = oses.marching_cubes(res["f"], o, hh)
    v = mc["vertices"].reshape(-1, 3)
    R = r + rp
    rho_c = math.sqrt(R * R - (d / 2) ** 2)
    neck = rho_c - rp
    # exterior wedge at the crease circle: angle pi - psi, cos psi = (rho_c^2 - (d/2)^2) / R^2
    psi = math.acos((rho_c ** 2 - (d / 2) ** 2) / R ** 2)
    slack = h * H_SQRT3 / 2 * (1 + 1 / math.sin((math.pi - psi) / 2))
    mid = np.abs(v[:, 0]) <= h
    radial = np.hypot(v[mid, 1], v[mid, 2])
    assert radial.size > 20
    assert radial.min() >= neck - h - 1e-9 and radial.max() <= neck + slack + h + 1e-9
    assert closed_and_oriented(mc["vertices"])


def test_probe_separates_distant_atoms():
    r, rp, h = 1.5, 1.4, 0.25
    d = 2 * (r + rp) + 1.0
    c = np.array([[-d / 2, 0.0, 0.0], [d / 2, 0.0, 0.0]], dtype=np.float32)
    rad = np.array([r, r], dtype=np.float32)
    o, hh, dims = grid_for(c, rad, rp, h)
    res = oses.ses_field(c, rad, rp, o, hh, dims)
    v = oses.marching_cubes(res["f"], o, hh)["vertices"].reshape(-1, 3)
    assert v.shape[0] > 100
    assert np.abs(v[:, 0]).min() >= d / 2 - r - (H_SQRT3 + 1) * h - 1e-9
