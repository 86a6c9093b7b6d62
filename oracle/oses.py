"""O-ses: the solvent excluded surface on a grid, extracted by marching cubes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this module; only
the tests use it.  It shares no code with the HIP path.

What it computes (paper, Methods, "Cartoon and SES representations": the
solvent excluded surface is computed by a discrete approach and extracted by
marching cubes).  The paper gives no formulas; the readings are ours:

  R10 grid    grid point (i, j, k) sits at o + h (i, j, k) (FP64 of the FP32
              origin o and spacing h); linear index i + nx (j + ny k).
  R11 SAS     a grid point lies inside the solvent-accessible region when
              some atom has |p - c|^2 < (r + rp)^2, each square and sum
              rounded once in FP64 (no fused operations); the other points
              are probe-centre positions ("exterior").
  R12 SES     D(p) = min(h sqrt(g), W h), g the least squared grid distance
              from p to an exterior point (0 for exterior points), W =
              ceil(rp / h) + 2; f(p) = D(p) - rp, rounded to FP32.  The SES
              encloses {f >= 0}: points at least rp from every probe centre.
              Beyond W h only the sign of f is used, so the distance is
              clamped there.
  R13 MC      cube (i, j, k) has corners c = 0..7 at (i + c&1, j + c>>1&1,
              k + c>>2&1); its case is the bit set of corners with f >= 0.
              The case's triangles come from tracing the surface's boundary
              on the six faces: a face with two crossing edges gets one
              segment, a face whose inside corners are diagonal gets two,
              each cutting off one inside corner; the segments close into
              loops, each oriented so that its normal (right-hand rule over
              the edge midpoints) points from the inside corners to the
              outside ones, and rotated to start at its lowest edge; loops
              are taken by lowest edge.  A loop of three edges is one
              triangle; a longer loop is a fan of triangles (centre, v_i,
              v_i+1) around its centre, the mean of its vertices, so that no
              triangle edge other than the loop's own runs along a cube face
              (a chord there would meet the neighbouring cube's surface in a
              line).  A vertex lies on edge (a, b), a the lower corner, at
              t = f_a / (f_a - f_b) of the way (FP32 values of f).
"""
from __future__ import annotations

import math

import numpy as np

# edges: corner pairs, x-edges, then y-, then z-edges
EDGES = [(0, 1), (2, 3), (4, 5), (6, 7),
         (0, 2), (1, 3), (4, 6), (5, 7),
         (0, 4), (1, 5), (2, 6), (3, 7)]
# faces: corners in cyclic order around the face
FACES = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]


def _corner(c):
    return np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1], dtype=np.float64)


def _edge_of(a, b):
    key = (min(a, b), max(a, b))
    return EDGES.index(key)


def mc_case(m):
    """The oriented edge loops of case m (R13)."""
    inside = [(m >> c) & 1 for c in range(8)]
    # segments on the faces
    seg = []
    for face in FACES:
        s = [inside[c] for c in face]
        e = [_edge_of(face[i], face[(i + 1) % 4]) for i in range(4)]
        cross = [i for i in range(4) if s[i] != s[(i + 1) % 4]]
        if len(cross) == 2:
            seg.append((e[cross[0]], e[cross[1]]))
        elif len(cross) == 4:
            for i in range(4):
                if s[i]:
                    seg.append((e[(i - 1) % 4], e[i]))
    # each crossing edge is in two segments: close the loops
    nbr = {}
    for a, b in seg:
        nbr.setdefault(a, []).append(b)
        nbr.setdefault(b, []).append(a)
    used = set()
    loops = []
    for start in sorted(nbr):
        if start in used:
            continue
        loop = [start]
        used.add(start)
        prev, cur = start, nbr[start][0]
        while cur != start:
            loop.append(cur)
            used.add(cur)
            a, b = nbr[cur]
            prev, cur = cur, (b if a == prev else a)
        loops.append(loop)
    out_loops = []
    for loop in loops:
        mids = [(_corner(EDGES[e][0]) + _corner(EDGES[e][1])) / 2 for e in loop]
        nrm = np.zeros(3)
        for i in range(len(mids)):
            nrm += np.cross(mids[i], mids[(i + 1) % len(mids)])
        out = np.zeros(3)
        for e in loop:
            a, b = EDGES[e]
            out += (_corner(b) - _corner(a)) if inside[a] else (_corner(a) - _corner(b))
        if float(nrm @ out) < 0:
            loop = loop[::-1]
        k = loop.index(min(loop))
        out_loops.append(loop[k:] + loop[:k])
    return out_loops


def loop_triangles(loop_pts):
    """Triangles of one loop of vertex positions (R13): the loop itself when
    it has three vertices, else the fan around the mean of its vertices."""
    k = len(loop_pts)
    if k == 3:
        return [tuple(loop_pts)]
    c = np.mean(np.asarray(loop_pts), axis=0)
    return [(c, loop_pts[i], loop_pts[(i + 1) % k]) for i in range(k)]


def mc_table():
    """The loops of all 256 cases."""
    return [mc_case(m) for m in range(256)]


def case_triangles(loops):
    """Number of triangles a case's loops make."""
    return sum(1 if len(lp) == 3 else len(lp) for lp in loops)


def ses_field(positions, radii, probe, origin, spacing, dims):
    """R10-R12 on the grid: f (FP32, shape (nz, ny, nx)), the exterior mask
    and the exact integer squared distances g (-1 where clamped)."""
    from scipy.spatial import cKDTree
    nx, ny, nz = (int(d) for d in dims)
    o = np.asarray(origin, dtype=np.float32).astype(np.float64)
    h = float(np.float32(spacing))
    rp = float(np.float32(probe))
    pos = np.asarray(positions, dtype=np.float32).astype(np.float64)
    rad = np.asarray(radii, dtype=np.float32).astype(np.float64)
    R = rad + rp
    interior = np.zeros((nz, ny, nx), dtype=bool)
    xs = o[0] + h * np.arange(nx)
    ys = o[1] + h * np.arange(ny)
    zs = o[2] + h * np.arange(nz)
    for c, Ri in zip(pos, R):
        lo = np.floor((c - Ri - o) / h).astype(np.int64) - 1
        hi = np.ceil((c + Ri - o) / h).astype(np.int64) + 1
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, np.array([nx - 1, ny - 1, nz - 1]))
        if np.any(lo > hi):
            continue
        dx = xs[lo[0]:hi[0] + 1] - c[0]
        dy = ys[lo[1]:hi[1] + 1] - c[1]
        dz = zs[lo[2]:hi[2] + 1] - c[2]
        d2 = (dx[None, None, :] * dx[None, None, :] + dy[None, :, None] * dy[None, :, None]) + \
            dz[:, None, None] * dz[:, None, None]
        interior[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] |= d2 < Ri * Ri
    W = int(math.ceil(rp / h)) + 2
    g = np.zeros((nz, ny, nx), dtype=np.int64)
    ext = np.argwhere(~interior)           # (k, j, i)
    ins = np.argwhere(interior)
    if ins.size:
        if ext.size:
            tree = cKDTree(ext)
            dist, idx = tree.query(ins, k=1, distance_upper_bound=W + 0.5)
            ok = np.isfinite(dist)
            gi = np.full(ins.shape[0], -1, dtype=np.int64)
            d = ext[idx[ok]] - ins[ok]
            gi[ok] = (d * d).sum(axis=1)
            gi[gi > W * W] = -1
        else:
            gi = np.full(ins.shape[0], -1, dtype=np.int64)
        g[tuple(ins.T)] = gi
    D = np.where(g < 0, W * h, np.minimum(h * np.sqrt(np.maximum(g, 0).astype(np.float64)), W * h))
    f = (D - rp).astype(np.float32)
    return dict(f=f, exterior=~interior, g=g, W=W)


def marching_cubes(f, origin, spacing, table=None):
    """R13 over an FP32 field of shape (nz, ny, nx): triangle vertices (T, 3, 3)
    in FP64, the linear index of each triangle's cube and its case, in the
    order of the cubes (x fastest) and of each case's triangles."""
    table = table or mc_table()
    f = np.asarray(f, dtype=np.float32)
    nz, ny, nx = f.shape
    o = np.asarray(origin, dtype=np.float32).astype(np.float64)
    h = float(np.float32(spacing))
    inside = f >= 0
    m = np.zeros((nz - 1, ny - 1, nx - 1), dtype=np.int64)
    for c in range(8):
        dx, dy, dz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        m |= inside[dz:nz - 1 + dz, dy:ny - 1 + dy, dx:nx - 1 + dx].astype(np.int64) << c
    ntri = np.array([case_triangles(t) for t in table])
    cubes = np.nonzero(ntri[m.ravel()])[0]
    verts, cube_of, case_of = [], [], []
    for q in cubes:
        k, rem = divmod(int(q), (ny - 1) * (nx - 1))
        j, i = divmod(rem, nx - 1)
        mm = int(m[k, j, i])
        for loop in table[mm]:
            pts = []
            for e in loop:
                a, b = EDGES[e]
                ca, cb = _corner(a).astype(int), _corner(b).astype(int)
                fa = float(f[k + ca[2], j + ca[1], i + ca[0]])
                fb = float(f[k + cb[2], j + cb[1], i + cb[0]])
                t = fa / (fa - fb)
                pts.append(o + h * (np.array([i, j, k], dtype=np.float64) + ca + t * (cb - ca)))
            for tri in loop_triangles(pts):
                verts.append(tri)
                cube_of.append(int(q))
                case_of.append(mm)
    return dict(vertices=np.array(verts, dtype=np.float64).reshape(-1, 3, 3),
                cube=np.array(cube_of, dtype=np.int64), case=np.array(case_of, dtype=np.int64))
