"""O-full: brute-force FP64 reference renderer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this module; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the HIP renderer.

What it computes (paper, Methods, "Molecular Graphics Engine" and
"High Quality Rendering"): a molecule is atom positions, radii and
connectivity; atoms are drawn as spheres and bonds as cylinders, each
displayed by ray-casting the primitive's implicit surface ("meshless
impostors"), which is pixel-exact; a deferred pass then applies screen-space
ambient occlusion and shading.  The paper gives no formulas, so every
numbered reading below is ours and is listed with its reason in the design
notes:

  R1 camera     basis f = |target-eye|, s = |f x up|, u = s x f; view depth
                z = (p-eye).f; pixel (i, j), row 0 at the top, has NDC centre
                (2(i+1/2)/W - 1, 1 - 2(j+1/2)/H); perspective rays leave the
                eye, orthographic rays are parallel to f.
  R2 sphere     front root of |o + t d - c| = r in the stable form
                b = oc.d, q = oc - b d, disc = r^2 - q.q, t = b - sqrt(disc);
                a hit counts only if znear <= z <= zfar (the back root is
                never used).
  R3 cylinder   closed, flat-capped; the entry point is the smallest t among
                the side's front root with 0 <= s <= L and the front-facing
                cap whose disk contains the plane hit; colour is the nearer
                atom's (two halves).
  R4 visibility lexicographic minimum of (z, id); atoms have id i, bonds
                N + b; background is id 0xFFFFFFFF with z = +inf.
  R5 shading    headlight Phong: c = albedo (ka + kd n.V) AO + ks max(0,
                2(n.V)^2 - 1)^alpha, clamped, q = floor(255 c + 1/2).
  R6 SSAO       K fixed hemisphere samples oriented by the normal with the
                branchless orthonormal basis of Duff et al. (JCGT 2017),
                projected to a pixel and compared with that pixel's depth.
  R6b noise     optional: the classic noise-and-blur form of screen-space
                AO, made deterministic.  Each pixel's tangent frame turns
                about its normal by an angle from a 4x4 ordered-dither
                (Bayer) table, so neighbouring pixels sample different
                directions; a 4x4 box blur over the hit pixels then averages
                the 16 rotations back into a smooth term.
  R7 post       the deferred post-passes the paper lists (shading flat,
                matte, glossy, toon; fog; outline): glossy is R5; matte drops
                its specular term; flat is albedo AO; toon replaces n.V by
                min(floor(4 n.V), 3)/3 in matte; linear fog blends towards a
                colour between two view depths; a hit pixel with an in-image
                4-neighbour that is background or deeper than z (1 + t) takes
                the outline colour.
  R8 clip       a world plane a x + b y + c z + d >= 0 keeps its side: a
                primitive's hit on the cut side is dropped (the primitive
                draws nothing at that pixel; interiors are not drawn).
  R9 AA         exact supersampling: the frame rendered at S times the
                size, each output channel the rounded-half-up mean of its
                S x S samples, depth and id the nearest (z, id) among them.

Because FP32 on the device and FP64 here can disagree where a result is
decided by a near-tie, every pixel also carries an accept set: the ids that
are correct answers within the stated tolerances (see ``accept_sets``).

Everything is evaluated for every pixel centre against every primitive: no
footprint, culling or ordering is used.
"""
from __future__ import annotations

import math

import numpy as np

KA, KD, KS, SHININESS = 0.2, 0.8, 0.25, 32.0
TAU = 1.0e-5                 # relative band for depth ties and grazing hits
BACKGROUND_ID = 0xFFFFFFFF
MAX_ACCEPT = 8
GOLDEN_STEP = 0.6180339887498949


# ---------------------------------------------------------------------------
# R1: camera and pixel rays
# ---------------------------------------------------------------------------
def camera_frame(cam):
    """World-space eye and orthonormal basis (s right, u up, f forward)."""
    e = np.asarray(cam.eye, dtype=np.float64)
    f = np.asarray(cam.target, dtype=np.float64) - e
    f = f / np.linalg.norm(f)
    s = np.cross(f, np.asarray(cam.up, dtype=np.float64))
    s = s / np.linalg.norm(s)
    u = np.cross(s, f)
    return e, s, u, f


def pixel_ndc(W, H, window):
    x0, y0, w, h = window
    nx = 2.0 * (np.arange(x0, x0 + w, dtype=np.float64) + 0.5) / W - 1.0
    ny = 1.0 - 2.0 * (np.arange(y0, y0 + h, dtype=np.float64) + 0.5) / H
    NX, NY = np.meshgrid(nx, ny)
    return NX.ravel(), NY.ravel()


def pixel_rays(cam, W, H, window):
    """World-space ray origins and unit directions, one per pixel, row-major."""
    e, s, u, f = camera_frame(cam)
    nx, ny = pixel_ndc(W, H, window)
    aspect = W / H
    if cam.projection == 0:
        th = math.tan(cam.fovy / 2.0)
        d = f[None, :] + (nx * th * aspect)[:, None] * s[None, :] + (ny * th)[:, None] * u[None, :]
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
        o = np.broadcast_to(e, d.shape).copy()
    else:
        hh = cam.ortho_half_height
        o = e[None, :] + (nx * hh * aspect)[:, None] * s[None, :] + (ny * hh)[:, None] * u[None, :]
        d = np.broadcast_to(f, o.shape).copy()
    return o, d


def _dot(a, b):
    return np.einsum("ij,ij->i", a, b)


# ---------------------------------------------------------------------------
# R2: sphere
# ---------------------------------------------------------------------------
def sphere_candidates(o, d, c, r, e, f, znear, zfar):
    """Per-pixel candidate record of one sphere.

    Returns a dict of arrays over the pixels that are a hit or a grazing
    near-hit: index, z, valid, graze, normal (world), unstable-shading flag.
    """
    oc = c[None, :] - o
    b = _dot(oc, d)
    q = oc - b[:, None] * d
    qn = np.sqrt(_dot(q, q))
    ocn = np.sqrt(_dot(oc, oc))
    geom_graze = np.abs(r - qn) <= TAU * ocn
    disc = r * r - qn * qn
    geom_hit = disc >= 0.0
    keep = np.nonzero(geom_hit | geom_graze)[0]
    if keep.size == 0:
        return None
    oc, b, qn, ocn, disc = oc[keep], b[keep], qn[keep], ocn[keep], disc[keep]
    gh, gg = geom_hit[keep], geom_graze[keep]
    oo, dd = o[keep], d[keep]
    t = np.where(gh, b - np.sqrt(np.maximum(disc, 0.0)), b)
    x = oo + t[:, None] * dd
    z = (x - e[None, :]) @ f
    zin = (z >= znear) & (z <= zfar)
    zgr = (np.abs(z - znear) <= TAU * np.maximum(np.abs(z), znear)) | (np.abs(z - zfar) <= TAU * zfar)
    cand = zin | zgr
    valid = gh & zin
    graze = cand & (gg | zgr)
    sel = np.nonzero(cand)[0]
    if sel.size == 0:
        return None
    n = (x[sel] - c[None, :]) / r
    return dict(pix=keep[sel], z=z[sel], valid=valid[sel], graze=graze[sel], normal=n,
                side=np.zeros(sel.size, dtype=np.int8), unstable=np.zeros(sel.size, dtype=bool),
                tangent_nv=-_dot(n, dd[sel]), x=x[sel])


# ---------------------------------------------------------------------------
# R3: capped cylinder
# ---------------------------------------------------------------------------
def cylinder_candidates(o, d, A, B, rho, e, f, znear, zfar):
    """Per-pixel candidate record of one bond cylinder between points A and B.

    side = 0 for the lateral surface, 1 for cap A (normal -a), 2 for cap B
    (normal +a); the albedo half is decided by s = (x - A).a against L/2.
    """
    AB = B - A
    L = float(np.linalg.norm(AB))
    if L == 0.0:
        return None
    a = AB / L
    P = o.shape[0]
    w = o - A[None, :]
    wn = np.sqrt(_dot(w, w))
    da = d @ a
    wa = w @ a
    dp = d - da[:, None] * a[None, :]
    wp = w - wa[:, None] * a[None, :]
    k = _dot(dp, dp)
    tol = TAU * wn

    inf = np.full(P, np.inf)
    # lateral surface
    with np.errstate(divide="ignore", invalid="ignore"):
        tc = np.where(k > 0, -_dot(wp, dp) / np.where(k > 0, k, 1.0), 0.0)
    qv = wp + tc[:, None] * dp
    qn = np.sqrt(_dot(qv, qv))
    disc = rho * rho - qn * qn
    side_geom = (k > 0) & (disc >= 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        ts = np.where(side_geom, tc - np.sqrt(np.maximum(disc, 0.0) / np.where(k > 0, k, 1.0)), tc)
    ss = wa + ts * da
    side_valid = side_geom & (ss >= 0.0) & (ss <= L)
    side_sil = (k > 0) & (np.abs(rho - qn) <= tol) & (ss >= -tol) & (ss <= L + tol)
    side_end = side_geom & ((np.abs(ss) <= tol) | (np.abs(ss - L) <= tol))
    side_graze = side_sil | side_end

    # caps: the plane hit is computed whenever the ray is not parallel to it;
    # it counts as an entry only if the ray meets the cap from outside.
    nonpar = np.abs(da) >= 1e-12
    with np.errstate(divide="ignore", invalid="ignore"):
        tA = np.where(nonpar, -wa / np.where(nonpar, da, 1.0), np.inf)
        tB = np.where(nonpar, (L - wa) / np.where(nonpar, da, 1.0), np.inf)
    pA = w + np.where(nonpar, tA, 0.0)[:, None] * d
    pB = w + np.where(nonpar, tB, 0.0)[:, None] * d - L * a[None, :]
    rA = np.sqrt(_dot(pA, pA))
    rB = np.sqrt(_dot(pB, pB))
    capA_geom = nonpar & (da > 0) & (rA <= rho)
    capB_geom = nonpar & (da < 0) & (rB <= rho)
    edge_on = np.abs(da) <= TAU
    capA_graze = nonpar & (da > -TAU) & (np.abs(rA - rho) <= tol) | (edge_on & (rA <= rho + tol))
    capB_graze = nonpar & (da < TAU) & (np.abs(rB - rho) <= tol) | (edge_on & (rB <= rho + tol))

    t_side = np.where(side_valid, ts, inf)
    t_capA = np.where(capA_geom, tA, inf)
    t_capB = np.where(capB_geom, tB, inf)
    stack = np.stack([t_side, t_capA, t_capB], axis=1)
    kind = np.argmin(stack, axis=1)
    t = stack[np.arange(P), kind]
    geom_hit = np.isfinite(t)
    # grazing parameters for near-misses: closest approach of the surface concerned
    t_gr = np.full(P, np.inf)
    t_gr = np.where(side_graze, np.minimum(t_gr, ts), t_gr)
    t_gr = np.where(capA_graze & np.isfinite(tA), np.minimum(t_gr, tA), t_gr)
    t_gr = np.where(capB_graze & np.isfinite(tB), np.minimum(t_gr, tB), t_gr)
    any_graze = side_graze | capA_graze | capB_graze
    keep = np.nonzero(geom_hit | (any_graze & np.isfinite(t_gr)))[0]
    if keep.size == 0:
        return None
    t_use = np.where(geom_hit[keep], t[keep], t_gr[keep])
    oo, dd = o[keep], d[keep]
    x = oo + t_use[:, None] * dd
    z = (x - e[None, :]) @ f
    zin = (z >= znear) & (z <= zfar)
    zgr = (np.abs(z - znear) <= TAU * np.maximum(np.abs(z), znear)) | (np.abs(z - zfar) <= TAU * zfar)
    cand = zin | zgr
    valid = geom_hit[keep] & zin
    graze = cand & (any_graze[keep] | zgr)
    sel = np.nonzero(cand)[0]
    if sel.size == 0:
        return None
    kk = kind[keep][sel]
    xs = x[sel]
    rel = xs - A[None, :]
    s_hit = rel @ a
    radial = rel - s_hit[:, None] * a[None, :]
    n = np.where((kk == 0)[:, None], radial / rho,
                 np.where((kk == 1)[:, None], -a[None, :], a[None, :]))
    half_b = np.where(kk == 0, s_hit >= 0.5 * L, kk == 2)
    tolk = tol[keep][sel]
    colour_edge = (kk == 0) & (np.abs(s_hit - 0.5 * L) <= tolk)
    unstable = colour_edge | (side_end[keep][sel]) | (kk != 0) & (capA_graze | capB_graze)[keep][sel]
    return dict(pix=keep[sel], z=z[sel], valid=valid[sel], graze=graze[sel], normal=n,
                side=kk.astype(np.int8), half_b=half_b, unstable=unstable,
                tangent_nv=-_dot(n, dd[sel]), x=xs)


# ---------------------------------------------------------------------------
# R4: G-buffer with accept sets
# ---------------------------------------------------------------------------
def _rgb(c):
    c = int(c)
    return np.array([c & 255, (c >> 8) & 255, (c >> 16) & 255, (c >> 24) & 255], dtype=np.float64)


REP_BALL_AND_STICK, REP_VAN_DER_WAALS, REP_STICKS, REP_SAS = 0, 1, 2, 3


def representation_scene(scene, opts):
    """The spheres and cylinders a molecular representation draws (paper,
    Methods, "Meshless Representations": ball-and-stick, van der Waals,
    sticks and the solvent-accessible surface are drawn with the same sphere
    and cylinder impostors).  Reading: van der Waals and the SAS draw no
    bonds; sticks draw every atom at the bond radius; the SAS adds the probe
    radius (default 1.4 A) to each radius, summed in FP32 like the inputs.
    Ids keep their meaning: atom i stays i and bond b stays N + b."""
    rep = int(getattr(opts, "representation", REP_BALL_AND_STICK))
    if rep == REP_BALL_AND_STICK:
        return scene
    radii, bonds = scene.radii, scene.bonds
    if rep in (REP_VAN_DER_WAALS, REP_SAS):
        bonds = np.zeros((0, 2), dtype=np.uint32)
    if rep == REP_STICKS:
        radii = np.full(scene.n_atoms, np.float32(opts.bond_radius), dtype=np.float32)
    elif rep == REP_SAS:
        radii = (scene.radii.astype(np.float32) + np.float32(getattr(opts, "probe_radius", 1.4))).astype(np.float32)
    return type(scene)(scene.positions, radii, scene.colors, bonds)


def gbuffer(scene, cam, opts, W, H, window=None):
    """Brute-force G-buffer over ``window`` = (x0, y0, w, h) of the W x H image.

    Returns a dict of per-pixel arrays (shape (h, w)):
      z, id            exact winner (lexicographic min of (z, id) over valid hits)
      normal_view      winner's unit normal in view coordinates (x right, y up, z forward)
      albedo           winner's packed RGBA8 colour
      unstable         winner's shading may flip between cap/side or colour halves
      acc_n, acc_id, acc_z, acc_bg
                       accept set: every id whose selection is correct within the
                       tolerances (depth ties within TAU z, grazing hits), its z,
                       and whether background is acceptable
      nv               winner's n.V (cosine between normal and view direction)
      fragments        number of (primitive, pixel) valid hits
    """
    if window is None:
        window = (0, 0, W, H)
    scene = representation_scene(scene, opts)
    x0, y0, w, h = window
    P = w * h
    o, d = pixel_rays(cam, W, H, window)
    e, s, u, f = camera_frame(cam)
    znear, zfar = float(cam.znear), float(cam.zfar)
    pos = scene.positions.astype(np.float64)
    rad = scene.radii.astype(np.float64)
    N = scene.n_atoms
    rec = {k: [] for k in ("pix", "id", "z", "valid", "graze", "normal", "albedo", "unstable", "nv")}
    plane = np.asarray(getattr(opts, "clip_plane", (0.0, 0.0, 0.0, 0.0)), dtype=np.float64)

    def add(c, pid, alb):
        if np.any(plane != 0.0):
            # R8 clip plane: a surface point with a x + b y + c z + d < 0 is
            # cut away (the primitive draws nothing there); within rounding
            # of the plane either outcome is accepted
            terms = c["x"] * plane[None, :3]
            v = terms.sum(axis=1) + plane[3]
            tol = TAU * (np.abs(terms).sum(axis=1) + abs(plane[3]))
            keep = v >= -tol
            c = {k: (a[keep] if isinstance(a, np.ndarray) and a.shape[:1] == keep.shape else a) for k, a in c.items()}
            alb = alb[keep]
            v, tol = v[keep], tol[keep]
            c["valid"] = c["valid"] & (v >= 0.0)
            c["graze"] = c["graze"] | (np.abs(v) <= tol)
        m = c["pix"].size
        rec["pix"].append(c["pix"])
        rec["id"].append(np.full(m, pid, dtype=np.int64))
        rec["z"].append(c["z"])
        rec["valid"].append(c["valid"])
        rec["graze"].append(c["graze"])
        rec["normal"].append(c["normal"])
        rec["albedo"].append(alb)
        rec["unstable"].append(c["unstable"])
        rec["nv"].append(c["tangent_nv"])

    for i in range(N):
        c = sphere_candidates(o, d, pos[i], rad[i], e, f, znear, zfar)
        if c is not None:
            add(c, i, np.full(c["pix"].size, scene.colors[i], dtype=np.uint32))
    rho = float(opts.bond_radius)
    for b in range(scene.n_bonds):
        ia, ib = int(scene.bonds[b, 0]), int(scene.bonds[b, 1])
        if ia == ib:
            continue
        c = cylinder_candidates(o, d, pos[ia], pos[ib], rho, e, f, znear, zfar)
        if c is not None:
            alb = np.where(c["half_b"], scene.colors[ib], scene.colors[ia]).astype(np.uint32)
            add(c, N + b, alb)
    out = _resolve(rec, P, (h, w), (s, u, f))
    out["view"] = (cam, W, H, window)
    return out


def _resolve(rec, P, shape, basis):
    s, u, f = basis
    out = dict(
        z=np.full(P, np.inf), id=np.full(P, BACKGROUND_ID, dtype=np.int64),
        normal_view=np.zeros((P, 3)), albedo=np.zeros(P, dtype=np.uint32),
        unstable=np.zeros(P, dtype=bool), nv=np.zeros(P),
        acc_n=np.zeros(P, dtype=np.int32), acc_id=np.full((P, MAX_ACCEPT), BACKGROUND_ID, dtype=np.int64),
        acc_z=np.full((P, MAX_ACCEPT), np.inf), acc_bg=np.ones(P, dtype=bool), fragments=0)
    if rec["pix"]:
        pix = np.concatenate(rec["pix"])
        pid = np.concatenate(rec["id"])
        z = np.concatenate(rec["z"])
        valid = np.concatenate(rec["valid"])
        graze = np.concatenate(rec["graze"])
        nrm = np.concatenate(rec["normal"])
        alb = np.concatenate(rec["albedo"])
        uns = np.concatenate(rec["unstable"])
        nv = np.concatenate(rec["nv"])
        out["fragments"] = int(np.count_nonzero(valid))
        order = np.lexsort((pid, z, pix))
        pix, pid, z, valid, graze = pix[order], pid[order], z[order], valid[order], graze[order]
        nrm, alb, uns, nv = nrm[order], alb[order], uns[order], nv[order]
        # exact winner: first valid candidate of each pixel in (z, id) order
        vi = np.nonzero(valid)[0]
        upix, first = np.unique(pix[vi], return_index=True)
        win = vi[first]
        out["z"][upix] = z[win]
        out["id"][upix] = pid[win]
        out["normal_view"][upix] = np.stack([nrm[win] @ s, nrm[win] @ u, nrm[win] @ f], axis=1)
        out["albedo"][upix] = alb[win]
        out["unstable"][upix] = uns[win]
        out["nv"][upix] = nv[win]
        # accept sets: solid hits decide the reference depth z*
        solid = valid & ~graze
        si = np.nonzero(solid)[0]
        zstar = np.full(P, np.inf)
        spix, sfirst = np.unique(pix[si], return_index=True)
        zstar[spix] = z[si[sfirst]]
        out["acc_bg"][:] = True
        out["acc_bg"][spix] = False
        cand = (solid | graze) & (z <= zstar[pix] * (1.0 + TAU))
        ci = np.nonzero(cand)[0]
        cp = pix[ci]
        # rank of each accepted candidate inside its pixel
        starts = np.r_[0, np.nonzero(np.diff(cp))[0] + 1]
        counts = np.diff(np.r_[starts, cp.size])
        rank = np.arange(cp.size) - np.repeat(starts, counts)
        np.add.at(out["acc_n"], cp, 1)
        ok = rank < MAX_ACCEPT
        out["acc_id"][cp[ok], rank[ok]] = pid[ci[ok]]
        out["acc_z"][cp[ok], rank[ok]] = z[ci[ok]]
    h, w = shape
    for k in ("z", "id", "albedo", "unstable", "nv", "acc_n", "acc_bg"):
        out[k] = out[k].reshape(h, w)
    out["normal_view"] = out["normal_view"].reshape(h, w, 3)
    out["acc_id"] = out["acc_id"].reshape(h, w, MAX_ACCEPT)
    out["acc_z"] = out["acc_z"].reshape(h, w, MAX_ACCEPT)
    return out


# ---------------------------------------------------------------------------
# R6: screen-space ambient occlusion
# ---------------------------------------------------------------------------
def ssao_kernel(K):
    """Hemisphere directions h_k and scales s_k, evaluated in FP64 and
    rounded to FP32 (then widened back), k = 0..K-1."""
    k = np.arange(K, dtype=np.float64)
    cos_t = 1.0 - (k + 0.5) / K
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    phi = 2.0 * math.pi * np.mod(k * GOLDEN_STEP, 1.0)
    hvec = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)
    scale = 0.1 + 0.9 * ((k + 1.0) / K) ** 2
    return hvec.astype(np.float32).astype(np.float64), scale.astype(np.float32).astype(np.float64)


def onb_duff(n):
    """Branchless orthonormal basis (Duff, Burgess, Christensen, Hery, Kensler,
    Liani, Villemin: "Building an Orthonormal Basis, Revisited", JCGT 6(1), 2017).
    Returns tangent T and bitangent B for unit normals n (rows)."""
    sign = np.copysign(1.0, n[:, 2])
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    T = np.stack([1.0 + sign * n[:, 0] ** 2 * a, sign * b, -sign * n[:, 0]], axis=1)
    Bv = np.stack([b, sign + n[:, 1] ** 2 * a, -n[:, 1]], axis=1)
    return T, Bv


def view_position(cam, W, H, window, z):
    """View-space position of the surface point at depth z on each pixel's ray."""
    nx, ny = pixel_ndc(W, H, window)
    aspect = W / H
    zz = z.ravel()
    if cam.projection == 0:
        th = math.tan(cam.fovy / 2.0)
        return np.stack([zz * nx * th * aspect, zz * ny * th, zz], axis=1)
    hh = cam.ortho_half_height
    return np.stack([nx * hh * aspect, ny * hh, zz], axis=1)


def view_dir(cam, W, H, window):
    """Unit view-space direction of each pixel's ray."""
    nx, ny = pixel_ndc(W, H, window)
    aspect = W / H
    if cam.projection == 0:
        th = math.tan(cam.fovy / 2.0)
        d = np.stack([nx * th * aspect, ny * th, np.ones_like(nx)], axis=1)
        return d / np.linalg.norm(d, axis=1, keepdims=True)
    return np.tile(np.array([0.0, 0.0, 1.0]), (nx.size, 1))


def _smoothstep01(x):
    x = np.clip(x, 0.0, 1.0)
    return x * x * (3.0 - 2.0 * x)


BAYER4 = np.array([[0, 8, 2, 10], [12, 4, 14, 6], [3, 11, 1, 9], [15, 7, 13, 5]])


def noise_rotation(W, H, window):
    """R6b: cosine and sine of the turn of each pixel's tangent frame about its
    normal, 2 pi (B[Y mod 4][X mod 4] + 1/2) / 16 for pixel column X and row
    Y, B the 4x4 Bayer matrix; evaluated in FP64, rounded to FP32."""
    x0, y0, w, h = window
    X = np.arange(x0, x0 + w)[None, :] + np.zeros((h, 1), dtype=np.int64)
    Y = np.arange(y0, y0 + h)[:, None] + np.zeros((1, w), dtype=np.int64)
    th = 2.0 * math.pi * (BAYER4[Y % 4, X % 4] + 0.5) / 16.0
    c = np.cos(th).astype(np.float32).astype(np.float64).ravel()
    s = np.sin(th).astype(np.float32).astype(np.float64).ravel()
    return c, s


def ssao(cam, W, H, window, Pv, Nv, hit, depth_buf, depth_win, K, R, bias,
         edge_px=1e-3, depth_rel=1e-5, ambiguous=None, rotation=None):
    """Ambient occlusion at the pixels of ``window``.

    Pv, Nv: (n, 3) view-space position and unit normal per pixel; hit: (n,) bool.
    depth_buf: view depth (+inf background) over ``depth_win`` = (x0, y0, w, h).
    ambiguous: optional bool mask over depth_win of pixels whose visible
    primitive is not unique (several accepted answers); a sample that reads
    one counts as unstable, since a correct G-buffer may hold another depth
    there.
    rotation: optional (cos, sin) per pixel (R6b): the tangent frame becomes
    T' = cos T + sin B, B' = cos B - sin T.
    Returns (ao (n,), unstable (n,) count of samples whose outcome may flip,
    outside (n,) count of on-screen samples that fell outside depth_buf).
    """
    n = Pv.shape[0]
    ao = np.ones(n)
    unstable = np.zeros(n, dtype=np.int32)
    outside = np.zeros(n, dtype=np.int32)
    if K <= 0:
        return ao, unstable, outside
    hk, sk = ssao_kernel(K)
    T, Bv = onb_duff(np.where(hit[:, None], Nv, np.array([0.0, 0.0, -1.0])))
    if rotation is not None:
        rc, rs = rotation
        T, Bv = rc[:, None] * T + rs[:, None] * Bv, rc[:, None] * Bv - rs[:, None] * T
    flip = hit & (np.abs(Nv[:, 2]) <= 1e-4)
    unstable[flip] = K
    bx0, by0, bw, bh = depth_win
    occ_sum = np.zeros(n)
    znear = float(cam.znear)
    zP = Pv[:, 2]
    for k in range(K):
        dirv = hk[k, 0] * T + hk[k, 1] * Bv + hk[k, 2] * Nv
        S = Pv + (R * sk[k]) * dirv
        if cam.projection == 0:
            fpx = (H / 2.0) / math.tan(cam.fovy / 2.0)
            with np.errstate(divide="ignore", invalid="ignore"):
                px = W / 2.0 + fpx * S[:, 0] / S[:, 2]
                py = H / 2.0 - fpx * S[:, 1] / S[:, 2]
        else:
            sc = (H / 2.0) / cam.ortho_half_height
            px = W / 2.0 + S[:, 0] * sc
            py = H / 2.0 - S[:, 1] * sc
        front = S[:, 2] > znear
        near_edge = np.abs(S[:, 2] - znear) <= depth_rel * np.maximum(np.abs(S[:, 2]), znear)
        with np.errstate(invalid="ignore"):
            qx = np.floor(px)
            qy = np.floor(py)
        onscreen = front & (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
        fx = px - qx
        fy = py - qy
        edge = (np.minimum(fx, 1 - fx) <= edge_px) | (np.minimum(fy, 1 - fy) <= edge_px)
        ix = np.where(onscreen, qx, 0).astype(np.int64) - bx0
        iy = np.where(onscreen, qy, 0).astype(np.int64) - by0
        inbuf = (ix >= 0) & (ix < bw) & (iy >= 0) & (iy < bh)
        zq = np.full(n, np.inf)
        ok = onscreen & inbuf
        zq[ok] = depth_buf[iy[ok], ix[ok]]
        thr = S[:, 2] - bias
        occ = ok & (zq <= thr)
        with np.errstate(divide="ignore", invalid="ignore"):
            wgt = _smoothstep01(R / np.abs(zP - zq))
        wgt = np.where(np.isfinite(zq), wgt, 0.0)
        occ_sum += np.where(hit & occ, wgt, 0.0)
        margin = np.abs(zq - thr) <= depth_rel * np.abs(S[:, 2])
        if ambiguous is not None:
            amb = np.zeros(n, dtype=bool)
            amb[ok] = ambiguous[iy[ok], ix[ok]]
            margin = margin | amb
        unstable += (hit & ((front & edge) | near_edge | (ok & margin))).astype(np.int32)
        outside += (hit & onscreen & ~inbuf).astype(np.int32)
    ao = np.where(hit, 1.0 - occ_sum / K, 1.0)
    return ao, unstable, outside


# ---------------------------------------------------------------------------
# R5: shading
# ---------------------------------------------------------------------------
SHADE_GLOSSY, SHADE_MATTE, SHADE_FLAT, SHADE_TOON = 0, 1, 2, 3


def rgb_of(packed):
    """(P, 3) channels in [0, 1] of packed RGBA8 values."""
    packed = np.asarray(packed, dtype=np.uint32)
    return np.stack([(packed >> sh) & 255 for sh in (0, 8, 16)], axis=-1).astype(np.float64) / 255.0


def shade(Nv, Vv, albedo, ao, hit, background, shading=SHADE_GLOSSY, z=None, fog=None):
    """Packed RGBA8 per pixel (R5, R7 without the outline) and the pixels
    whose toon band sits on an edge.  Vv is the unit direction towards the
    camera; fog = (start, end, packed colour) or None."""
    nv = np.maximum(0.0, np.einsum("ij,ij->i", Nv, Vv))
    alb = rgb_of(albedo)
    band_edge = np.zeros(nv.shape, dtype=bool)
    if shading == SHADE_FLAT:
        c = alb * ao[:, None]
    elif shading == SHADE_TOON:
        b = np.minimum(np.floor(4.0 * nv), 3.0) / 3.0
        k = np.round(4.0 * nv)
        band_edge = (np.abs(4.0 * nv - k) <= 1e-4) & (k >= 1) & (k <= 3)
        c = alb * (KA + KD * b)[:, None] * ao[:, None]
    else:
        c = alb * (KA + KD * nv)[:, None] * ao[:, None]
        if shading == SHADE_GLOSSY:
            c = c + (KS * np.maximum(0.0, 2.0 * nv * nv - 1.0) ** SHININESS)[:, None]
    if fog is not None and fog[1] > fog[0]:
        f = np.clip((z - fog[0]) / (fog[1] - fog[0]), 0.0, 1.0)[:, None]
        c = (1.0 - f) * c + f * rgb_of(fog[2])
    q = np.floor(255.0 * np.clip(c, 0.0, 1.0) + 0.5).astype(np.uint32)
    rgba = q[:, 0] | (q[:, 1] << 8) | (q[:, 2] << 16) | (np.uint32(255) << 24)
    return np.where(hit, rgba, np.uint32(background)).astype(np.uint32), band_edge & hit


def outline(W, H, window, z, depth_buf, depth_win, t, depth_rel=1e-5):
    """R7 outline over the window: pixels to recolour, and pixels where a
    neighbour's depth is within depth_rel z of the threshold (or is not in
    depth_buf)."""
    x0, y0, w, h = window
    bx0, by0, bw, bh = depth_win
    zz = z.reshape(h, w)
    hit = np.isfinite(zz)
    thr = zz * (1.0 + t)
    edge = np.zeros((h, w), dtype=bool)
    unsure = np.zeros((h, w), dtype=bool)
    X = x0 + np.arange(w)[None, :] + np.zeros((h, 1), dtype=np.int64)
    Y = y0 + np.arange(h)[:, None] + np.zeros((1, w), dtype=np.int64)
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        qx, qy = X + dx, Y + dy
        in_img = (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
        ix, iy = qx - bx0, qy - by0
        in_buf = in_img & (ix >= 0) & (ix < bw) & (iy >= 0) & (iy < bh)
        zq = np.full((h, w), np.inf)
        zq[in_buf] = depth_buf[iy[in_buf], ix[in_buf]]
        with np.errstate(invalid="ignore"):
            edge |= hit & in_buf & (zq > thr)
            unsure |= hit & in_buf & np.isfinite(zq) & (np.abs(zq - thr) <= depth_rel * np.abs(zz))
        unsure |= hit & in_img & ~in_buf
    return edge, unsure


def blurred_ssao(cam, opts, W, H, window, depth_buf, depth_win, normal_buf, edge_px, depth_rel, ambiguous):
    """R6b: the AO of the window's pixels as the mean of the rotated raw AO
    over the hit pixels (X + dx, Y + dy), dx, dy in {-2, -1, 0, 1}, inside
    the image.  Raw values are taken over the window grown by that footprint
    within the depth buffer; a neighbour the buffer does not cover counts as
    outside, and the unstable and outside counts of every raw value taken
    add up."""
    x0, y0, w, h = window
    bx0, by0, bw, bh = depth_win
    gx0, gy0 = max(x0 - 2, bx0), max(y0 - 2, by0)
    gx1, gy1 = min(x0 + w + 1, bx0 + bw), min(y0 + h + 1, by0 + bh)
    gwin = (gx0, gy0, gx1 - gx0, gy1 - gy0)
    db = np.asarray(depth_buf, dtype=np.float64)
    zg = db[gy0 - by0:gy1 - by0, gx0 - bx0:gx1 - bx0].ravel()
    ng = np.asarray(normal_buf, dtype=np.float64)[gy0 - by0:gy1 - by0, gx0 - bx0:gx1 - bx0].reshape(-1, 3)
    hit = np.isfinite(zg)
    Pv = view_position(cam, W, H, gwin, np.where(hit, zg, 1.0))
    raw, uns, outside = ssao(cam, W, H, gwin, Pv, ng, hit, depth_buf, depth_win,
                             int(opts.ssao_samples), float(opts.ssao_radius), float(opts.ssao_bias),
                             edge_px=edge_px, depth_rel=depth_rel, ambiguous=ambiguous,
                             rotation=noise_rotation(W, H, gwin))
    gh, gw = gy1 - gy0, gx1 - gx0
    raw, uns, outside, hit = (a.reshape(gh, gw) for a in (raw, uns, outside, hit))
    ao = np.ones((h, w))
    uo = np.zeros((h, w), dtype=np.int32)
    oo = np.zeros((h, w), dtype=np.int32)
    total = np.zeros((h, w))
    count = np.zeros((h, w))
    jj, ii = np.mgrid[y0:y0 + h, x0:x0 + w]
    for dy in (-2, -1, 0, 1):
        for dx in (-2, -1, 0, 1):
            qx, qy = ii + dx, jj + dy
            in_img = (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
            in_g = in_img & (qx >= gx0) & (qx < gx1) & (qy >= gy0) & (qy < gy1)
            oo += (in_img & ~in_g).astype(np.int32)
            gi, gj = np.where(in_g, qx - gx0, 0), np.where(in_g, qy - gy0, 0)
            take = in_g & hit[gj, gi]
            total += np.where(take, raw[gj, gi], 0.0)
            count += take
            uo += np.where(take, uns[gj, gi], 0)
            oo += np.where(take, outside[gj, gi], 0)
    ao = np.where(count > 0, total / np.maximum(count, 1), 1.0)
    return ao.ravel(), uo.ravel(), oo.ravel()


def shade_gbuffer(cam, opts, W, H, window, z, normal_view, albedo, depth_buf=None, depth_win=None,
                  edge_px=1e-3, depth_rel=1e-5, ambiguous=None, normal_buf=None):
    """Deferred pass: SSAO then shading over ``window``.

    z, normal_view, albedo cover the window; depth_buf/depth_win give the depth
    visible to the SSAO samples (defaults to the window itself).
    Returns dict(rgba, ao, ssao_unstable, ssao_outside) with (h, w) arrays.
    """
    x0, y0, w, h = window
    zz = z.ravel()
    hit = np.isfinite(zz)
    Pv = view_position(cam, W, H, window, np.where(hit, zz, 1.0))
    Nv = normal_view.reshape(-1, 3)
    if depth_buf is None:
        depth_buf, depth_win = z, window
        normal_buf = normal_view
    if normal_buf is None and tuple(depth_win) == tuple(window):
        normal_buf = normal_view
    if int(getattr(opts, "ssao_noise", 0)) and int(opts.ssao_samples) > 0:
        if normal_buf is None:
            raise ValueError("SSAO noise needs the normals over the depth buffer (normal_buf)")
        ao, uns, outside = blurred_ssao(cam, opts, W, H, window, depth_buf, depth_win, normal_buf,
                                        edge_px, depth_rel, ambiguous)
        ao = np.where(hit, ao, 1.0)
        uns = np.where(hit, uns, 0)
        outside = np.where(hit, outside, 0)
    else:
        ao, uns, outside = ssao(cam, W, H, window, Pv, Nv, hit, depth_buf, depth_win,
                                int(opts.ssao_samples), float(opts.ssao_radius), float(opts.ssao_bias),
                                edge_px=edge_px, depth_rel=depth_rel, ambiguous=ambiguous)
    Vv = -view_dir(cam, W, H, window)
    fog = (float(getattr(opts, "fog_start", 0.0)), float(getattr(opts, "fog_end", 0.0)),
           int(getattr(opts, "fog_color", 0)))
    rgba, band_edge = shade(Nv, Vv, albedo.ravel().astype(np.uint32), ao, hit, int(opts.background),
                            shading=int(getattr(opts, "shading", SHADE_GLOSSY)), z=zz, fog=fog)
    # decisions of the post-passes that FP32 may take the other way count
    # as unstable samples
    uns = uns + band_edge.astype(uns.dtype)
    t = float(getattr(opts, "outline_depth", 0.0))
    if t > 0.0:
        edge, unsure = outline(W, H, window, zz, np.asarray(depth_buf, dtype=np.float64), depth_win, t,
                               depth_rel=depth_rel)
        oc = np.uint32((int(getattr(opts, "outline_color", 0)) & 0xFFFFFF) | 0xFF000000)
        rgba = np.where(edge.ravel(), oc, rgba).astype(np.uint32)
        uns = uns + unsure.ravel().astype(uns.dtype)
    return dict(rgba=rgba.reshape(h, w), ao=ao.reshape(h, w),
                ssao_unstable=uns.reshape(h, w), ssao_outside=outside.reshape(h, w))


def supersample_reduce(res, S):
    """R9 anti-aliasing by exact supersampling: an (S H) x (S W) render
    ``res`` (full frame, from either oracle) reduced to H x W.  Each RGBA
    channel is the mean of the pixel's S x S samples rounded half up
    (integers); depth and id are the lexicographic minimum of (z, id); a
    pixel is checkable when all its samples are strict and free of unstable
    deferred-pass decisions."""
    z, ids, rgba = res["z"], res["id"].astype(np.int64), res["rgba"].astype(np.int64)
    HH, WW = z.shape
    H, W = HH // S, WW // S
    blk = lambda a: a.reshape(H, S, W, S).transpose(0, 2, 1, 3).reshape(H, W, S * S)
    zb, ib = blk(z), blk(ids)
    order = np.lexsort((ib, zb), axis=-1)[..., 0]
    zmin = np.take_along_axis(zb, order[..., None], -1)[..., 0]
    idmin = np.take_along_axis(ib, order[..., None], -1)[..., 0]
    n = S * S
    out = np.zeros((H, W), dtype=np.int64)
    for ch in range(4):
        total = blk((rgba >> (8 * ch)) & 255).sum(axis=-1)
        out |= ((total + n // 2) // n) << (8 * ch)
    strict = (((res["acc_n"] == 1) & ~res["acc_bg"] & ~res["unstable"]) | ((res["acc_n"] == 0) & res["acc_bg"]))
    ok = strict & (res["ssao_unstable"] == 0) & (res["ssao_outside"] == 0)
    return dict(z=zmin, id=idmin, rgba=out.astype(np.uint32), stable=blk(ok).all(axis=-1))


def render(scene, cam, opts, W, H, window=None, halo=0, edge_px=1e-3, depth_rel=1e-5):
    """End to end: G-buffer over the window grown by ``halo`` pixels, then
    SSAO and shading of the window.  Returns the G-buffer dict restricted to
    the window plus rgba/ao/ssao_unstable/ssao_outside."""
    if window is None:
        window = (0, 0, W, H)
    x0, y0, w, h = window
    gx0, gy0 = max(0, x0 - halo), max(0, y0 - halo)
    gx1, gy1 = min(W, x0 + w + halo), min(H, y0 + h + halo)
    gwin = (gx0, gy0, gx1 - gx0, gy1 - gy0)
    g = gbuffer(scene, cam, opts, W, H, gwin)
    sl = (slice(y0 - gy0, y0 - gy0 + h), slice(x0 - gx0, x0 - gx0 + w))
    inner = {k: (v[sl] if isinstance(v, np.ndarray) and v.ndim >= 2 else v) for k, v in g.items()}
    sh = shade_gbuffer(cam, opts, W, H, window, inner["z"], inner["normal_view"], inner["albedo"],
                       depth_buf=g["z"], depth_win=gwin, edge_px=edge_px, depth_rel=depth_rel,
                       ambiguous=ambiguous_pixels(g), normal_buf=g["normal_view"])
    inner.update(sh)
    inner["view"] = (cam, W, H, window)
    return inner


def ambiguous_pixels(g):
    """Pixels of a G-buffer whose visible primitive is not unique: the
    accept set holds several primitives, or a grazing hit and background."""
    return (g["acc_n"] + g["acc_bg"].astype(np.int32)) > 1
