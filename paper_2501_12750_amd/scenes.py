"""Seeded synthetic molecular scenes.

This module only draws inputs: atom positions, radii, colours, bonds and
camera/option parameter values.  It holds none of the rendering arithmetic,
so both the HIP renderer and the CPU oracle can be fed from it.

A molecule is given by its atom positions, their radii and their connectivity
(paper, Methods, "Molecular Graphics Engine").  The paper's benchmark systems
(Performance evaluation and its table: 107,640 / 1,074,183 / 11,003,162 /
101,753,154 atoms) are not available here; these generators stand in for them
at the same scales.  Every generator uses ``numpy.random.default_rng(seed)``,
draws in FP64 and rounds once to FP32.  Camera values are rounded to FP32 as
well, so every consumer sees bit-identical inputs.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Element table: C, N, O, S, H.
ELEMENT_MIX = np.array([0.50, 0.15, 0.20, 0.02, 0.13])
ELEMENT_VDW = np.array([1.70, 1.55, 1.52, 1.80, 1.20], dtype=np.float32)
ELEMENT_RGBA = np.array([
    (144, 144, 144, 255),   # C grey
    (48, 80, 248, 255),     # N blue
    (255, 13, 13, 255),     # O red
    (255, 255, 48, 255),    # S yellow
    (255, 255, 255, 255),   # H white
], dtype=np.uint32)

PERSPECTIVE = 0
ORTHOGRAPHIC = 1


def pack_rgba(r, g, b, a=255) -> int:
    """RGBA8 packed in a u32, R in the low byte."""
    return int(r) | (int(g) << 8) | (int(b) << 16) | (int(a) << 24)


ELEMENT_COLOR = (ELEMENT_RGBA[:, 0] | (ELEMENT_RGBA[:, 1] << 8)
                 | (ELEMENT_RGBA[:, 2] << 16) | (ELEMENT_RGBA[:, 3] << 24)).astype(np.uint32)


def f32(x) -> float:
    """Round a Python float to the nearest FP32 value."""
    return float(np.float32(x))


@dataclasses.dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple = (0.0, 1.0, 0.0)
    fovy: float = f32(math.radians(45.0))
    projection: int = PERSPECTIVE
    ortho_half_height: float = 1.0
    znear: float = 1.0
    zfar: float = 1.0e5

    def __post_init__(self):
        self.eye = tuple(f32(v) for v in self.eye)
        self.target = tuple(f32(v) for v in self.target)
        self.up = tuple(f32(v) for v in self.up)
        self.fovy = f32(self.fovy)
        self.ortho_half_height = f32(self.ortho_half_height)
        self.znear = f32(self.znear)
        self.zfar = f32(self.zfar)


@dataclasses.dataclass
class Options:
    bond_radius: float = 0.15
    ssao_samples: int = 0
    ssao_radius: float = 2.0
    ssao_bias: float = 0.05
    background: int = 0          # packed RGBA8
    tile_size: int = 0           # 0: library default
    flags: int = 0
    representation: int = 0      # 0 ball-and-stick, 1 van der Waals, 2 sticks, 3 solvent-accessible surface
    probe_radius: float = 1.4
    shading: int = 0             # 0 glossy, 1 matte, 2 flat, 3 toon
    fog_color: int = 0           # packed RGBA8
    fog_start: float = 0.0       # view depths; no fog unless fog_end > fog_start
    fog_end: float = 0.0
    outline_color: int = 0       # packed RGBA8
    outline_depth: float = 0.0   # relative depth step of an outline; 0: none
    clip_plane: tuple = (0.0, 0.0, 0.0, 0.0)   # a, b, c, d: a x + b y + c z + d >= 0 is kept
    supersample: int = 1         # samples per pixel side (1..4)
    ssao_noise: int = 0          # 1: per-pixel rotation of the SSAO samples from a 4x4 table, then a 4x4 blur

    def __post_init__(self):
        self.bond_radius = f32(self.bond_radius)
        self.ssao_radius = f32(self.ssao_radius)
        self.ssao_bias = f32(self.ssao_bias)
        self.probe_radius = f32(self.probe_radius)
        self.fog_start = f32(self.fog_start)
        self.fog_end = f32(self.fog_end)
        self.outline_depth = f32(self.outline_depth)
        self.clip_plane = tuple(f32(v) for v in self.clip_plane)


@dataclasses.dataclass
class Scene:
    positions: np.ndarray        # (N, 3) float32
    radii: np.ndarray            # (N,) float32
    colors: np.ndarray           # (N,) uint32 RGBA8
    bonds: np.ndarray            # (M, 2) uint32

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def n_bonds(self) -> int:
        return int(self.bonds.shape[0])

    def permuted(self, perm_atoms: np.ndarray, perm_bonds: np.ndarray | None = None) -> "Scene":
        """Same molecule with atoms listed in order ``perm_atoms`` (new i = old perm[i])."""
        inv = np.empty_like(perm_atoms)
        inv[perm_atoms] = np.arange(perm_atoms.size)
        bonds = inv[self.bonds.astype(np.int64)].astype(np.uint32) if self.n_bonds else self.bonds
        if perm_bonds is not None and self.n_bonds:
            bonds = bonds[perm_bonds]
        return Scene(self.positions[perm_atoms].copy(), self.radii[perm_atoms].copy(),
                     self.colors[perm_atoms].copy(), np.ascontiguousarray(bonds))


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    camera: Camera
    options: Options
    width: int
    height: int


def _elements(rng, n):
    return rng.choice(5, size=n, p=ELEMENT_MIX)


def _vdw_scene(rng, pos64) -> Scene:
    el = _elements(rng, pos64.shape[0])
    return Scene(np.ascontiguousarray(pos64.astype(np.float32)),
                 np.ascontiguousarray(ELEMENT_VDW[el]),
                 np.ascontiguousarray(ELEMENT_COLOR[el]),
                 np.zeros((0, 2), dtype=np.uint32))


# ---------------------------------------------------------------------------
# Plain method, small: uniform cube, spheres only, 256x256, no SSAO.
# ---------------------------------------------------------------------------
def plain_small(n_atoms=4096, width=256, height=256, seed=1, half_extent=20.0,
                eye_distance=120.0) -> Workload:
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-half_extent, half_extent, size=(n_atoms, 3))
    scene = _vdw_scene(rng, pos)
    cam = Camera(eye=(0.0, 0.0, eye_distance), target=(0.0, 0.0, 0.0))
    return Workload("plain_small_4k_256", scene, cam, Options(ssao_samples=0), width, height)


# ---------------------------------------------------------------------------
# Ball-and-stick: 2,000 Gaussian globules of 500 atoms, ~1.05M bonds.
# ---------------------------------------------------------------------------
def greedy_bonds(pos32: np.ndarray, cutoff=1.6, max_degree=4) -> np.ndarray:
    """All atom pairs closer than ``cutoff``, taken in (distance, i, j) order
    while both atoms have fewer than ``max_degree`` bonds."""
    from scipy.spatial import cKDTree
    p = pos32.astype(np.float64)
    pairs = cKDTree(p).query_pairs(cutoff, output_type="ndarray")
    if pairs.size == 0:
        return np.zeros((0, 2), dtype=np.uint32)
    i, j = pairs[:, 0], pairs[:, 1]
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    dist = np.linalg.norm(p[lo] - p[hi], axis=1)
    order = np.lexsort((hi, lo, dist))
    lo, hi = lo[order], hi[order]
    # An atom with at most max_degree candidate pairs never reaches the cap
    # before its last one, so only pairs touching a "hot" atom (more
    # candidates than the cap) can be refused, and only by a hot endpoint's
    # degree: the greedy pass runs over those pairs alone, in order.
    cand = np.bincount(np.concatenate([lo, hi]), minlength=p.shape[0])
    hot = cand > max_degree
    contested = np.flatnonzero(hot[lo] | hot[hi])
    keep = np.ones(lo.size, dtype=bool)
    deg = {}
    for k, a, b in zip(contested.tolist(), lo[contested].tolist(), hi[contested].tolist()):
        da, db = deg.get(a, 0), deg.get(b, 0)
        if da < max_degree and db < max_degree:
            deg[a] = da + 1
            deg[b] = db + 1
        else:
            keep[k] = False
    out = np.stack([lo[keep], hi[keep]], axis=1)
    out = out[np.lexsort((out[:, 1], out[:, 0]))]      # listed in atom order, like a topology
    return np.ascontiguousarray(out.astype(np.uint32))


def fit_camera(pos32: np.ndarray, fovy_deg=45.0) -> Camera:
    """Camera on +z of the centroid, far enough that 99.9% of atoms fit."""
    p = pos32.astype(np.float64)
    c = p.mean(axis=0)
    r999 = float(np.percentile(np.linalg.norm(p - c, axis=1), 99.9))
    dist = r999 / math.sin(math.radians(fovy_deg) / 2)
    return Camera(eye=(c[0], c[1], c[2] + dist), target=tuple(c), fovy=math.radians(fovy_deg))


def ball_and_stick(n_globules=2000, atoms_per_globule=500, sigma=12.0, pitch=14.3,
                   width=1920, height=1080, seed=2, ssao_samples=16) -> Workload:
    rng = np.random.default_rng(seed)
    g = max(1, int(round(n_globules ** (1.0 / 3.0))))
    while g ** 3 < n_globules:
        g += 1
    cells = np.stack(np.meshgrid(np.arange(g), np.arange(g), np.arange(g), indexing="ij"),
                     axis=-1).reshape(-1, 3)[:n_globules]
    centres = (cells + 0.5) * pitch + rng.uniform(-pitch / 4, pitch / 4, size=(n_globules, 3))
    pos = (centres[:, None, :] + rng.normal(0.0, sigma, size=(n_globules, atoms_per_globule, 3)))
    pos32 = np.ascontiguousarray(pos.reshape(-1, 3).astype(np.float32))
    n = pos32.shape[0]
    el = _elements(rng, n)
    bonds = greedy_bonds(pos32)
    scene = Scene(pos32, np.full(n, 0.3, dtype=np.float32),
                  np.ascontiguousarray(ELEMENT_COLOR[el]), bonds)
    cam = fit_camera(pos32)
    opts = Options(bond_radius=0.15, ssao_samples=ssao_samples, ssao_radius=2.0)
    return Workload(f"ball_and_stick_{n // 1000}k_{width}x{height}", scene, cam, opts, width, height)


# ---------------------------------------------------------------------------
# Whole-cell-like: clustered compartments in a 5,000 A box, vdW spheres.
# ---------------------------------------------------------------------------
def whole_cell(n_atoms=100_000_000, n_compartments=200, box=5000.0, r_min=300.0, r_max=900.0,
               width=3840, height=2160, seed=3, ssao_samples=16, eye_clearance=50.0) -> Workload:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, box, size=(n_compartments, 3))
    radii = rng.uniform(r_min, r_max, size=n_compartments)
    w = radii ** 3 / np.sum(radii ** 3)
    out = np.empty((n_atoms, 3), dtype=np.float32)
    have = 0
    chunk = 1 << 22
    while have < n_atoms:
        need = min(n_atoms - have, chunk)
        counts = rng.multinomial(need, w)
        comp = np.repeat(np.arange(n_compartments), counts)
        d = rng.normal(size=(need, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rr = radii[comp] * np.cbrt(rng.uniform(size=need))
        p = centres[comp] + d * rr[:, None]
        inside = np.all((p >= 0.0) & (p <= box), axis=1)
        p = p[inside]
        take = min(p.shape[0], n_atoms - have)
        out[have:have + take] = p[:take]
        have += take
    el = _elements(rng, n_atoms)
    scene = Scene(out, np.ascontiguousarray(ELEMENT_VDW[el]),
                  np.ascontiguousarray(ELEMENT_COLOR[el]), np.zeros((0, 2), dtype=np.uint32))
    while True:
        eye = rng.uniform(0.1 * box, 0.9 * box, size=3)
        if np.all(np.linalg.norm(centres - eye, axis=1) - radii >= eye_clearance):
            break
    cam = Camera(eye=tuple(eye), target=(box / 2, box / 2, box / 2))
    opts = Options(ssao_samples=ssao_samples, ssao_radius=2.0)
    return Workload(f"whole_cell_{n_atoms // 1_000_000}M_{width}x{height}", scene, cam, opts,
                    width, height)


# ---------------------------------------------------------------------------
# Batched trajectory: 50k-atom globule, 64 random-walk frames, 4 viewports.
# ---------------------------------------------------------------------------
TRAJECTORY_VIEWPORTS = ((1280, 720), (1600, 900), (1920, 1080), (2560, 1440))


def trajectory(n_atoms=50_000, n_frames=64, density=0.1, step_sigma=0.5, eye_distance=142.0,
               seed=4, ssao_samples=16):
    """Returns (scene at frame 0, positions (F, N, 3) float32, cameras[4], options, viewports)."""
    rng = np.random.default_rng(seed)
    radius = (3.0 * n_atoms / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    d = rng.normal(size=(n_atoms, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pos = d * (radius * np.cbrt(rng.uniform(size=n_atoms)))[:, None]
    scene = _vdw_scene(rng, pos)
    frames = np.empty((n_frames, n_atoms, 3), dtype=np.float32)
    frames[0] = scene.positions
    for t in range(1, n_frames):
        step = rng.normal(0.0, step_sigma, size=(n_atoms, 3)).astype(np.float32)
        frames[t] = frames[t - 1] + step          # FP32 add of FP32 values
    cams = []
    for k in range(4):
        ang = math.radians(90.0 * k)
        cams.append(Camera(eye=(eye_distance * math.sin(ang), 0.0, eye_distance * math.cos(ang)),
                           target=(0.0, 0.0, 0.0)))
    opts = Options(ssao_samples=ssao_samples, ssao_radius=2.0)
    return scene, frames, cams, opts, TRAJECTORY_VIEWPORTS


WORKLOADS = {
    "plain_small": plain_small,
    "ball_and_stick": ball_and_stick,
    "whole_cell": whole_cell,
}


# ---------------------------------------------------------------------------
# Served mix: many clients, each a session of consecutive frames of one scene.
# ---------------------------------------------------------------------------
SERVE_RESOLUTIONS = ((1280, 720), (1920, 1080), (3840, 2160))


@dataclasses.dataclass
class ServedScene:
    """One scene of the served pool: vdW spheres (the whole-cell generator
    scaled to n atoms at the same density) or ball-and-stick globules of 500
    atoms (the ball-and-stick generator)."""
    kind: str
    n_atoms: int
    seed: int

    def build(self):
        """Returns (scene, centre, radius of the sphere around the centre that
        holds 99.9% of the atoms)."""
        if self.kind == "ball_and_stick":
            wl = ball_and_stick(n_globules=max(1, self.n_atoms // 500), seed=self.seed)
        else:
            s = (self.n_atoms / 1e8) ** (1.0 / 3.0)
            wl = whole_cell(n_atoms=self.n_atoms, box=5000.0 * s, r_min=300.0 * s, r_max=900.0 * s,
                            seed=self.seed, eye_clearance=0.0)
        p = wl.scene.positions.astype(np.float64)
        c = p.mean(axis=0)
        r999 = float(np.percentile(np.linalg.norm(p - c, axis=1), 99.9))
        return wl.scene, c, r999


@dataclasses.dataclass
class ServedRequest:
    t: float                 # arrival time, seconds from the start
    session: int
    scene: int               # index into the pool
    frame: int               # frame of the session (0, 1, ...)
    width: int
    height: int
    angle: float             # orbit angle of the camera, radians


def orbit_camera(centre, radius, angle, fovy_deg=45.0) -> Camera:
    """Camera on a horizontal circle around `centre`, far enough that a
    sphere of `radius` fits the vertical field of view."""
    dist = radius / math.sin(math.radians(fovy_deg) / 2)
    eye = (centre[0] + dist * math.sin(angle), centre[1], centre[2] + dist * math.cos(angle))
    return Camera(eye=eye, target=tuple(centre), fovy=math.radians(fovy_deg))


def served_mix(duration_s=60.0, rate_hz=200.0, n_scenes=24, n_min=1e4, n_max=1e7, mean_session=8.0,
               frame_interval_s=1.0 / 30.0, degrees_per_frame=2.0, seed=5):
    """A seeded arrival schedule: sessions start as a Poisson process of rate
    rate_hz / mean_session; each lasts a geometric number of frames (mean
    mean_session) requested every frame_interval_s on one scene of the pool
    (n log-uniform in [n_min, n_max], vdW and ball-and-stick alternately), at
    one resolution (uniform over 720p, 1080p, 4K), with the camera orbiting
    the scene.  Returns (pool, requests sorted by arrival)."""
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(n_scenes):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        pool.append(ServedScene("vdw" if k % 2 == 0 else "ball_and_stick", n, 100 + k))
    reqs = []
    t, sid = 0.0, 0
    while True:
        t += rng.exponential(mean_session / rate_hz)
        if t >= duration_s:
            break
        length = int(rng.geometric(1.0 / mean_session))
        scene = int(rng.integers(n_scenes))
        W, H = SERVE_RESOLUTIONS[int(rng.integers(len(SERVE_RESOLUTIONS)))]
        a0 = float(rng.uniform(0.0, 2.0 * math.pi))
        for f in range(length):
            tf = t + f * frame_interval_s
            if tf >= duration_s:
                break
            reqs.append(ServedRequest(tf, sid, scene, f, W, H, a0 + math.radians(degrees_per_frame) * f))
        sid += 1
    reqs.sort(key=lambda r: (r.t, r.session))
    return pool, reqs
