"""Seeded synthetic scenes: Gaussians, a textured room-box mesh and cameras.

This module only draws inputs. It holds none of the renderer's arithmetic and
is shared by the HIP path, the CPU oracle, the tests and the benchmark.

The paper evaluates on captured indoor scenes (Deep Blending, ScanNet++,
Replica; Sec. 4 "Datasets"), which are not available here. These synthetic
rooms stand in for them with the paper's sizes: 0.3-3.4 M Gaussians
(Table 1), a mesh of about 1e5 triangles with 2048x2048 RGB textures (Sec. 4.1
"Implementation Details"), and cameras inside the room.

Conventions (shared by both implementations by definition):
  * world and camera axes: x right, y down, z forward (OpenCV); the room is
    x in [-3, 3], y in [-1.5, 1.5] (y = +1.5 is the floor), z in [-2, 2];
  * camera: p_cam = R @ p_world + t, pinhole fx, fy, cx, cy; the pixel (i, j)
    is sampled at (i + 0.5, j + 0.5);
  * quaternions are (w, x, y, z), not normalised;
  * SH coefficients are stored [N, (d+1)^2, 3]; the DC term of a colour c is
    (c - 0.5) / Y00 with Y00 = 1 / (2 sqrt(pi));
  * textures are [n_tex, H, W, 3] float32; per-corner UVs are [F, 3, 2].

Seeds: the scene of workload k uses seed 1000*k, view v uses 1000*k + 1 + v.
All random draws are float64 from numpy's PCG64 and then cast to float32;
those float32 arrays are the ground truth for every implementation.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))

ROOM_MIN = np.array([-3.0, -1.5, -2.0])
ROOM_MAX = np.array([3.0, 1.5, 2.0])

RESOLUTIONS = [(640, 480), (1280, 720), (1600, 1064), (1920, 1080)]


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # [3,3] float64, world -> camera
    t: np.ndarray  # [3] float64

    @property
    def centre(self) -> np.ndarray:
        return -self.R.T @ self.t


@dataclasses.dataclass
class Gaussians:
    means: np.ndarray  # [N,3] f32
    log_scales: np.ndarray  # [N,3] f32
    quats: np.ndarray  # [N,4] f32 (w,x,y,z)
    opacity_logits: np.ndarray  # [N] f32
    sh: np.ndarray  # [N,(d+1)^2,3] f32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Gaussians":
        return Gaussians(self.means[idx], self.log_scales[idx], self.quats[idx],
                         self.opacity_logits[idx], self.sh[idx], self.sh_degree)


@dataclasses.dataclass
class Mesh:
    verts: np.ndarray  # [V,3] f32
    faces: np.ndarray  # [F,3] i32
    uvs: np.ndarray  # [F,3,2] f32
    face_tex: np.ndarray  # [F] i32
    tex: np.ndarray  # [n_tex,H,W,3] f32

    @property
    def n_faces(self) -> int:
        return int(self.faces.shape[0])


@dataclasses.dataclass
class Scene:
    name: str
    gaussians: Gaussians
    mesh: Optional[Mesh]
    cameras: List[Camera]
    target: Optional[List[np.ndarray]] = None  # per camera [3,H,W] f32


def empty_mesh() -> Mesh:
    return Mesh(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32),
                np.zeros((0, 3, 2), np.float32), np.zeros((0,), np.int32),
                np.zeros((1, 1, 1, 3), np.float32))


# ---------------------------------------------------------------- cameras --
def pinhole(width: int, height: int, fov_x_deg: float = 70.0):
    f = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    return f, f, width / 2.0, height / 2.0


def look_camera(width, height, centre, yaw, pitch, fov_x_deg=70.0) -> Camera:
    """Camera at `centre` turned by yaw about world y, then pitch about its x."""
    cy_, sy_ = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    ry = np.array([[cy_, 0.0, sy_], [0.0, 1.0, 0.0], [-sy_, 0.0, cy_]])
    rx = np.array([[1.0, 0.0, 0.0], [0.0, cp, -sp], [0.0, sp, cp]])
    r_wc = ry @ rx
    r_cw = r_wc.T
    t = -r_cw @ np.asarray(centre, np.float64)
    fx, fy, cx, cy = pinhole(width, height, fov_x_deg)
    return Camera(width, height, fx, fy, cx, cy, r_cw, t)


def random_room_camera(rng: np.random.Generator, width: int, height: int) -> Camera:
    lo = ROOM_MIN + 0.5
    hi = ROOM_MAX - 0.5
    centre = rng.uniform(lo, hi)
    yaw = rng.uniform(0.0, 2.0 * math.pi)
    pitch = math.radians(rng.uniform(-20.0, 20.0))
    return look_camera(width, height, centre, yaw, pitch)


# -------------------------------------------------------------- gaussians --
def _quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _sh_coeffs(rng, n, degree, colour_dc):
    k = (degree + 1) ** 2
    sh = np.zeros((n, k, 3))
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.2, size=(n, k - 1, 3))
    sh[:, 0, :] = (colour_dc - 0.5) / Y00
    return sh


def make_gaussians(means, log_scales, quats, opacity_logits, sh, degree) -> Gaussians:
    return Gaussians(np.ascontiguousarray(means, np.float32),
                     np.ascontiguousarray(log_scales, np.float32),
                     np.ascontiguousarray(quats, np.float32),
                     np.ascontiguousarray(opacity_logits, np.float32),
                     np.ascontiguousarray(sh, np.float32), int(degree))


def cluster_gaussians(rng, n, degree=3, log_scale_range=(-5.0, -2.0), n_clusters=64) -> Gaussians:
    """Means drawn around `n_clusters` isotropic clusters inside the room."""
    centres = rng.uniform(ROOM_MIN + 0.3, ROOM_MAX - 0.3, size=(n_clusters, 3))
    sig = rng.uniform(0.05, 0.3, size=n_clusters)
    which = rng.integers(0, n_clusters, size=n)
    means = centres[which] + sig[which, None] * rng.standard_normal((n, 3))
    means = np.clip(means, ROOM_MIN + 0.02, ROOM_MAX - 0.02)
    ls = rng.uniform(log_scale_range[0], log_scale_range[1], size=(n, 3))
    q = _quats(rng, n)
    op = rng.standard_normal(n)
    sh = _sh_coeffs(rng, n, degree, rng.uniform(0.0, 1.0, size=(n, 3)))
    return make_gaussians(means, ls, q, op, sh, degree)


def wall_gaussians(rng, n, degree=3, log_scale_range=(-6.0, -3.0)) -> Gaussians:
    """Gaussians 1 cm inside the four walls and the floor, area weighted."""
    # (axis, value, inward sign); the floor is y = +1.5 (y points down)
    planes = [(0, -3.0, +1), (0, 3.0, -1), (2, -2.0, +1), (2, 2.0, -1), (1, 1.5, -1)]
    areas = []
    for ax, _, _ in planes:
        others = [a for a in range(3) if a != ax]
        ext = ROOM_MAX - ROOM_MIN
        areas.append(ext[others[0]] * ext[others[1]])
    p = np.array(areas) / np.sum(areas)
    which = rng.choice(len(planes), size=n, p=p)
    means = rng.uniform(ROOM_MIN, ROOM_MAX, size=(n, 3))
    for k, (ax, val, sgn) in enumerate(planes):
        sel = which == k
        means[sel, ax] = val + sgn * 0.01
    ls = rng.uniform(log_scale_range[0], log_scale_range[1], size=(n, 3))
    q = _quats(rng, n)
    op = rng.standard_normal(n)
    sh = _sh_coeffs(rng, n, degree, rng.uniform(0.0, 1.0, size=(n, 3)))
    return make_gaussians(means, ls, q, op, sh, degree)


def outside_gaussians(rng, n, degree=3, margin=1.5, log_scale_range=(-4.0, -2.0)) -> Gaussians:
    """Gaussians in a shell up to `margin` outside the room box: what the
    walls hide from every camera inside (mesh-depth culling drops them)."""
    lo, hi = ROOM_MIN - margin, ROOM_MAX + margin
    out = np.zeros((0, 3))
    while out.shape[0] < n:
        p = rng.uniform(lo, hi, size=(2 * n, 3))
        inside = np.all((p > ROOM_MIN + 0.05) & (p < ROOM_MAX - 0.05), axis=1)
        wall = np.any((p > ROOM_MIN - 0.05) & (p < ROOM_MIN + 0.05) | (p > ROOM_MAX - 0.05) & (p < ROOM_MAX + 0.05), axis=1)
        out = np.concatenate([out, p[~inside & ~wall]])
    means = out[:n]
    ls = rng.uniform(log_scale_range[0], log_scale_range[1], size=(n, 3))
    sh = _sh_coeffs(rng, n, degree, rng.uniform(0.0, 1.0, size=(n, 3)))
    return make_gaussians(means, ls, _quats(rng, n), rng.standard_normal(n), sh, degree)


def concat_gaussians(a: Gaussians, b: Gaussians) -> Gaussians:
    assert a.sh_degree == b.sh_degree
    return Gaussians(*(np.concatenate([x, y]) for x, y in
                       ((a.means, b.means), (a.log_scales, b.log_scales), (a.quats, b.quats),
                        (a.opacity_logits, b.opacity_logits), (a.sh, b.sh))), a.sh_degree)


# ------------------------------------------------------------------- mesh --
def room_mesh(rng, target_faces: int, tex_size: int, n_tex: int = 4) -> Mesh:
    """The room box split into a grid of square cells, two triangles each.

    Vertices on shared box edges are shared, so the box is watertight. Each of
    the six box faces maps affinely onto [0,1]^2 of its texture: floor 0,
    ceiling 1, x walls 2, z walls 3. Textures are i.i.d. U[0,1] texels.
    """
    area = 2 * (6 * 4 + 6 * 3 + 4 * 3)
    s = math.sqrt(2.0 * area / target_faces)
    ext = ROOM_MAX - ROOM_MIN
    nseg = [max(1, int(round(e / s))) for e in ext]
    vid = {}
    verts = []

    def vertex(ijk):
        key = tuple(ijk)
        if key not in vid:
            vid[key] = len(verts)
            verts.append(ROOM_MIN + ext * np.array([key[d] / nseg[d] for d in range(3)]))
        return vid[key]

    faces, uvs, ftex = [], [], []
    # (fixed axis, fixed index 0 or nseg, texture id)
    boxfaces = [(1, 1, 0), (1, 0, 1), (0, 0, 2), (0, 1, 2), (2, 0, 3), (2, 1, 3)]
    for ax, side, tid in boxfaces:
        a, b = [d for d in range(3) if d != ax]
        na, nb = nseg[a], nseg[b]
        for i in range(na):
            for j in range(nb):
                corners = []
                for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                    ijk = [0, 0, 0]
                    ijk[ax] = side * nseg[ax]
                    ijk[a] = i + di
                    ijk[b] = j + dj
                    corners.append((vertex(ijk), ((i + di) / na, (j + dj) / nb)))
                for tri in ((0, 1, 2), (0, 2, 3)):
                    faces.append([corners[k][0] for k in tri])
                    uvs.append([corners[k][1] for k in tri])
                    ftex.append(tid)
    tex = rng.uniform(0.0, 1.0, size=(n_tex, tex_size, tex_size, 3)).astype(np.float32)
    return Mesh(np.asarray(verts, np.float32), np.asarray(faces, np.int32),
                np.asarray(uvs, np.float32), np.asarray(ftex, np.int32), tex)


def quad_mesh(rng, z=5.0, half=2.5, tex_size=256) -> Mesh:
    verts = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]],
                     np.float32)
    faces = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    corner_uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    uvs = corner_uv[faces]
    tex = rng.uniform(0.0, 1.0, size=(1, tex_size, tex_size, 3)).astype(np.float32)
    return Mesh(verts, faces, uvs.astype(np.float32), np.zeros(2, np.int32), tex)


# ---------------------------------------------------------------- configs --
def config1(seed: int = 1000) -> Scene:
    """64x64, identity camera, 2000 Gaussians (SH 0) and one textured quad at z=5."""
    rng = np.random.default_rng(seed)
    n = 2000
    means = np.column_stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    ls = rng.uniform(-4.0, -2.0, size=(n, 3))
    q = _quats(rng, n)
    op = rng.standard_normal(n)
    sh = _sh_coeffs(rng, n, 0, rng.uniform(0.0, 1.0, size=(n, 3)))
    g = make_gaussians(means, ls, q, op, sh, 0)
    mesh = quad_mesh(rng)
    cam = Camera(64, 64, 64.0, 64.0, 32.0, 32.0, np.eye(3), np.zeros(3))
    return Scene("config1_64x64_quad", g, mesh, [cam])


def config2(seed: int = 2000, n: int = 300_000, faces: int = 50_000, tex: int = 2048,
            n_views: int = 8) -> Scene:
    rng = np.random.default_rng(seed)
    g = cluster_gaussians(rng, n)
    mesh = room_mesh(rng, faces, tex)
    cams = [random_room_camera(np.random.default_rng(seed + 1 + v), 1280, 720)
            for v in range(n_views)]
    return Scene("config2_720p_300k", g, mesh, cams)


def config3(seed: int = 3000, n: int = 1_000_000, faces: int = 100_000, tex: int = 2048) -> Scene:
    rng = np.random.default_rng(seed)
    g = cluster_gaussians(rng, n)
    mesh = room_mesh(rng, faces, tex)
    vr = np.random.default_rng(seed + 1)
    cam = random_room_camera(vr, 1600, 1064)
    target = vr.uniform(0.0, 1.0, size=(3, 1064, 1600)).astype(np.float32)
    return Scene("config3_1600x1064_1M", g, mesh, [cam], [target])


def config4(seed: int = 4000, n: int = 1_000_000, faces: int = 200_000, tex: int = 2048,
            n_cams: int = 16) -> Scene:
    rng = np.random.default_rng(seed)
    g = cluster_gaussians(rng, n)
    mesh = room_mesh(rng, faces, tex)
    cams, targets = [], []
    for v in range(n_cams):
        vr = np.random.default_rng(seed + 1 + v)
        w, h = RESOLUTIONS[int(vr.integers(0, len(RESOLUTIONS)))]
        cams.append(random_room_camera(vr, w, h))
        targets.append(vr.uniform(0.0, 1.0, size=(3, h, w)).astype(np.float32))
    return Scene("config4_16cams_1M", g, mesh, cams, targets)


def config5(variant: str = "hybrid", seed: int = 5000, n_views: int = 32) -> Scene:
    """1920x1080 views of a Gaussian-only room (3M) or a hybrid room (600k + mesh)."""
    rng = np.random.default_rng(seed if variant == "hybrid" else seed + 500)
    if variant == "hybrid":
        g = cluster_gaussians(rng, 600_000)
        mesh = room_mesh(rng, 200_000, 4096)
    elif variant == "gaussian_only":
        walls = wall_gaussians(rng, 1_800_000)
        g = concat_gaussians(walls, cluster_gaussians(rng, 1_200_000))
        mesh = None
    else:
        raise ValueError(variant)
    cams, targets = [], []
    for v in range(n_views):
        vr = np.random.default_rng(seed + 1 + v)
        cams.append(random_room_camera(vr, 1920, 1080))
    return Scene(f"config5_1080p_{variant}", g, mesh, cams)


def small_room(seed: int, n: int = 3000, faces: int = 2000, tex: int = 64,
               width: int = 96, height: int = 80, n_cams: int = 1, degree: int = 3) -> Scene:
    """A scaled-down room with the same structure, for oracle-sized tests."""
    rng = np.random.default_rng(seed)
    g = cluster_gaussians(rng, n, degree)
    mesh = room_mesh(rng, faces, tex)
    cams, targets = [], []
    for v in range(n_cams):
        vr = np.random.default_rng(seed + 1 + v)
        cams.append(random_room_camera(vr, width, height))
        targets.append(vr.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32))
    return Scene(f"small_room_{seed}", g, mesh, cams, targets)
