"""CPU FP64 oracle of the hybrid mesh-Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY. Only `tests/`, `__graft_entry__.smoke()` and the
benchmark's `cpu_baseline` leg may import this package. It shares no code with
the HIP implementation: the C++ core in `oracle.cpp` is built with g++ (no HIP
headers) and the loss below is plain numpy.

Functions (one camera per call; several cameras are a loop):
  project(scene, cam)  per-Gaussian records             (Sec. 3.1: Sigma, Sigma', Eq. 1)
  keys(scene, cam)     sorted (tile|depth, index) pairs  (Sec. 1: tile-wise sorting)
  render(scene, cam)   image, T, counts, mesh buffers    (Sec. 3.1 Eq. 2, Sec. 3.4)
  backward(...)        reverse mode over a stored tape   (Sec. 3.4, texture optimisable)
  loss(...)            L1 + lambda * L_t with M_T        (Sec. 3.4, transmittance-aware supervision)
  full_loss(...)       Eq. 3 with D-SSIM and the mask variants of Table 3
  adam(...)            one Adam step                     (the optimiser of the joint optimisation)
  lambda_t_schedule(i) the L_t weight of Alg. 1 at iteration i
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

FP64_RECORDS = 1
TILE_ELLIPSE = 8  # keep only the tiles the alpha >= alpha_min ellipse can reach
MIP_2D = 4  # Mip-Splatting 2D filter: low_pass is the pixel filter, opacity compensated
CULL_MESH = 2  # drop (Gaussian, tile) pairs at or behind the tile's largest mesh depth


def build(force: bool = False) -> str:
    """Compile the oracle core with g++ (host only, OpenMP).

    ORACLE_LIB names another build of the core to load instead (the mutation
    tests point it at copies with planted mistakes)."""
    if os.environ.get("ORACLE_LIB"):
        return os.environ["ORACLE_LIB"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c++17",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _setup(_lib)
    return _lib


class Scene_(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p),
                ("n_verts", C.c_int32), ("n_faces", C.c_int32), ("n_tex", C.c_int32),
                ("tex_h", C.c_int32), ("tex_w", C.c_int32),
                ("verts", C.c_void_p), ("faces", C.c_void_p), ("uvs", C.c_void_p),
                ("face_tex", C.c_void_p), ("tex", C.c_void_p), ("filter3d", C.c_void_p)]


class Camera_(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("R", C.c_double * 9), ("t", C.c_double * 3)]


class Params_(C.Structure):
    _fields_ = [("bg", C.c_double * 3), ("low_pass", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("t_min", C.c_double), ("near_gs", C.c_double),
                ("near_mesh", C.c_double), ("clamp_fov", C.c_double), ("tile", C.c_int32),
                ("flags", C.c_int32), ("amb_alpha", C.c_double), ("amb_t", C.c_double)]


class ProjOut_(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("mean2d", "conic", "cov2d", "opacity", "rgb", "depth",
                                          "depth_bits", "radius", "rect", "tiles", "amb")]


class RenderOut_(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("image", "final_T", "n_contrib", "n_blended",
                                          "n_processed", "amb", "tri_id", "mesh_depth",
                                          "mesh_rgb", "trace", "n_alt", "alts")]


MAX_ALT = 16  # outcomes kept per pixel by render(..., alts=True)
AMB_ALPHA, AMB_T, AMB_PROJ, AMB_MESH, AMB_MANY = 1, 2, 4, 16, 32  # bits of render()["amb"]


class Grads_(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("means", "log_scales", "quats", "opacity_logits",
                                          "sh", "tex", "mean2d")]


def _setup(L):
    P = C.c_void_p
    L.or_project.argtypes = [P, P, P, P]
    L.or_project.restype = C.c_int
    L.or_keys.argtypes = [P, P, P, P, P, P, C.c_int64]
    L.or_keys.restype = C.c_int64
    L.or_render.argtypes = [P, P, P, C.c_int, C.c_int, C.c_int, C.c_int, P]
    L.or_render.restype = C.c_int
    L.or_backward.argtypes = [P, P, P, C.c_int, C.c_int, C.c_int, C.c_int, P, P, P, P]
    L.or_backward.restype = C.c_int
    L.or_sh_basis.argtypes = [C.c_int, C.c_int, P, P]
    L.or_sh_basis.restype = None
    L.or_quat_to_rot.argtypes = [P, P]
    L.or_quat_to_rot.restype = None
    L.or_mip_filter3d.argtypes = [P, P, C.c_int, P, C.c_double, P]
    L.or_mip_filter3d.restype = C.c_int
    L.or_max_threads.argtypes = []
    L.or_max_threads.restype = C.c_int


def threads():
    """Threads the oracle's parallel loops run on (OpenMP)."""
    return int(lib().or_max_threads())


def _p(a):
    return None if a is None else a.ctypes.data


# The renderer's conventions, as FP32 values (the kernel's settings are FP32,
# and both sides must compare against the same thresholds). amb_alpha and
# amb_t are the relative slacks under which an alpha-skip or T-stop decision
# counts as ambiguous: about 10x the relative error of alpha (~1e-6) and of T
# (~1e-5 after tens of blends) that an FP32 evaluation carries.
def default_params(**kw):
    d = dict(bg=(0.0, 0.0, 0.0), low_pass=0.3, alpha_min=1.0 / 255.0, alpha_max=0.99,
             t_min=1e-4, near_gs=0.2, near_mesh=0.05, clamp_fov=1.3, tile=16, flags=0,
             amb_alpha=2e-5, amb_t=1e-4)
    d.update(kw)
    return d


def _params(d):
    f32 = lambda v: float(np.float32(v))
    p = Params_()
    for i in range(3):
        p.bg[i] = f32(d["bg"][i])
    for k in ("low_pass", "alpha_min", "alpha_max", "t_min", "near_gs", "near_mesh", "clamp_fov"):
        setattr(p, k, f32(d[k]))
    p.tile = int(d["tile"])
    p.flags = int(d["flags"])
    p.amb_alpha = float(d["amb_alpha"])
    p.amb_t = float(d["amb_t"])
    return p


def _camera(cam):
    c = Camera_()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64).reshape(3)
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = t[i]
    return c


class _SceneArrays:
    """FP64 copies of the FP32 scene arrays, kept alive for the C call."""

    def __init__(self, g, mesh, overrides=None, filter3d=None):
        o = overrides or {}
        f64 = lambda a: np.ascontiguousarray(a, np.float64)
        self.filter3d = None if filter3d is None else f64(filter3d)
        self.means = f64(o.get("means", g.means))
        self.log_scales = f64(o.get("log_scales", g.log_scales))
        self.quats = f64(o.get("quats", g.quats))
        self.opacity_logits = f64(o.get("opacity_logits", g.opacity_logits))
        self.sh = f64(o.get("sh", g.sh))
        s = Scene_()
        s.n = self.means.shape[0]
        s.sh_degree = g.sh_degree
        s.means, s.log_scales, s.quats = _p(self.means), _p(self.log_scales), _p(self.quats)
        s.opacity_logits, s.sh = _p(self.opacity_logits), _p(self.sh)
        if self.filter3d is not None:
            assert self.filter3d.shape == (s.n,)
            s.filter3d = _p(self.filter3d)
        if mesh is not None and mesh.faces.shape[0] > 0:
            self.verts = f64(mesh.verts)
            self.faces = np.ascontiguousarray(mesh.faces, np.int32)
            self.uvs = f64(mesh.uvs)
            self.face_tex = np.ascontiguousarray(mesh.face_tex, np.int32)
            self.tex = np.ascontiguousarray(o.get("tex", mesh.tex), np.float32)
            s.n_verts, s.n_faces = self.verts.shape[0], self.faces.shape[0]
            s.n_tex, s.tex_h, s.tex_w = self.tex.shape[0], self.tex.shape[1], self.tex.shape[2]
            s.verts, s.faces, s.uvs = _p(self.verts), _p(self.faces), _p(self.uvs)
            s.face_tex, s.tex = _p(self.face_tex), _p(self.tex)
        else:
            s.n_verts = s.n_faces = 0
            s.n_tex, s.tex_h, s.tex_w = 1, 1, 1
            self.tex = np.zeros((1, 1, 1, 3), np.float32)
            s.tex = _p(self.tex)
        self.s = s


def project(gaussians, cam, params=None, filter3d=None):
    P = _params(params or default_params())
    sa = _SceneArrays(gaussians, None, filter3d=filter3d)
    n = gaussians.n
    out = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), cov2d=np.zeros((n, 3)),
               opacity=np.zeros(n), rgb=np.zeros((n, 3)), depth=np.zeros(n),
               depth_bits=np.zeros(n, np.uint32), radius=np.zeros(n, np.int32),
               rect=np.zeros((n, 4), np.int32), tiles=np.zeros(n, np.int32),
               amb=np.zeros(n, np.uint8))
    o = ProjOut_(**{k: _p(v) for k, v in out.items()})
    c = _camera(cam)
    rc = lib().or_project(C.byref(sa.s), C.byref(c), C.byref(P), C.byref(o))
    assert rc == 0
    return out


def keys(gaussians, cam, params=None, mesh=None, filter3d=None):
    """Sorted tile keys; the mesh matters only with the CULL_MESH flag."""
    P = _params(params or default_params())
    sa = _SceneArrays(gaussians, mesh, filter3d=filter3d)
    c = _camera(cam)
    K = lib().or_keys(C.byref(sa.s), C.byref(c), C.byref(P), None, None, None, 0)
    assert K >= 0
    tiles = ((cam.width + P.tile - 1) // P.tile) * ((cam.height + P.tile - 1) // P.tile)
    k = np.zeros(K, np.uint64)
    v = np.zeros(K, np.uint32)
    r = np.zeros((tiles, 2), np.uint32)
    K2 = lib().or_keys(C.byref(sa.s), C.byref(c), C.byref(P), _p(k), _p(v), _p(r), K)
    assert K2 == K
    return k, v, r


def render(gaussians, mesh, cam, params=None, window=None, overrides=None, filter3d=None,
           alts=False):
    """Forward render; `window` = (x0, y0, x1, y1) restricts the pixels computed.

    With alts=True, also `n_alt` [h,w] and `alts` [h,w,MAX_ALT,7]: for a pixel
    whose alpha-skip or transmittance-stop decision lies inside the ambiguity
    slack (FP32 cannot be sure of it), the outcome (r, g, b, T, n_contrib,
    n_blended, n_processed) of every path through those decisions taken
    either way; alts[..., 0, :] is the FP64 outcome itself."""
    P = _params(params or default_params())
    sa = _SceneArrays(gaussians, mesh, overrides, filter3d)
    x0, y0, x1, y1 = window or (0, 0, cam.width, cam.height)
    h, w = y1 - y0, x1 - x0
    out = dict(image=np.zeros((3, h, w)), final_T=np.zeros((h, w)),
               n_contrib=np.zeros((h, w), np.int32), n_blended=np.zeros((h, w), np.int32),
               n_processed=np.zeros((h, w), np.int32), amb=np.zeros((h, w), np.uint8),
               tri_id=np.zeros((h, w), np.int32), mesh_depth=np.zeros((h, w), np.float32),
               mesh_rgb=np.zeros((3, h, w)), trace=np.zeros(1, np.uint64))
    if alts:
        out["n_alt"] = np.zeros((h, w), np.int32)
        out["alts"] = np.zeros((h, w, MAX_ALT, 7))
    o = RenderOut_(**{k: _p(v) for k, v in out.items()})
    c = _camera(cam)
    rc = lib().or_render(C.byref(sa.s), C.byref(c), C.byref(P), x0, y0, x1, y1, C.byref(o))
    assert rc == 0
    out["trace"] = int(out["trace"][0])
    return out


def backward(gaussians, mesh, cam, g_image, g_T=None, g_mesh_rgb=None, params=None, window=None,
             overrides=None, want_tex=True, filter3d=None):
    """Gradient of sum(g_image*I_h) + sum(g_T*T) + sum(g_mesh_rgb*I_m) over the window.

    Besides the parameter gradients, `mean2d` [n,2] is the gradient with
    respect to each Gaussian's projected mean (u, v) in pixels: the quantity
    whose norm 3DGS densification accumulates."""
    P = _params(params or default_params())
    sa = _SceneArrays(gaussians, mesh, overrides, filter3d)
    x0, y0, x1, y1 = window or (0, 0, cam.width, cam.height)
    n = gaussians.n
    K = (gaussians.sh_degree + 1) ** 2
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, K, 3)), mean2d=np.zeros((n, 2)))
    if want_tex and mesh is not None and mesh.faces.shape[0] > 0:
        out["tex"] = np.zeros(mesh.tex.shape, np.float64)
    o = Grads_(**{k: _p(v) for k, v in out.items()})
    c = _camera(cam)
    f64 = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
    gi, gt, gm = f64(g_image), f64(g_T), f64(g_mesh_rgb)
    rc = lib().or_backward(C.byref(sa.s), C.byref(c), C.byref(P), x0, y0, x1, y1, _p(gi), _p(gt),
                           _p(gm), C.byref(o))
    assert rc == 0
    return out


def sh_basis(degree, dirs):
    dirs = np.ascontiguousarray(dirs, np.float64)
    K = (degree + 1) ** 2
    out = np.zeros((dirs.shape[0], K))
    lib().or_sh_basis(degree, dirs.shape[0], _p(dirs), _p(out))
    return out


def quat_to_rot(q):
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    lib().or_quat_to_rot(_p(q), _p(R))
    return R.reshape(3, 3)


def loss(image, final_T, mesh_rgb, tri_id, target, lambda_t=0.1, k=20.0, detach_mask=False):
    """L = mean|I_h - I| + lambda_t * mean_{p,c}[ M_T(p) (I~ - I~_m)^2 ].

    M_T = 1 / (1 + exp(-k (T - 0.5))); I~ and I~_m are the target and the mesh
    colour where a triangle covers the pixel, else 0 (Sec. 3.4, transmittance-
    aware supervision). The mean runs over pixels and channels. Returns the
    loss and its gradients with respect to the image, T and the mesh colour.
    """
    image = np.asarray(image, np.float64)
    T = np.asarray(final_T, np.float64)
    Im = np.asarray(mesh_rgb, np.float64)
    tgt = np.asarray(target, np.float64)
    has = (np.asarray(tri_id) >= 0)[None]
    n = image.size
    MT = 1.0 / (1.0 + np.exp(-k * (T - 0.5)))
    diff = np.where(has, tgt - Im, 0.0)
    sq = np.sum(diff * diff, axis=0)
    L = np.sum(np.abs(image - tgt)) / n + lambda_t * np.sum(MT * sq) / n
    g_image = np.sign(image - tgt) / n
    g_mesh = np.where(has, lambda_t * MT[None] * 2.0 * (Im - tgt) / n, 0.0)
    g_T = np.zeros_like(T) if detach_mask else lambda_t * sq * MT * (1.0 - MT) * k / n
    return L, g_image, g_T, g_mesh


# ----------------------------------------------------------- full loss --
MASK_MODES = ("none", "one", "T", "sigmoid")


def ssim_window(size=11, sigma=1.5):
    """Normalised 2-D Gaussian window, the outer product of a 1-D one."""
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(x * x) / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def full_loss(images, final_T, mesh_rgb, tri_id, target, lambda_c=0.2, lambda_t=0.1, k=20.0,
              mask_mode="sigmoid", detach_mask=False, c1=0.01 ** 2, c2=0.03 ** 2):
    """Eq. 3 with the transmittance-aware term of Sec. 3.4, over several images.

    L = (1 - lambda_c) * mean|I_h - I| + lambda_c * (1 - mean SSIM(I_h, I))
        + lambda_t * mean_{p,c}[ M_T(p) (I~ - I~_m)^2 ]
    SSIM per channel with an 11x11 Gaussian window (sigma 1.5) over zero-padded
    images; M_T: "none" (no L_t), "one", "T", or "sigmoid" 1/(1+exp(-k(T-1/2)))
    (the ablation of Table 3). Means run over every pixel and channel of every
    image. Arguments are lists of per-image arrays ([3,H,W] and [H,W]).
    Returns the loss and its gradients with respect to the images, T and I_m,
    by reverse mode in float64 (plain PyTorch CPU).
    """
    import torch
    f = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    X = [f(a) for a in images]
    T = [f(a) for a in final_T]
    M = [f(a) for a in mesh_rgb]
    Y = [torch.tensor(np.asarray(a, np.float64)) for a in target]
    has = [torch.tensor(np.asarray(a) >= 0) for a in tri_id]
    n = sum(x.numel() for x in X)
    w = torch.tensor(ssim_window())[None, None].repeat(3, 1, 1, 1)
    l1 = sum((x - y).abs().sum() for x, y in zip(X, Y)) / n
    ssim_sum = 0.0
    for x, y in zip(X, Y):
        xb, yb = x[None], y[None]
        conv = lambda z: torch.nn.functional.conv2d(z, w, padding=5, groups=3)
        mx, my = conv(xb), conv(yb)
        sxx = conv(xb * xb) - mx * mx
        syy = conv(yb * yb) - my * my
        sxy = conv(xb * yb) - mx * my
        s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
        ssim_sum = ssim_sum + s.sum()
    L = (1 - lambda_c) * l1 + lambda_c * (1 - ssim_sum / n)
    if mask_mode != "none":
        lt = 0.0
        for t, m, y, h in zip(T, M, Y, has):
            if mask_mode == "one":
                mt = torch.ones_like(t)
            elif mask_mode == "T":
                mt = t
            else:
                mt = 1.0 / (1.0 + torch.exp(-k * (t - 0.5)))
            if detach_mask:
                mt = mt.detach()
            d = torch.where(h[None], y - m, torch.zeros_like(m))
            lt = lt + (mt * (d * d).sum(0)).sum()
        L = L + lambda_t * lt / n
    L.backward()
    z = lambda v, like: (v.grad if v.grad is not None else torch.zeros_like(like)).numpy()
    return (float(L), [z(x, x) for x in X], [z(t, t) for t in T], [z(m, m) for m in M])


def adam(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15, lr_head=None, head=0,
         row=0):
    """One Adam step (Kingma and Ba, Algorithm 1, with bias-corrected moments) in
    float64; returns the new (param, m, v). When row > 0, elements whose flat
    index modulo row is below head take lr_head (the degree-0 SH rate)."""
    p = np.asarray(param, np.float64).reshape(-1)
    g = np.asarray(grad, np.float64).reshape(-1)
    m1 = beta1 * np.asarray(m, np.float64).reshape(-1) + (1.0 - beta1) * g
    v1 = beta2 * np.asarray(v, np.float64).reshape(-1) + (1.0 - beta2) * g * g
    m_hat = m1 / (1.0 - beta1 ** step)
    v_hat = v1 / (1.0 - beta2 ** step)
    rate = np.full(p.shape, float(lr))
    if row > 0:
        rate[(np.arange(p.size) % row) < head] = lr_head
    return p - rate * m_hat / (np.sqrt(v_hat) + eps), m1, v1


def lambda_t_schedule(i, lam=0.1, warmup=3000, densify_until=15000):
    """Weight of L_t at iteration i (Alg. 1): the full loss strictly after the
    warm-up and strictly before the end of densification, L_c alone otherwise."""
    return lam if warmup < i < densify_until else 0.0


def mip_filter3d(gaussians, cams, s=0.2, params=None):
    """Mip-Splatting 3D smoothing variance per Gaussian (s over the squared
    highest sampling rate fx/z among the cameras that see it)."""
    P = _params(params or default_params())
    sa = _SceneArrays(gaussians, None)
    arr = (Camera_ * len(cams))(*[_camera(c) for c in cams])
    out = np.zeros(gaussians.n)
    assert lib().or_mip_filter3d(C.byref(sa.s), arr, len(cams), C.byref(P), float(s), _p(out)) == 0
    return out
