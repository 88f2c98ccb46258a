"""Python binding of libhybrid_raster (include/hr.h): argument marshalling only.

Every step of the rasterizer runs in the HIP library; torch provides device
memory and the current stream. Importing this module does not touch the GPU;
`load()` raises when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhybrid_raster.so")

HR_OK, HR_ERR_INVALID_ARGUMENT, HR_ERR_CAPACITY, HR_ERR_HIP, HR_ERR_UNSUPPORTED, HR_ERR_INTERNAL = range(6)
HR_FLAG_NO_SYNC = 1 << 0
HR_FLAG_DETACH_MASK = 1 << 1
HR_FLAG_EXPORT_KEYS = 1 << 2
HR_FLAG_CULL_BEHIND_MESH = 1 << 3
HR_FLAG_MIP_2D = 1 << 4
HR_FLAG_TILE_ELLIPSE = 1 << 5
HR_FLAG_MESH_REUSED = 1 << 6
HR_N_STAGES = 7
STAGES = ("projection", "depth_sort", "binning", "blend", "stats", "mesh", "forward")
HR_N_BWD_STAGES = 4
BWD_STAGES = ("blend_backward", "projection_backward", "texture_backward", "backward")

P = C.c_void_p


class hr_gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("means", P), ("log_scales", P),
                ("quats", P), ("opacity_logits", P), ("sh", P), ("filter3d", P)]


class hr_mesh(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_faces", C.c_int32), ("n_tex", C.c_int32),
                ("tex_h", C.c_int32), ("tex_w", C.c_int32), ("verts", P), ("faces", P),
                ("uvs", P), ("face_tex", P), ("tex", P)]


class hr_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("R", C.c_double * 9), ("t", C.c_double * 3)]


class hr_settings(C.Structure):
    _fields_ = [("bg", C.c_float * 3), ("low_pass", C.c_float), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("t_min", C.c_float), ("near_gs", C.c_float),
                ("near_mesh", C.c_float), ("clamp_fov", C.c_float), ("flags", C.c_uint32),
                ("batch", C.c_int32), ("variant", C.c_int32), ("batch_bwd", C.c_int32)]


class hr_outputs(C.Structure):
    _fields_ = [(k, P) for k in ("image", "final_T", "mesh_rgb", "mesh_depth", "tri_id",
                                 "n_contrib", "n_blended", "n_processed", "radii", "keys",
                                 "values", "ranges", "stats")]


class hr_grads(C.Structure):
    _fields_ = [(k, P) for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex",
                                 "mean2d_norm", "mean2d_count")]


class hr_adam_group(C.Structure):
    _fields_ = [("param", P), ("grad", P), ("m", P), ("v", P), ("n", C.c_int64), ("lr", C.c_float),
                ("lr_head", C.c_float), ("head", C.c_int32), ("row", C.c_int32)]


EXPORTED = ["hr_default_settings", "hr_query_workspace", "hr_render_hybrid", "hr_render_hybrid_timed",
            "hr_render_hybrid_backward", "hr_render_hybrid_backward_timed", "hr_blend_forward", "hr_loss_scratch_bytes", "hr_hybrid_loss",
            "hr_hybrid_loss_noalloc",
            "hr_full_loss_scratch_bytes", "hr_full_loss", "hr_adam_step", "hr_mip_filter3d", "hr_autotune", "hr_autotune_backward",
            "hr_autotune_key", "hr_autotune_cache_lookup", "hr_autotune_cache_store",
            "hr_batch_create", "hr_batch_launch", "hr_batch_status", "hr_batch_destroy",
            "hr_status_string",
            "hr_last_error", "hr_abi_version"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2506_06988_amd/build.py")
    L = C.CDLL(path)
    L.hr_default_settings.restype = hr_settings
    L.hr_default_settings.argtypes = []
    L.hr_query_workspace.restype = C.c_size_t
    L.hr_query_workspace.argtypes = [P, P, P, C.c_int32, P, C.c_int64]
    L.hr_render_hybrid.restype = C.c_int
    L.hr_render_hybrid.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t, P, P]
    L.hr_render_hybrid_timed.restype = C.c_int
    L.hr_render_hybrid_timed.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t, P, P, P]
    L.hr_render_hybrid_backward.restype = C.c_int
    L.hr_render_hybrid_backward.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t, P, P,
                                            P, P, P]
    L.hr_render_hybrid_backward_timed.restype = C.c_int
    L.hr_render_hybrid_backward_timed.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t,
                                                  P, P, P, P, P, C.c_int32, P]
    L.hr_blend_forward.restype = C.c_int
    L.hr_blend_forward.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t, P, P]
    L.hr_loss_scratch_bytes.restype = C.c_size_t
    L.hr_loss_scratch_bytes.argtypes = [P, C.c_int32]
    L.hr_hybrid_loss.restype = C.c_int
    L.hr_hybrid_loss.argtypes = [P, P, P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_uint32, P,
                                 P, P, P, P, P]
    L.hr_hybrid_loss_noalloc.restype = C.c_int
    L.hr_hybrid_loss_noalloc.argtypes = [P, P, P, P, P, P, C.c_int32, C.c_float, C.c_float,
                                         C.c_uint32, P, P, P, P, P]
    L.hr_mip_filter3d.restype = C.c_int
    L.hr_mip_filter3d.argtypes = [P, P, C.c_int32, P, C.c_double, P, P]
    L.hr_adam_step.restype = C.c_int
    L.hr_adam_step.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, P]
    L.hr_full_loss_scratch_bytes.restype = C.c_size_t
    L.hr_full_loss_scratch_bytes.argtypes = [P, C.c_int32]
    L.hr_full_loss.restype = C.c_int
    L.hr_full_loss.argtypes = [P, P, P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float,
                               C.c_int32, C.c_uint32, P, P, P, P, P, P]
    L.hr_autotune_backward.restype = C.c_int
    L.hr_autotune_backward.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t, P, P,
                                       C.c_int32, P]
    L.hr_autotune_key.restype = C.c_size_t
    L.hr_autotune_key.argtypes = [C.c_char_p, C.c_int32, P, P, P, C.c_int32, P, C.c_int32,
                                  C.c_char_p, C.c_size_t]
    L.hr_autotune_cache_lookup.restype = C.c_int32
    L.hr_autotune_cache_lookup.argtypes = [C.c_char_p, C.c_char_p, P, P]
    L.hr_autotune_cache_store.restype = C.c_int
    L.hr_autotune_cache_store.argtypes = [C.c_char_p, C.c_char_p, C.c_int32, C.c_int32]
    L.hr_autotune.restype = C.c_int
    L.hr_autotune.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t, P, C.c_int32, P]
    L.hr_batch_create.restype = C.c_int
    L.hr_batch_create.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, C.c_size_t, P, P, C.c_float,
                                  C.c_float, P, P, P, P, P, P, P, P]
    L.hr_batch_launch.restype = C.c_int
    L.hr_batch_launch.argtypes = [P, P]
    L.hr_batch_status.restype = C.c_int
    L.hr_batch_status.argtypes = [P, P, P]
    L.hr_batch_destroy.restype = None
    L.hr_batch_destroy.argtypes = [P]
    L.hr_status_string.restype = C.c_char_p
    L.hr_status_string.argtypes = [C.c_int]
    L.hr_last_error.restype = C.c_char_p
    L.hr_last_error.argtypes = []
    L.hr_abi_version.restype = C.c_int32
    L.hr_abi_version.argtypes = []
    _lib = L
    return L


class HRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(rc):
    if rc != HR_OK:
        raise HRError(rc, load().hr_last_error().decode())


def default_settings(**kw) -> hr_settings:
    s = load().hr_default_settings()
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                s.bg[i] = float(v[i])
        else:
            setattr(s, k, v)
    return s


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------- device data --
@dataclasses.dataclass
class DevGaussians:
    means: "torch.Tensor"
    log_scales: "torch.Tensor"
    quats: "torch.Tensor"
    opacity_logits: "torch.Tensor"
    sh: "torch.Tensor"
    sh_degree: int
    filter3d: Optional["torch.Tensor"] = None  # [n] Mip-Splatting 3D smoothing variance

    @property
    def n(self):
        return int(self.means.shape[0])

    def struct(self) -> hr_gaussians:
        g = hr_gaussians()
        g.n, g.sh_degree = self.n, self.sh_degree
        g.means, g.log_scales, g.quats = _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats)
        g.opacity_logits, g.sh = _ptr(self.opacity_logits), _ptr(self.sh)
        if self.filter3d is not None:
            assert self.filter3d.numel() == self.n and self.filter3d.is_contiguous()
        g.filter3d = _ptr(self.filter3d)
        return g


@dataclasses.dataclass
class DevMesh:
    verts: "torch.Tensor"
    faces: "torch.Tensor"
    uvs: "torch.Tensor"
    face_tex: "torch.Tensor"
    tex: "torch.Tensor"

    @property
    def n_faces(self):
        return int(self.faces.shape[0])

    def struct(self, tex=None) -> hr_mesh:
        m = hr_mesh()
        t = self.tex if tex is None else tex
        m.n_verts, m.n_faces = int(self.verts.shape[0]), self.n_faces
        m.n_tex, m.tex_h, m.tex_w = int(t.shape[0]), int(t.shape[1]), int(t.shape[2])
        m.verts, m.faces, m.uvs = _ptr(self.verts), _ptr(self.faces), _ptr(self.uvs)
        m.face_tex, m.tex = _ptr(self.face_tex), _ptr(t)
        return m


def to_device(gaussians, mesh=None, device="cuda"):
    import torch
    f = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt).contiguous()
    g = DevGaussians(f(gaussians.means), f(gaussians.log_scales), f(gaussians.quats),
                     f(gaussians.opacity_logits), f(gaussians.sh), gaussians.sh_degree)
    m = None
    if mesh is not None and mesh.faces.shape[0] > 0:
        m = DevMesh(f(mesh.verts), f(mesh.faces, torch.int32), f(mesh.uvs),
                    f(mesh.face_tex, torch.int32), f(mesh.tex))
    return g, m


def empty_mesh_struct() -> hr_mesh:
    m = hr_mesh()
    m.n_verts = m.n_faces = 0
    m.n_tex = m.tex_h = m.tex_w = 1
    return m


def camera_array(cams: Sequence) -> "C.Array":
    arr = (hr_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].width, arr[i].height = int(c.width), int(c.height)
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        R = np.asarray(c.R, np.float64).reshape(9)
        t = np.asarray(c.t, np.float64).reshape(3)
        for k in range(9):
            arr[i].R[k] = R[k]
        for k in range(3):
            arr[i].t[k] = t[k]
    return arr


def pixel_offsets(cams) -> List[int]:
    off, o = [], 0
    for c in cams:
        off.append(o)
        o += int(c.width) * int(c.height)
    off.append(o)
    return off


def n_tiles(cams, tile=16) -> int:
    return sum(((c.width + tile - 1) // tile) * ((c.height + tile - 1) // tile) for c in cams)


# ------------------------------------------------------------- the renderer --
@dataclasses.dataclass
class Frame:
    """Outputs of one forward, packed over cameras (see hr.h)."""
    image: "torch.Tensor"
    final_T: "torch.Tensor"
    mesh_rgb: "torch.Tensor"
    mesh_depth: "torch.Tensor"
    tri_id: "torch.Tensor"
    n_contrib: "torch.Tensor"
    n_blended: "torch.Tensor"
    n_processed: "torch.Tensor"
    radii: "torch.Tensor"
    stats: "torch.Tensor"
    keys: Optional["torch.Tensor"] = None
    values: Optional["torch.Tensor"] = None
    ranges: Optional["torch.Tensor"] = None
    offsets: Optional[List[int]] = None

    def view(self, c, cams):
        """(image [3,H,W], T [H,W], mesh_rgb, mesh_depth, tri_id, n_contrib, n_blended, n_processed)."""
        o0 = self.offsets[c]
        H, W = int(cams[c].height), int(cams[c].width)
        hw = H * W
        im = self.image[3 * o0:3 * o0 + 3 * hw].view(3, H, W)
        mr = self.mesh_rgb[3 * o0:3 * o0 + 3 * hw].view(3, H, W)
        sl = lambda t: t[o0:o0 + hw].view(H, W)
        return (im, sl(self.final_T), mr, sl(self.mesh_depth), sl(self.tri_id), sl(self.n_contrib),
                sl(self.n_blended), sl(self.n_processed))

    def stats_dict(self):
        return stats_to_dict(self.stats.cpu().numpy())


class hr_stats(C.Structure):
    _fields_ = [("n_visible", C.c_uint32), ("n_keys", C.c_uint32), ("overflow", C.c_uint32),
                ("n_tris", C.c_uint32), ("n_processed", C.c_uint64), ("n_blended", C.c_uint64),
                ("wait_limit", C.c_uint32), ("reserved", C.c_uint32)]


STATS_WORDS = C.sizeof(hr_stats) // 8


def stats_to_dict(raw) -> dict:
    st = hr_stats.from_buffer_copy(np.ascontiguousarray(raw).tobytes()[:C.sizeof(hr_stats)])
    return {k: int(getattr(st, k)) for k, _ in hr_stats._fields_ if k != "reserved"}


@dataclasses.dataclass
class Context:
    """What one forward leaves for its backward: the Gaussian and texture
    tensors it read, its workspace (the library's saved context), the key
    capacity and settings that workspace was laid out for, and the cameras."""
    g: DevGaussians
    tex: Optional["torch.Tensor"]
    ws: "torch.Tensor"
    key_capacity: int
    settings: hr_settings
    cam_arr: "C.Array"
    n_cams: int


class Renderer:
    """One scene/camera configuration: its Gaussians, mesh, cameras, settings and
    a reusable workspace. The autograd path (`forward_context`) gives every
    forward a workspace of its own instead."""

    def __init__(self, gaussians: DevGaussians, mesh: Optional[DevMesh], cams, settings=None,
                 key_capacity: Optional[int] = None):
        self.L = load()
        self.g = gaussians
        self.mesh = mesh
        self.cams = list(cams)
        self.cam_arr = camera_array(self.cams)
        self.settings = settings if settings is not None else default_settings()
        self.offsets = pixel_offsets(self.cams)
        self.P = self.offsets[-1]
        self.tiles = n_tiles(self.cams)
        self.device = gaussians.means.device
        if key_capacity is None:
            key_capacity = max(1 << 16, 64 * self.P)
        self.key_capacity = int(min(key_capacity, 0xffffffff))
        self.ws = None
        self._alloc_ws()

    @property
    def sizes(self):
        return [(int(c.width), int(c.height)) for c in self.cams]

    def _structs(self, tex=None, g=None):
        gs = (self.g if g is None else g).struct()
        ms = self.mesh.struct(tex) if self.mesh is not None else empty_mesh_struct()
        return gs, ms

    def workspace_bytes(self, key_capacity=None, g=None) -> int:
        gs, ms = self._structs(g=g)
        cap = self.key_capacity if key_capacity is None else int(key_capacity)
        nbytes = int(self.L.hr_query_workspace(C.byref(gs), C.byref(ms), self.cam_arr,
                                               len(self.cams), C.byref(self.settings), cap))
        if nbytes == 0:
            raise HRError(HR_ERR_INVALID_ARGUMENT, self.L.hr_last_error().decode())
        return nbytes

    def _alloc_ws(self):
        import torch
        nbytes = self.workspace_bytes()
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = None
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ws_bytes = int(self.ws.numel())

    def grow_capacity(self, needed: int):
        """Key capacity for `needed` pairs plus a quarter; regrows the workspace."""
        self.key_capacity = int(min(0xffffffff, int(needed) * 5 // 4 + 1024))
        self._alloc_ws()

    def new_frame(self, export_keys=False) -> Frame:
        import torch
        d = self.device
        P, n = self.P, self.g.n
        f = Frame(image=torch.empty(3 * P, dtype=torch.float32, device=d),
                  final_T=torch.empty(P, dtype=torch.float32, device=d),
                  mesh_rgb=torch.empty(3 * P, dtype=torch.float32, device=d),
                  mesh_depth=torch.empty(P, dtype=torch.float32, device=d),
                  tri_id=torch.empty(P, dtype=torch.int32, device=d),
                  n_contrib=torch.empty(P, dtype=torch.int32, device=d),
                  n_blended=torch.empty(P, dtype=torch.int32, device=d),
                  n_processed=torch.empty(P, dtype=torch.int32, device=d),
                  radii=torch.empty(max(1, n * len(self.cams)), dtype=torch.int32, device=d),
                  stats=torch.zeros(STATS_WORDS, dtype=torch.int64, device=d), offsets=self.offsets)
        if export_keys:
            f.keys = torch.empty(self.key_capacity, dtype=torch.int64, device=d)
            f.values = torch.empty(self.key_capacity, dtype=torch.int32, device=d)
            f.ranges = torch.empty(2 * self.tiles, dtype=torch.int32, device=d)
        return f

    def outputs_struct(self, f: Frame) -> hr_outputs:
        o = hr_outputs()
        o.image, o.final_T, o.mesh_rgb = _ptr(f.image), _ptr(f.final_T), _ptr(f.mesh_rgb)
        o.mesh_depth, o.tri_id, o.n_contrib = _ptr(f.mesh_depth), _ptr(f.tri_id), _ptr(f.n_contrib)
        o.n_blended, o.n_processed, o.radii = _ptr(f.n_blended), _ptr(f.n_processed), _ptr(f.radii)
        o.keys, o.values, o.ranges = _ptr(f.keys), _ptr(f.values), _ptr(f.ranges)
        o.stats = _ptr(f.stats)
        return o

    def _forward(self, f: Frame, g: DevGaussians, tex, ws, cap: int, sync_check: bool):
        gs, ms = self._structs(tex, g)
        o = self.outputs_struct(f)
        s = hr_settings.from_buffer_copy(self.settings)
        if not sync_check:
            s.flags |= HR_FLAG_NO_SYNC
        return self.L.hr_render_hybrid(C.byref(gs), C.byref(ms), self.cam_arr, len(self.cams),
                                       C.byref(s), int(cap), _ptr(ws), int(ws.numel()), C.byref(o),
                                       _stream())

    def render_hybrid(self, frame: Optional[Frame] = None, export_keys=False, tex=None,
                      sync_check=True) -> Frame:
        """hr_render_hybrid into the renderer's workspace; grows the key capacity
        and retries on HR_ERR_CAPACITY."""
        f = frame if frame is not None else self.new_frame(export_keys)
        for _ in range(3):
            rc = self._forward(f, self.g, tex, self.ws, self.key_capacity, sync_check)
            if rc != HR_ERR_CAPACITY:
                check(rc)
                return f
            self.grow_capacity(f.stats_dict()["n_keys"])
            if export_keys:
                f = self.new_frame(export_keys)
        raise HRError(HR_ERR_CAPACITY, "key capacity did not converge")

    def render_hybrid_timed(self, frame: Frame, mesh_reused=False) -> dict:
        """hr_render_hybrid_timed into the renderer's workspace (synchronises);
        returns the stage times in milliseconds."""
        gs, ms = self._structs()
        o = self.outputs_struct(frame)
        s = hr_settings.from_buffer_copy(self.settings)
        if mesh_reused:
            s.flags |= HR_FLAG_MESH_REUSED
        out = (C.c_float * HR_N_STAGES)()
        check(self.L.hr_render_hybrid_timed(C.byref(gs), C.byref(ms), self.cam_arr, len(self.cams),
                                            C.byref(s), self.key_capacity, _ptr(self.ws),
                                            self.ws_bytes, C.byref(o), _stream(), out))
        return {k: float(out[i]) for i, k in enumerate(STAGES)}

    def forward_context(self, g: DevGaussians, tex=None):
        """hr_render_hybrid of Gaussians `g` (and texture `tex`) into a workspace
        of its own; the renderer's Gaussians and workspace are left as they are.
        Returns (frame, Context) for backward_context."""
        import torch
        f = self.new_frame()
        cap = self.key_capacity
        for _ in range(3):
            ws = torch.empty(self.workspace_bytes(cap, g), dtype=torch.uint8, device=self.device)
            rc = self._forward(f, g, tex, ws, cap, True)
            if rc != HR_ERR_CAPACITY:
                check(rc)
                ctx = Context(g, tex, ws, cap, hr_settings.from_buffer_copy(self.settings),
                              self.cam_arr, len(self.cams))
                return f, ctx
            cap = int(min(0xffffffff, f.stats_dict()["n_keys"] * 5 // 4 + 1024))
            self.key_capacity = max(self.key_capacity, cap)  # a hint for later forwards
        raise HRError(HR_ERR_CAPACITY, "key capacity did not converge")

    def _zero_grads(self, g: DevGaussians, tex=None):
        import torch
        grads = dict(means=torch.zeros_like(g.means), log_scales=torch.zeros_like(g.log_scales),
                     quats=torch.zeros_like(g.quats),
                     opacity_logits=torch.zeros_like(g.opacity_logits), sh=torch.zeros_like(g.sh))
        if self.mesh is not None:
            grads["tex"] = torch.zeros_like(self.mesh.tex if tex is None else tex)
        return grads

    def _backward(self, g, tex, ws, cap, settings, cam_arr, n_cams, grad_image, grad_final_T,
                  grad_mesh_rgb, grads):
        gr = hr_grads()
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex", "mean2d_norm",
                  "mean2d_count"):
            setattr(gr, k, _ptr(grads.get(k)))
        gs, ms = self._structs(tex, g)
        check(self.L.hr_render_hybrid_backward(
            C.byref(gs), C.byref(ms), cam_arr, n_cams, C.byref(settings), int(cap), _ptr(ws),
            int(ws.numel()), _ptr(grad_image.contiguous()),
            _ptr(None if grad_final_T is None else grad_final_T.contiguous()),
            _ptr(None if grad_mesh_rgb is None else grad_mesh_rgb.contiguous()), C.byref(gr),
            _stream()))
        return grads

    def render_hybrid_backward_timed(self, grad_image, grad_final_T=None, grad_mesh_rgb=None,
                                     serial=True):
        """hr_render_hybrid_backward_timed of the last render_hybrid; returns the
        stage times in ms keyed by BWD_STAGES, and the gradients (fresh tensors)."""
        grads = self._zero_grads(self.g)
        gr = hr_grads()
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex", "mean2d_norm",
                  "mean2d_count"):
            setattr(gr, k, _ptr(grads.get(k)))
        gs, ms = self._structs()
        t = (C.c_float * HR_N_BWD_STAGES)()
        check(self.L.hr_render_hybrid_backward_timed(
            C.byref(gs), C.byref(ms), self.cam_arr, len(self.cams), C.byref(self.settings),
            int(self.key_capacity), _ptr(self.ws), int(self.ws.numel()),
            _ptr(grad_image.contiguous()),
            _ptr(None if grad_final_T is None else grad_final_T.contiguous()),
            _ptr(None if grad_mesh_rgb is None else grad_mesh_rgb.contiguous()), C.byref(gr),
            _stream(), 1 if serial else 0, t))
        return dict(zip(BWD_STAGES, list(t))), grads

    def render_hybrid_backward(self, grad_image, grad_final_T=None, grad_mesh_rgb=None, grads=None,
                               tex=None):
        """hr_render_hybrid_backward of the last render_hybrid; returns a dict of
        gradient tensors (accumulated into `grads`)."""
        grads = self._zero_grads(self.g, tex) if grads is None else grads
        return self._backward(self.g, tex, self.ws, self.key_capacity, self.settings, self.cam_arr,
                              len(self.cams), grad_image, grad_final_T, grad_mesh_rgb, grads)

    def backward_context(self, ctx: Context, grad_image, grad_final_T=None, grad_mesh_rgb=None,
                         grads=None):
        """hr_render_hybrid_backward of the forward that produced `ctx`."""
        grads = self._zero_grads(ctx.g, ctx.tex) if grads is None else grads
        return self._backward(ctx.g, ctx.tex, ctx.ws, ctx.key_capacity, ctx.settings, ctx.cam_arr,
                              ctx.n_cams, grad_image, grad_final_T, grad_mesh_rgb, grads)

    def set_cameras(self, cams):
        """Switch to other cameras of the same sizes (the workspace is reused)."""
        cams = list(cams)
        assert [(c.width, c.height) for c in cams] == [(c.width, c.height) for c in self.cams]
        self.cams = cams
        self.cam_arr = camera_array(cams)

    def blend_forward(self, frame: Frame):
        """hr_blend_forward: re-run only the blend of the last forward."""
        gs, ms = self._structs()
        o = self.outputs_struct(frame)
        check(self.L.hr_blend_forward(C.byref(gs), C.byref(ms), self.cam_arr, len(self.cams),
                                      C.byref(self.settings), self.key_capacity, _ptr(self.ws),
                                      self.ws_bytes, C.byref(o), _stream()))

    def autotune(self, frame: Frame, repeats=5):
        gs, ms = self._structs()
        o = self.outputs_struct(frame)
        check(self.L.hr_autotune(C.byref(gs), C.byref(ms), self.cam_arr, len(self.cams),
                                 C.byref(self.settings), self.key_capacity, _ptr(self.ws),
                                 self.ws_bytes, C.byref(o), int(repeats), _stream()))
        return int(self.settings.batch), int(self.settings.variant)

    def autotune_backward(self, grad_image, grad_final_T=None, repeats=5):
        """hr_autotune_backward after a forward of this renderer; returns (batch_bwd, variant)."""
        gs, ms = self._structs()
        check(self.L.hr_autotune_backward(
            C.byref(gs), C.byref(ms), self.cam_arr, len(self.cams), C.byref(self.settings),
            self.key_capacity, _ptr(self.ws), self.ws_bytes, _ptr(grad_image.contiguous()),
            _ptr(None if grad_final_T is None else grad_final_T.contiguous()), int(repeats),
            _stream()))
        return int(self.settings.batch_bwd), int(self.settings.variant)


def _sizes_array(sizes):
    return (C.c_int32 * (2 * len(sizes)))(*[int(v) for wh in sizes for v in wh])


def loss_scratch_bytes(sizes) -> int:
    nb = int(load().hr_loss_scratch_bytes(_sizes_array(sizes), len(sizes)))
    if nb == 0:
        raise HRError(HR_ERR_INVALID_ARGUMENT, "invalid image sizes")
    return nb


def hybrid_loss(image, final_T, mesh_rgb, tri_id, target, sizes=None, lambda_t=0.1, k=20.0,
                detach_mask=False, out=None):
    """hr_hybrid_loss over images packed like the renderer's outputs; `sizes` is
    the (width, height) of each image (default: one planar image of all pixels).
    `out` = (loss, g_image, g_T, g_mesh_rgb, scratch) reuses buffers (else they
    are allocated). Returns (loss, g_image, g_T, g_mesh_rgb)."""
    import torch
    L = load()
    n_pix = int(final_T.numel())
    sizes = [(n_pix, 1)] if sizes is None else [(int(w), int(h)) for (w, h) in sizes]
    assert sum(w * h for w, h in sizes) == n_pix, "sizes do not cover the pixels"
    d = image.device
    if out is None:
        out = (torch.zeros(1, dtype=torch.float32, device=d), torch.empty_like(image),
               torch.empty_like(final_T), torch.empty_like(mesh_rgb),
               torch.empty(loss_scratch_bytes(sizes), dtype=torch.uint8, device=d))
    loss, gi, gt, gm, scratch = out
    sz = _sizes_array(sizes)
    check(L.hr_hybrid_loss(_ptr(image), _ptr(final_T), _ptr(mesh_rgb), _ptr(tri_id), _ptr(target),
                           sz, len(sizes), float(lambda_t), float(k),
                           HR_FLAG_DETACH_MASK if detach_mask else 0, _ptr(loss), _ptr(gi), _ptr(gt),
                           _ptr(gm), _ptr(scratch), _stream()))
    return loss, gi, gt, gm


MASK_MODES = {"none": 0, "one": 1, "T": 2, "sigmoid": 3}


def mip_filter3d(gaussians: DevGaussians, cams, settings=None, scale=0.2, out=None):
    """hr_mip_filter3d: the Mip-Splatting 3D smoothing variance [n] for these views."""
    import torch
    out = torch.empty(gaussians.n, dtype=torch.float32, device=gaussians.means.device) if out is None else out
    st = settings if settings is not None else default_settings()
    g = gaussians.struct()
    check(load().hr_mip_filter3d(C.byref(g), camera_array(cams), len(cams), C.byref(st),
                                 float(scale), _ptr(out), _stream()))
    return out


def adam_step(groups, step, beta1=0.9, beta2=0.999, eps=1e-15):
    """hr_adam_step over [(param, grad, m, v, lr[, lr_head, head, row]), ...]
    (contiguous float32 device tensors of equal sizes within a group)."""
    arr = (hr_adam_group * len(groups))()
    for i, grp in enumerate(groups):
        p_, g_, m_, v_, lr = grp[:5]
        lr_head, head, row = grp[5:] if len(grp) > 5 else (lr, 0, 0)
        for t in (g_, m_, v_):
            assert t.numel() == p_.numel() and t.is_contiguous() and t.dtype == p_.dtype
        assert p_.is_contiguous()
        arr[i].param, arr[i].grad, arr[i].m, arr[i].v = _ptr(p_), _ptr(g_), _ptr(m_), _ptr(v_)
        arr[i].n, arr[i].lr = int(p_.numel()), float(lr)
        arr[i].lr_head, arr[i].head, arr[i].row = float(lr_head), int(head), int(row)
    check(load().hr_adam_step(arr, len(groups), float(beta1), float(beta2), float(eps), int(step),
                              _stream()))


def full_loss(image, final_T, mesh_rgb, tri_id, target, sizes, lambda_c=0.2, lambda_t=0.1, k=20.0,
              mask_mode="sigmoid", detach_mask=False):
    """hr_full_loss (Eq. 3 + transmittance-aware term) over packed images of the
    given (width, height) sizes; returns (loss, g_image, g_T, g_mesh_rgb)."""
    import torch
    L = load()
    sz = _sizes_array(sizes)
    d = image.device
    loss = torch.zeros(1, dtype=torch.float32, device=d)
    gi = torch.empty_like(image)
    gt = torch.empty_like(final_T)
    gm = torch.empty_like(mesh_rgb)
    nb = int(L.hr_full_loss_scratch_bytes(sz, len(sizes)))
    if nb == 0:
        raise HRError(HR_ERR_INVALID_ARGUMENT, "invalid image sizes")
    scratch = torch.empty(nb, dtype=torch.uint8, device=d)
    check(L.hr_full_loss(_ptr(image), _ptr(final_T), _ptr(mesh_rgb), _ptr(tri_id), _ptr(target), sz,
                         len(sizes), float(lambda_c), float(lambda_t), float(k),
                         MASK_MODES[mask_mode], HR_FLAG_DETACH_MASK if detach_mask else 0,
                         _ptr(loss), _ptr(gi), _ptr(gt), _ptr(gm), _ptr(scratch), _stream()))
    return loss, gi, gt, gm


# --------------------------------------------------------------- autograd --
def _autograd_fn():
    import torch

    class HybridRenderFn(torch.autograd.Function):
        """(renderer, means, log_scales, quats, opacity_logits, sh, tex)
        -> (image, final_T, mesh_rgb, tri_id), packed over the renderer's cameras.

        image, final_T and mesh_rgb are differentiable (T through the
        transmittance-aware loss, I_m into the texture); tri_id is not. Each
        call renders into a workspace of its own, kept in ctx with the tensors
        it read, so several forwards may precede their backwards. The renderer
        supplies the mesh, cameras and settings and is not modified (except
        for its key-capacity hint)."""

        @staticmethod
        def forward(ctx, renderer, means, log_scales, quats, opacity_logits, sh, tex):
            g = DevGaussians(means.detach().contiguous(), log_scales.detach().contiguous(),
                             quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                             sh.detach().contiguous(), renderer.g.sh_degree, renderer.g.filter3d)
            t = None if tex is None else tex.detach().contiguous()
            f, c = renderer.forward_context(g, t)
            ctx.renderer = renderer
            ctx.hr_ctx = c
            ctx.mark_non_differentiable(f.tri_id)
            return f.image, f.final_T, f.mesh_rgb, f.tri_id

        @staticmethod
        def backward(ctx, g_image, g_T, g_mesh, g_tri):
            c = ctx.hr_ctx
            if g_image is None:
                g_image = torch.zeros(3 * ctx.renderer.P, dtype=torch.float32,
                                      device=c.g.means.device)
            grads = ctx.renderer.backward_context(c, g_image, g_T, g_mesh)
            ctx.hr_ctx = None  # the workspace is released with the graph
            return (None, grads["means"], grads["log_scales"], grads["quats"],
                    grads["opacity_logits"], grads["sh"], grads.get("tex"))

    return HybridRenderFn


def _loss_fn():
    import torch

    class HybridLossFn(torch.autograd.Function):
        """(image, final_T, mesh_rgb, tri_id, target, sizes, lambda_t, k, detach_mask)
        -> loss [1]: hr_hybrid_loss; its backward scales the kernel's dL/dI_h,
        dL/dT and dL/dI_m by the incoming gradient."""

        @staticmethod
        def forward(ctx, image, final_T, mesh_rgb, tri_id, target, sizes=None, lambda_t=0.1,
                    k=20.0, detach_mask=False):
            L, gi, gt, gm = hybrid_loss(image.detach().contiguous(), final_T.detach().contiguous(),
                                        mesh_rgb.detach().contiguous(), tri_id.contiguous(),
                                        target.detach().contiguous(), sizes, lambda_t, k,
                                        detach_mask)
            ctx.save_for_backward(gi, gt, gm)
            return L

        @staticmethod
        def backward(ctx, g):
            gi, gt, gm = ctx.saved_tensors
            return (gi * g, gt * g, gm * g, None, None, None, None, None, None)

    return HybridLossFn


_HybridRenderFn = None
_HybridLossFn = None


def HybridRenderFn():
    global _HybridRenderFn
    if _HybridRenderFn is None:
        _HybridRenderFn = _autograd_fn()
    return _HybridRenderFn


def HybridLossFn():
    global _HybridLossFn
    if _HybridLossFn is None:
        _HybridLossFn = _loss_fn()
    return _HybridLossFn


# ---------------------------------------------------------- batched graph --
class BatchedStep:
    """hr_batch_create / hr_batch_launch / hr_batch_status: forward + loss +
    backward of all the renderer's cameras in one hipGraph.

    `launch()` replays the graph; `check()` waits for it and reads the
    forward's device flags; `step()` does both and, when the pair count
    outgrew the key capacity, regrows the renderer's workspace, captures the
    graph again and replays it."""

    def __init__(self, renderer: Renderer, target, lambda_t=0.1, k=20.0, stream=None):
        import torch
        r = renderer
        self.r = r
        self.L = load()
        d = r.device
        self.lambda_t, self.k = float(lambda_t), float(k)
        self.frame = r.new_frame()
        self.target = target.contiguous()
        self.loss = torch.zeros(1, dtype=torch.float32, device=d)
        self.g_image = torch.empty(3 * r.P, dtype=torch.float32, device=d)
        self.g_T = torch.empty(r.P, dtype=torch.float32, device=d)
        self.g_mesh = torch.empty(3 * r.P, dtype=torch.float32, device=d)
        self.scratch = torch.empty(loss_scratch_bytes(r.sizes), dtype=torch.uint8, device=d)
        self.grads = r._zero_grads(r.g)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.recaptures = 0
        self.handle = None
        self._capture()

    def _capture(self):
        import torch
        r = self.r
        gr = hr_grads()
        for k_ in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex"):
            setattr(gr, k_, _ptr(self.grads.get(k_)))
        gs, ms = r._structs()
        o = r.outputs_struct(self.frame)
        s = hr_settings.from_buffer_copy(r.settings)
        s.flags |= HR_FLAG_NO_SYNC
        self._keep = (gs, ms, o, s, gr)
        h = C.c_void_p()
        torch.cuda.synchronize()
        check(self.L.hr_batch_create(C.byref(gs), C.byref(ms), r.cam_arr, len(r.cams), C.byref(s),
                                     r.key_capacity, _ptr(r.ws), r.ws_bytes, C.byref(o),
                                     _ptr(self.target), self.lambda_t, self.k, _ptr(self.loss),
                                     _ptr(self.g_image), _ptr(self.g_T), _ptr(self.g_mesh),
                                     _ptr(self.scratch), C.byref(gr),
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def launch(self):
        check(self.L.hr_batch_launch(self.handle, C.c_void_p(self.stream.cuda_stream)))

    def check(self) -> dict:
        """hr_batch_status: waits for the replays and raises HRError on a flag."""
        st = hr_stats()
        rc = self.L.hr_batch_status(self.handle, C.byref(st), C.c_void_p(self.stream.cuda_stream))
        self.last_stats = {k: int(getattr(st, k)) for k, _ in hr_stats._fields_ if k != "reserved"}
        check(rc)
        return self.last_stats

    def step(self, max_recaptures=3):
        """One checked replay; on HR_ERR_CAPACITY regrow, re-capture and replay."""
        for _ in range(max_recaptures + 1):
            self.launch()
            try:
                return self.check()
            except HRError as e:
                if e.status != HR_ERR_CAPACITY:
                    raise
                self.close()
                self.r.grow_capacity(self.last_stats["n_keys"])
                self._capture()
                self.recaptures += 1
        raise HRError(HR_ERR_CAPACITY, "key capacity did not converge")

    def close(self):
        if self.handle:
            self.L.hr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
