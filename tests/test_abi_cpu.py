"""The C ABI without a GPU: symbols, host-side validation and workspace planning."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2506_06988_amd import hr, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "hr.h")).read()
    return sorted(set(re.findall(r"\b(hr_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = hr.load()
    names = header_functions()
    assert "hr_render_hybrid" in names and "hr_render_hybrid_backward" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.hr_abi_version() == 2
    assert set(names) <= set(hr.EXPORTED) | {"hr_default_settings"}


def _structs(n=10, deg=0, faces=0):
    g = hr.hr_gaussians()
    g.n, g.sh_degree = n, deg
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        setattr(g, k, 4096)
    m = hr.empty_mesh_struct()
    if faces:
        m.n_verts, m.n_faces, m.n_tex, m.tex_h, m.tex_w = 4, faces, 1, 8, 8
        for k in ("verts", "faces", "uvs", "face_tex", "tex"):
            setattr(m, k, 4096)
    return g, m


def test_workspace_grows_with_inputs_and_capacity():
    L = hr.load()
    s = hr.default_settings()
    cam = scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3), np.zeros(3))
    cams = hr.camera_array([cam])
    sizes = []
    for n, cap in ((10, 1000), (1000, 1000), (1000, 100000)):
        g, m = _structs(n)
        sizes.append(L.hr_query_workspace(C.byref(g), C.byref(m), cams, 1, C.byref(s), cap))
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    assert sizes[2] - sizes[1] >= 4 * 99000
    cams2 = hr.camera_array([cam, cam])
    g, m = _structs(1000)
    assert L.hr_query_workspace(C.byref(g), C.byref(m), cams2, 2, C.byref(s), 1000) > sizes[1]


@pytest.mark.parametrize("mutate, msg", [
    (lambda g, m, s, c: setattr(g, "sh_degree", 4), "sh_degree"),
    (lambda g, m, s, c: setattr(g, "n", -1), "n must"),
    (lambda g, m, s, c: setattr(g, "means", None), "null Gaussian"),
    (lambda g, m, s, c: setattr(g, "quats", 4100), "aligned"),
    (lambda g, m, s, c: setattr(s, "alpha_min", 0.995), "alpha"),
    (lambda g, m, s, c: setattr(s, "t_min", 0.0), "t_min"),
    (lambda g, m, s, c: setattr(s, "batch", 48), "batch"),
    (lambda g, m, s, c: setattr(c[0], "width", 0), "camera size"),
    (lambda g, m, s, c: setattr(c[0], "fx", -1.0), "focal"),
    (lambda g, m, s, c: setattr(c[0], "width", 8000) or setattr(c[0], "height", 8000), "16384 tiles"),
])
def test_invalid_arguments_are_rejected_before_any_launch(mutate, msg):
    L = hr.load()
    g, m = _structs(100)
    s = hr.default_settings()
    cams = hr.camera_array([scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3), np.zeros(3))])
    mutate(g, m, s, cams)
    assert L.hr_query_workspace(C.byref(g), C.byref(m), cams, 1, C.byref(s), 1000) == 0
    assert msg in L.hr_last_error().decode()
    # the render call fails the same way without touching the (bogus) pointers
    out = hr.hr_outputs()
    out.image = 4096
    rc = L.hr_render_hybrid(C.byref(g), C.byref(m), cams, 1, C.byref(s), 1000, 4096, 1 << 30,
                            C.byref(out), None)
    assert rc in (hr.HR_ERR_INVALID_ARGUMENT, hr.HR_ERR_UNSUPPORTED)


def test_mesh_arguments_and_capacity_bounds():
    L = hr.load()
    s = hr.default_settings()
    cams = hr.camera_array([scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3), np.zeros(3))])
    g, m = _structs(10, faces=2)
    assert L.hr_query_workspace(C.byref(g), C.byref(m), cams, 1, C.byref(s), 1000) > 0
    m.tex = None
    assert L.hr_query_workspace(C.byref(g), C.byref(m), cams, 1, C.byref(s), 1000) == 0
    g, m = _structs(10)
    assert L.hr_query_workspace(C.byref(g), C.byref(m), cams, 1, C.byref(s), 1 << 32) == 0
    assert L.hr_query_workspace(C.byref(g), C.byref(m), cams, 0, C.byref(s), 10) == 0


def test_status_strings():
    L = hr.load()
    for k in range(6):
        assert L.hr_status_string(k)
    assert L.hr_status_string(hr.HR_ERR_CAPACITY) == b"key capacity too small"


@pytest.mark.parametrize("n", [2, 8])
def test_bench_refuses_several_gpus(n):
    """The benchmark measures one GPU: asked for more it exits with status 2
    and a message, before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and f"asked for {n}" in r.stderr
    assert r.stdout == ""


def test_loss_sizes_and_arguments_are_checked_on_the_host():
    """hr_loss_scratch_bytes / hr_hybrid_loss: image sizes per packed image,
    rejected before any launch when invalid."""
    L = hr.load()
    sz = hr._sizes_array([(37, 29), (64, 48)])
    nb = L.hr_loss_scratch_bytes(sz, 2)
    P = 37 * 29 + 64 * 48
    # the image table (3 offsets) plus at least one partial sum per 1024 pixels
    assert nb >= 3 * 8 + ((P + 1023) // 1024 + 1) * 8
    assert L.hr_loss_scratch_bytes(hr._sizes_array([(0, 5)]), 1) == 0
    assert L.hr_loss_scratch_bytes(sz, 0) == 0
    assert L.hr_loss_scratch_bytes(None, 1) == 0
    rc = L.hr_hybrid_loss(4096, 4096, 4096, 4096, 4096, hr._sizes_array([(5, -1)]), 1, 0.1, 20.0,
                          0, 4096, 4096, 4096, 4096, 4096, None)
    assert rc == hr.HR_ERR_INVALID_ARGUMENT and b"size" in L.hr_last_error()
    rc = L.hr_hybrid_loss(4096, None, 4096, 4096, 4096, sz, 2, 0.1, 20.0, 0, 4096, 4096, 4096,
                          4096, 4096, None)
    assert rc == hr.HR_ERR_INVALID_ARGUMENT and b"null" in L.hr_last_error()


def test_stats_layout_and_batch_status_argument_check():
    L = hr.load()
    assert C.sizeof(hr.hr_stats) == 40 and hr.STATS_WORDS == 5
    raw = np.zeros(5, np.int64)
    raw.view(np.uint32)[[0, 1, 2, 3]] = (7, 9, 1, 4)
    raw[2], raw[3] = 123, 45
    raw.view(np.uint32)[8] = 1
    d = hr.stats_to_dict(raw)
    assert d == dict(n_visible=7, n_keys=9, overflow=1, n_tris=4, n_processed=123, n_blended=45,
                     wait_limit=1)
    st = hr.hr_stats()
    assert L.hr_batch_status(None, C.byref(st), None) == hr.HR_ERR_INVALID_ARGUMENT


def _key(L, n=600000, cams=None, flags=0, backward=0, faces=2, deg=3, arch=b"gfx950", cus=256):
    g, m = _structs(n, deg=deg, faces=faces)
    s = hr.default_settings(flags=flags)
    cams = cams or [scenes.Camera(1920, 1080, 1000.0, 1000.0, 960.0, 540.0, np.eye(3), np.zeros(3))]
    arr = hr.camera_array(cams)
    need = L.hr_autotune_key(arch, cus, C.byref(g), C.byref(m), arr, len(cams), C.byref(s),
                             backward, None, 0)
    buf = C.create_string_buffer(need)
    assert L.hr_autotune_key(arch, cus, C.byref(g), C.byref(m), arr, len(cams), C.byref(s),
                             backward, buf, need) == need
    return buf.value.decode()


def test_autotune_cache_key_classes():
    """The key names the device and the workload class: powers of two of the
    pixel, Gaussian and camera counts, SH degree, mesh presence and the flags
    that change the tile lists (other flags do not)."""
    L = hr.load()
    k = _key(L)
    assert k == "fwd|gfx950|cu256|px2^20|n2^19|cams2^0|sh3|mesh1|flags0", k
    assert _key(L, backward=1).startswith("bwd|")
    assert _key(L, n=700000) == k                   # same power of two
    assert _key(L, n=1 << 20) != k
    assert _key(L, flags=hr.HR_FLAG_TILE_ELLIPSE).endswith("flags32")
    assert _key(L, flags=hr.HR_FLAG_NO_SYNC | hr.HR_FLAG_EXPORT_KEYS) == k
    assert "mesh0" in _key(L, faces=0) and "sh0" in _key(L, deg=0)
    cam = scenes.Camera(640, 480, 500.0, 500.0, 320.0, 240.0, np.eye(3), np.zeros(3))
    assert "cams2^4" in _key(L, cams=[cam] * 16) and "px2^22" in _key(L, cams=[cam] * 16)
    assert "cu304" in _key(L, cus=304) and "gfx942" in _key(L, arch=b"gfx942")
    # a truncated buffer still holds a NUL-terminated prefix
    g, m = _structs(10)
    s = hr.default_settings()
    arr = hr.camera_array([cam])
    small = C.create_string_buffer(8)
    assert L.hr_autotune_key(b"gfx950", 256, C.byref(g), C.byref(m), arr, 1, C.byref(s), 0,
                             small, 8) > 8
    assert small.value == b"fwd|gfx"
    assert L.hr_autotune_key(None, 256, C.byref(g), C.byref(m), arr, 1, C.byref(s), 0, None, 0) == 0


def test_autotune_cache_file_round_trip(tmp_path):
    L = hr.load()
    path = str(tmp_path / "tune.json").encode()
    b, v = C.c_int32(0), C.c_int32(0)
    assert L.hr_autotune_cache_lookup(path, b"fwd|x", C.byref(b), C.byref(v)) == 0  # no file
    assert L.hr_autotune_cache_store(path, b"fwd|gfx950|a", 256, 0) == hr.HR_OK
    assert L.hr_autotune_cache_store(path, b"bwd|gfx950|a", 128, 8) == hr.HR_OK
    assert L.hr_autotune_cache_store(path, b"fwd|gfx950|b", 64, 4) == hr.HR_OK
    assert L.hr_autotune_cache_store(path, b"fwd|gfx950|a", 128, 1) == hr.HR_OK  # replaced
    assert L.hr_autotune_cache_lookup(path, b"fwd|gfx950|a", C.byref(b), C.byref(v)) == 1
    assert (b.value, v.value) == (128, 1)
    assert L.hr_autotune_cache_lookup(path, b"bwd|gfx950|a", C.byref(b), C.byref(v)) == 1
    assert (b.value, v.value) == (128, 8)
    assert L.hr_autotune_cache_lookup(path, b"fwd|gfx950|c", C.byref(b), C.byref(v)) == 0
    # the file is JSON
    import json
    d = json.load(open(path))
    assert d["hr_autotune_cache"] == 1 and d["entries"]["fwd|gfx950|b"] == [64, 4]
    assert len(d["entries"]) == 3
    assert L.hr_autotune_cache_store(path, b"other|x", 1, 1) == hr.HR_ERR_INVALID_ARGUMENT
    assert L.hr_autotune_cache_store(path, b'fwd|"x', 1, 1) == hr.HR_ERR_INVALID_ARGUMENT
    assert L.hr_autotune_cache_store(None, b"fwd|x", 1, 1) == hr.HR_ERR_INVALID_ARGUMENT
    bad = str(tmp_path / "no_such_dir" / "t.json").encode()
    assert L.hr_autotune_cache_store(bad, b"fwd|x", 1, 1) == hr.HR_ERR_INTERNAL
