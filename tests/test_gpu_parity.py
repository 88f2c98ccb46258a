"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: integers (tile keys, ranges, triangle ids, per-pixel counts) bit-exact;
images and T within 1e-4 absolute; gradients within 1e-3 relative. A pixel
where the oracle finds a floating-point decision (alpha vs 1/255, T vs 1e-4)
closer than the FP32 kernel can resolve must equal one of the oracle's
outcomes of that decision taken either way; pixels next to a projection or
mesh-depth rounding boundary are left out of the blend checks and counted.
"""
import numpy as np
import pytest

import oracle
from helpers import check_pixels, grad_compare, say
from paper_2506_06988_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gpu_render(hr, scene, cams=None, export_keys=False, settings=None, key_capacity=None):
    cams = cams if cams is not None else scene.cameras
    g, m = hr.to_device(scene.gaussians, scene.mesh)
    r = hr.Renderer(g, m, cams, settings, key_capacity=key_capacity)
    f = r.render_hybrid(export_keys=export_keys)
    torch.cuda.synchronize()
    return r, f


def check_view(f, cams, c, orc, amb_frac_max=None, img_tol=1e-4):
    """Every pixel of camera c against the oracle (see helpers.check_pixels):
    FP64-path pixels exactly, pixels with an ambiguous alpha-skip or T-stop
    decision against the oracle's outcomes of those decisions taken either
    way; only pixels near a projection or mesh rounding boundary are left out
    of the blend checks, and those must stay rare."""
    view = [x.cpu().numpy() for x in f.view(c, cams)]
    hard, soft = check_pixels(view, orc, img_tol)
    n = orc["amb"].size
    say(f"view {c}: {cams[c].width}x{cams[c].height} ambiguous px: {soft} checked by paths, "
        f"{hard} left out ({hard / n:.2e})")
    if amb_frac_max is None:
        amb_frac_max = 1e-3
    assert hard <= amb_frac_max * n


def test_config1_forward_matches_oracle(hr):
    say("case: config1 forward")
    sc = scenes.config1()
    r, f = gpu_render(hr, sc)
    orc = oracle.render(sc.gaussians, sc.mesh, sc.cameras[0], alts=True)
    check_view(f, sc.cameras, 0, orc)
    st = f.stats_dict()
    say("stats", st)
    assert st["overflow"] == 0


def test_config1_keys_values_ranges_bit_exact(hr):
    say("case: config1 keys")
    sc = scenes.config1()
    r, f = gpu_render(hr, sc, export_keys=True)
    k, v, rg = oracle.keys(sc.gaussians, sc.cameras[0])
    st = f.stats_dict()
    assert st["n_keys"] == len(k)
    K = len(k)
    np.testing.assert_array_equal(f.keys[:K].cpu().numpy().view(np.uint64), k)
    np.testing.assert_array_equal(f.values[:K].cpu().numpy().view(np.uint32), v)
    np.testing.assert_array_equal(f.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), rg)
    pr = oracle.project(sc.gaussians, sc.cameras[0])
    np.testing.assert_array_equal(f.radii.cpu().numpy(), pr["radius"])


@pytest.mark.parametrize("seed,variant", [(7, 0), (8, 0), (7, 4)])
def test_small_room_three_uneven_cameras_in_one_call(hr, seed, variant):
    say(f"case: small room seed {seed} variant {variant}")
    sc = scenes.small_room(seed, n=4000, faces=3000, tex=64, n_cams=1)
    rng = np.random.default_rng(seed + 50)
    cams = [scenes.random_room_camera(rng, w, h) for (w, h) in ((96, 80), (50, 37), (130, 70))]
    r, f = gpu_render(hr, sc, cams=cams, export_keys=True,
                      settings=hr.default_settings(variant=variant))
    st = f.stats_dict()
    say("stats", st)
    key_base = 0
    tile_base = 0
    ranges = f.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = f.keys.cpu().numpy().view(np.uint64)
    vals = f.values.cpu().numpy().view(np.uint32)
    for c, cam in enumerate(cams):
        orc = oracle.render(sc.gaussians, sc.mesh, cam, alts=True)
        check_view(f, cams, c, orc)
        k, v, rg = oracle.keys(sc.gaussians, cam)
        ntl = rg.shape[0]
        # global tile ids are offset by the tiles of the cameras before
        np.testing.assert_array_equal(ranges[tile_base:tile_base + ntl] - key_base, rg)
        K = len(k)
        kk = keys[key_base:key_base + K]
        np.testing.assert_array_equal(kk - (np.uint64(tile_base) << np.uint64(32)), k)
        np.testing.assert_array_equal(vals[key_base:key_base + K], v)
        key_base += K
        tile_base += ntl
    assert st["n_keys"] == key_base


def test_many_cameras_grid_barrier_sort_keys_bit_exact(hr):
    # 700 cameras x 3000 Gaussians = 2.1M possible items, beyond the 2M where
    # the depth sort switches to the one-dispatch grid-barrier passes; with
    # more than 256 cameras the sort key has two camera bytes (6 passes)
    say("case: 700 cameras, grid-barrier depth sort")
    sc = scenes.small_room(41, n=3000, faces=300, tex=16, n_cams=1)
    rng = np.random.default_rng(4100)
    cams = [scenes.random_room_camera(rng, 32, 24) for _ in range(700)]
    r, f = gpu_render(hr, sc, cams=cams, export_keys=True)
    st = f.stats_dict()
    say("stats", st)
    assert st["wait_limit"] == 0
    ranges = f.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = f.keys.cpu().numpy().view(np.uint64)
    vals = f.values.cpu().numpy().view(np.uint32)
    key_base = tile_base = 0
    for c, cam in enumerate(cams):
        k, v, rg = oracle.keys(sc.gaussians, cam)
        ntl = rg.shape[0]
        np.testing.assert_array_equal(ranges[tile_base:tile_base + ntl] - key_base, rg)
        K = len(k)
        np.testing.assert_array_equal(keys[key_base:key_base + K] - (np.uint64(tile_base) << np.uint64(32)), k)
        np.testing.assert_array_equal(vals[key_base:key_base + K], v)
        key_base += K
        tile_base += ntl
    assert st["n_keys"] == key_base and st["n_visible"] > 0
    for c in (0, 349, 699):
        check_view(f, cams, c, oracle.render(sc.gaussians, sc.mesh, cams[c], alts=True))


def test_mesh_reused_and_blend_only_equal_the_full_forward(hr):
    # the full forward shades the mesh pixels in its blend; a forward with the
    # mesh reused and hr_blend_forward read the colour that shading left in the
    # workspace, give the same image, T and counts, and leave the mesh outputs
    say("case: mesh reused / blend only")
    sc = scenes.small_room(17, n=5000, faces=2000, tex=32, width=120, height=90)
    rng = np.random.default_rng(1700)
    cams = [sc.cameras[0], scenes.random_room_camera(rng, 70, 50)]
    r, f = gpu_render(hr, sc, cams=cams)
    ref = [x.clone() for x in (f.image, f.final_T, f.n_contrib, f.n_blended, f.n_processed)]
    mesh = [x.clone() for x in (f.mesh_rgb, f.mesh_depth, f.tri_id)]
    for c in range(len(cams)):
        check_view(f, cams, c, oracle.render(sc.gaussians, sc.mesh, cams[c], alts=True))
    for x in (f.image, f.final_T, f.mesh_rgb, f.mesh_depth):
        x.fill_(-7.0)
    f.tri_id.fill_(-7)
    r.render_hybrid_timed(f, mesh_reused=True)
    torch.cuda.synchronize()
    for x, y in zip(ref, (f.image, f.final_T, f.n_contrib, f.n_blended, f.n_processed)):
        assert torch.equal(x, y)
    assert bool((f.mesh_rgb == -7.0).all()) and bool((f.tri_id == -7).all())
    f.image.fill_(-7.0)
    r.blend_forward(f)
    torch.cuda.synchronize()
    assert torch.equal(ref[0], f.image)
    # a full forward again rewrites the mesh outputs as the first one did
    r.render_hybrid(f)
    torch.cuda.synchronize()
    for x, y in zip(mesh, (f.mesh_rgb, f.mesh_depth, f.tri_id)):
        assert torch.equal(x, y)


def test_many_rank_windows_and_pair_slices(hr):
    # > 8192 visible Gaussians per camera: tile lists span several rank
    # windows, and chunks hold more pairs than one binning slice
    say("case: windows and slices")
    sc = scenes.small_room(31, n=40000, faces=4000, tex=64, width=320, height=240)
    r, f = gpu_render(hr, sc, export_keys=True)
    st = f.stats_dict()
    say("stats", st)
    assert st["n_visible"] > 8192 and st["n_keys"] > 4 * 8192
    check_view(f, sc.cameras, 0, oracle.render(sc.gaussians, sc.mesh, sc.cameras[0], alts=True))
    k, v, rg = oracle.keys(sc.gaussians, sc.cameras[0])
    K = len(k)
    np.testing.assert_array_equal(f.keys[:K].cpu().numpy().view(np.uint64), k)
    np.testing.assert_array_equal(f.values[:K].cpu().numpy().view(np.uint32), v)
    # the one-wave kernels over the same windows: identical forward, and a
    # backward equal up to the order of its float atomics
    gi = torch.randn(3 * r.P, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    g0 = r.render_hybrid_backward(gi)
    outs0 = [x.clone() for x in (f.image, f.final_T, f.n_contrib, f.n_blended, f.n_processed)]
    r.settings.variant, r.settings.batch = 12, 128
    f4 = r.render_hybrid()
    g4 = r.render_hybrid_backward(gi)
    bb, bv = r.autotune_backward(gi, repeats=2)
    say(f"  backward autotune -> batch {bb} variant {bv}")
    assert bv & 4 and bb in (64, 128)  # the forward bit is kept
    torch.cuda.synchronize()
    for x, y in zip(outs0, (f4.image, f4.final_T, f4.n_contrib, f4.n_blended, f4.n_processed)):
        assert torch.equal(x, y)
    for k_ in g0:
        a_, b_ = g0[k_].double(), g4[k_].double()
        assert float((a_ - b_).norm()) <= 1e-4 * float(a_.norm()) + 1e-12, k_


def test_ragged_sizes_and_edge_cases(hr):
    say("case: ragged / empty")
    sc = scenes.small_room(3, n=500, faces=300, tex=16)
    for (w, h) in ((1, 1), (17, 15), (33, 1)):
        cam = scenes.random_room_camera(np.random.default_rng(w * 100 + h), w, h)
        r, f = gpu_render(hr, sc, cams=[cam])
        check_view(f, [cam], 0, oracle.render(sc.gaussians, sc.mesh, cam, alts=True), amb_frac_max=1.0)
    # no Gaussians: the image is the mesh
    g0 = sc.gaussians.subset(np.zeros(sc.gaussians.n, bool))
    sc0 = scenes.Scene("empty", g0, sc.mesh, sc.cameras)
    r, f = gpu_render(hr, sc0)
    im, T, mr = [x.cpu().numpy() for x in f.view(0, sc.cameras)[:3]]
    np.testing.assert_array_equal(im, mr)
    assert np.all(T == 1.0)
    # no mesh: Gaussians over the background
    sc1 = scenes.Scene("nomesh", sc.gaussians, None, sc.cameras)
    r, f = gpu_render(hr, sc1, settings=hr.default_settings(bg=(0.2, 0.4, 0.6)))
    orc = oracle.render(sc.gaussians, None, sc.cameras[0], params=oracle.default_params(bg=(0.2, 0.4, 0.6)),
                        alts=True)
    check_view(f, sc.cameras, 0, orc)


def test_forward_is_deterministic_and_variants_bit_identical(hr):
    say("case: determinism")
    sc = scenes.small_room(11, n=6000, faces=2000, tex=32, width=160, height=120)
    r, f = gpu_render(hr, sc)
    a = f.image.clone()
    f2 = r.render_hybrid()
    torch.cuda.synchronize()
    assert torch.equal(a, f2.image)
    ref = [x.clone() for x in (f2.final_T, f2.n_contrib, f2.n_blended, f2.n_processed, f2.stats)]
    for batch in (32, 64, 128, 256):
        for variant in (0, 1, 2, 3, 4):
            r.settings.batch, r.settings.variant = batch, variant
            f3 = r.render_hybrid()
            torch.cuda.synchronize()
            assert torch.equal(a, f3.image), (batch, variant)
            got = (f3.final_T, f3.n_contrib, f3.n_blended, f3.n_processed, f3.stats)
            for x, y in zip(ref, got):
                assert torch.equal(x, y), (batch, variant)
    b, v = r.autotune(f3, repeats=2)
    say("autotune ->", b, v)


def test_loss_kernel_matches_oracle_loss(hr):
    say("case: loss")
    rng = np.random.default_rng(3)
    H, W = 37, 53
    img, tgt, Im = (rng.uniform(0, 1, (3, H, W)).astype(np.float32) for _ in range(3))
    T = rng.uniform(0, 1, (H, W)).astype(np.float32)
    tri = np.where(rng.uniform(size=(H, W)) < 0.6, 5, -1).astype(np.int32)
    Lr, gi, gt, gm = oracle.loss(img, T, Im, tri, tgt)
    d = lambda a: torch.as_tensor(a.reshape(-1)).cuda()
    L, gI, gT, gM = hr.hybrid_loss(d(img), d(T), d(Im), d(tri), d(tgt))
    torch.cuda.synchronize()
    np.testing.assert_allclose(L.item(), Lr, rtol=1e-5)
    np.testing.assert_allclose(gI.cpu().numpy().reshape(3, H, W), gi, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(gT.cpu().numpy().reshape(H, W), gt, rtol=1e-4, atol=1e-10)
    np.testing.assert_allclose(gM.cpu().numpy().reshape(3, H, W), gm, rtol=1e-4, atol=1e-10)


_grad_compare = grad_compare


def tiny(seed, n=30, deg=3, w=48, h=40):
    rng = np.random.default_rng(seed)
    means = np.column_stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.5, 0.5, n), rng.uniform(1.5, 3.0, n)])
    sh = np.concatenate([((rng.uniform(0, 1, (n, 1, 3)) - 0.5) / scenes.Y00),
                         rng.normal(0, 0.2, (n, (deg + 1) ** 2 - 1, 3))], 1)
    g = scenes.make_gaussians(means, rng.uniform(-3.0, -1.8, (n, 3)), rng.standard_normal((n, 4)),
                              rng.normal(0, 1, n), sh, deg)
    mesh = scenes.quad_mesh(rng, z=2.4, half=1.0, tex_size=16)
    cam = scenes.Camera(w, h, 40.0, 40.0, w / 2 + 0.3, h / 2 - 0.2, np.eye(3), np.zeros(3))
    return scenes.Scene(f"tiny{seed}", g, mesh, [cam])


@pytest.mark.parametrize("seed,variant", [(101, 0), (102, 0), (103, 0), (101, 12), (104, 8)])
def test_backward_matches_oracle_gradient(hr, seed, variant):
    say(f"case: backward seed {seed} variant {variant}")
    sc = tiny(seed)
    cam = sc.cameras[0]
    r, f = gpu_render(hr, sc, settings=hr.default_settings(variant=variant))
    orc = oracle.render(sc.gaussians, sc.mesh, cam, alts=True)
    amb = orc["amb"] != 0
    rng = np.random.default_rng(seed)
    H, W = cam.height, cam.width
    gi = rng.normal(size=(3, H, W)).astype(np.float32)
    gt = rng.normal(size=(H, W)).astype(np.float32)
    gm = rng.normal(size=(3, H, W)).astype(np.float32)
    gi[:, amb] = 0
    gt[amb] = 0
    gm[:, amb] = 0
    d = lambda a: torch.as_tensor(a.reshape(-1)).cuda()
    grads = r.render_hybrid_backward(d(gi), d(gt), d(gm))
    torch.cuda.synchronize()
    ref = oracle.backward(sc.gaussians, sc.mesh, cam, gi, gt, gm)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex"):
        _grad_compare(k, grads[k].cpu().numpy(), ref[k])


def test_multicamera_backward_sums_over_cameras(hr):
    say("case: backward over 2 cameras")
    sc = tiny(111, n=40)
    cams = [sc.cameras[0], scenes.Camera(40, 36, 38.0, 38.0, 20.0, 18.0,
                                         scenes.look_camera(40, 36, [0.2, 0.1, -0.1], 0.1, 0.05).R,
                                         scenes.look_camera(40, 36, [0.2, 0.1, -0.1], 0.1, 0.05).t)]
    r, f = gpu_render(hr, sc, cams=cams)
    rng = np.random.default_rng(5)
    ups, refs = [], []
    for c, cam in enumerate(cams):
        orc = oracle.render(sc.gaussians, sc.mesh, cam, alts=True)
        amb = orc["amb"] != 0
        gi = rng.normal(size=(3, cam.height, cam.width)).astype(np.float32)
        gi[:, amb] = 0
        ups.append(gi)
        refs.append(oracle.backward(sc.gaussians, sc.mesh, cam, gi, None, None))
    g_img = torch.as_tensor(np.concatenate([u.reshape(-1) for u in ups])).cuda()
    grads = r.render_hybrid_backward(g_img)
    torch.cuda.synchronize()
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex"):
        _grad_compare(k, grads[k].cpu().numpy(), refs[0][k] + refs[1][k])


def test_graph_step_matches_eager(hr):
    say("case: hipGraph step")
    sc = scenes.small_room(21, n=3000, faces=1000, tex=32, width=64, height=48, n_cams=1)
    rng = np.random.default_rng(9)
    cams = [scenes.random_room_camera(rng, w, h) for (w, h) in ((64, 48), (40, 30))]
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, cams)
    f = r.render_hybrid()
    target = torch.rand(3 * r.P, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    L, gi, gt, gm = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target, r.sizes)
    ref = r.render_hybrid_backward(gi, gt, gm)
    torch.cuda.synchronize()
    step = hr.BatchedStep(r, target)
    for rep in range(3):
        step.launch()
        step.stream.synchronize()
        # eager work between replays
        _ = (f.image * 2).sum().item()
        assert torch.equal(step.frame.image, f.image), rep
        np.testing.assert_allclose(step.loss.item(), L.item(), rtol=1e-6)
        for k in ref:
            np.testing.assert_allclose(step.grads[k].cpu().numpy(), ref[k].cpu().numpy(),
                                       rtol=1e-4, atol=1e-7 * float(ref[k].abs().max()) + 1e-12)
    step.close()


@pytest.mark.parametrize("mode", ["none", "one", "T", "sigmoid"])
def test_full_loss_kernel_matches_oracle(hr, mode):
    say(f"case: full loss {mode}")
    rng = np.random.default_rng(17)
    sizes = [(37, 29), (64, 48), (5, 70)]
    ims, tgts, Ts, Ims, tris = [], [], [], [], []
    for (w, h) in sizes:
        ims.append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
        tgts.append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
        Ts.append(rng.uniform(0, 1, (h, w)).astype(np.float32))
        Ims.append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
        tris.append(np.where(rng.uniform(size=(h, w)) < 0.6, 3, -1).astype(np.int32))
    cat = lambda xs: torch.as_tensor(np.concatenate([x.reshape(-1) for x in xs])).cuda()
    L, gI, gT, gM = hr.full_loss(cat(ims), cat(Ts), cat(Ims), cat(tris), cat(tgts), sizes,
                                 mask_mode=mode)
    torch.cuda.synchronize()
    Lr, gi, gt, gm = oracle.full_loss(ims, Ts, Ims, tris, tgts, mask_mode=mode)
    np.testing.assert_allclose(L.item(), Lr, rtol=2e-5)
    for got, ref in ((gI, gi), (gT, gt), (gM, gm)):
        ref = np.concatenate([r.reshape(-1) for r in ref])
        got = got.cpu().numpy()
        scale = max(np.abs(ref).max(), 1e-12)
        np.testing.assert_allclose(got, ref, atol=2e-4 * scale, rtol=1e-3)


def test_mesh_depth_culling_matches_oracle(hr):
    say("case: mesh-depth culling, room with Gaussians outside the walls, 2 cameras")
    rng = np.random.default_rng(61)
    room = scenes.small_room(61, n=3000, faces=2000, tex=32)
    g = scenes.concat_gaussians(room.gaussians, scenes.outside_gaussians(rng, 3000))
    sc = scenes.Scene("room_outside", g, room.mesh, [])
    cams = [scenes.random_room_camera(rng, w, h) for (w, h) in ((96, 80), (70, 45))]
    st = hr.default_settings(flags=hr.HR_FLAG_CULL_BEHIND_MESH)
    r, f = gpu_render(hr, sc, cams=cams, export_keys=True, settings=st)
    stats = f.stats_dict()
    pc = oracle.default_params(flags=oracle.CULL_MESH)
    ranges = f.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = f.keys.cpu().numpy().view(np.uint64)
    vals = f.values.cpu().numpy().view(np.uint32)
    key_base = tile_base = uncut = 0
    for c, cam in enumerate(cams):
        orc = oracle.render(g, sc.mesh, cam, params=pc, alts=True)
        check_view(f, cams, c, orc)
        k, v, rg = oracle.keys(g, cam, params=pc, mesh=sc.mesh)
        uncut += len(oracle.keys(g, cam)[0])
        ntl = rg.shape[0]
        np.testing.assert_array_equal(ranges[tile_base:tile_base + ntl] - key_base, rg)
        K = len(k)
        np.testing.assert_array_equal(keys[key_base:key_base + K] - (np.uint64(tile_base) << np.uint64(32)), k)
        np.testing.assert_array_equal(vals[key_base:key_base + K], v)
        key_base += K
        tile_base += ntl
    say(f"  kept pairs {key_base} of {uncut}")
    assert stats["n_keys"] == key_base and key_base < 0.9 * uncut
    # a capacity between the kept and the uncut count is enough
    cap = (key_base + uncut) // 2
    r2, f2 = gpu_render(hr, sc, cams=cams, settings=st, key_capacity=cap)
    assert r2.key_capacity == cap  # no retry with a larger capacity was needed
    assert torch.equal(f2.image, f.image) and f2.stats_dict()["n_keys"] == key_base
    # and the images are those of the uncut lists
    r3, f3 = gpu_render(hr, sc, cams=cams)
    assert torch.equal(f3.image, f.image) and torch.equal(f3.final_T, f.final_T)


def test_mip_filter3d_matches_oracle(hr):
    say("case: Mip-Splatting 3D filter over 20 training views")
    sc = scenes.small_room(71, n=5000, faces=200, tex=8)
    rng = np.random.default_rng(71)
    cams = [scenes.random_room_camera(rng, *wh) for wh in [(96, 80), (40, 30)] * 10]
    # a few Gaussians outside the room, unseen by every view
    g = scenes.concat_gaussians(sc.gaussians, scenes.outside_gaussians(rng, 50, margin=40.0))
    dg, _ = hr.to_device(g, None)
    got = hr.mip_filter3d(dg, cams).cpu().numpy().astype(np.float64)
    ref = oracle.mip_filter3d(g, cams, s=0.2)
    np.testing.assert_allclose(got, ref, rtol=2e-6)
    say(f"  seen by none: {int((ref == ref.max()).sum())}, range {ref.min():.3e}..{ref.max():.3e}")


@pytest.mark.parametrize("seed", [131, 132])
def test_mip_filters_forward_and_backward_match_oracle(hr, seed):
    say(f"case: Mip-Splatting filters, seed {seed}")
    sc = tiny(seed, n=40)
    cam = sc.cameras[0]
    rng = np.random.default_rng(seed)
    s2 = np.exp(2.0 * sc.gaussians.log_scales.astype(np.float64)).mean(1)
    f3 = (rng.uniform(0.2, 1.5, sc.gaussians.n) * s2).astype(np.float32)
    st = hr.default_settings(low_pass=0.1, flags=hr.HR_FLAG_MIP_2D)
    pm = oracle.default_params(low_pass=0.1, flags=oracle.MIP_2D)
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    g.filter3d = torch.as_tensor(f3).cuda()
    r = hr.Renderer(g, m, [cam], st)
    f = r.render_hybrid()
    torch.cuda.synchronize()
    orc = oracle.render(sc.gaussians, sc.mesh, cam, params=pm, filter3d=f3, alts=True)
    check_view(f, [cam], 0, orc)
    # the filters change the image
    plain = oracle.render(sc.gaussians, sc.mesh, cam, alts=True)
    assert np.abs(plain["image"] - orc["image"]).max() > 1e-2
    amb = orc["amb"] != 0
    H, W = cam.height, cam.width
    gi = rng.normal(size=(3, H, W)).astype(np.float32)
    gt = rng.normal(size=(H, W)).astype(np.float32)
    gi[:, amb] = 0
    gt[amb] = 0
    d = lambda a: torch.as_tensor(a.reshape(-1)).cuda()
    grads = r.render_hybrid_backward(d(gi), d(gt))
    torch.cuda.synchronize()
    ref = oracle.backward(sc.gaussians, sc.mesh, cam, gi, gt, None, params=pm, filter3d=f3)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex"):
        _grad_compare(k, grads[k].cpu().numpy(), ref[k])


def test_tile_ellipse_culling_matches_oracle(hr):
    say("case: tile-ellipse culling, small room, 2 cameras, forward and backward")
    sc = scenes.small_room(81, n=6000, faces=2000, tex=32)
    rng = np.random.default_rng(81)
    cams = [scenes.random_room_camera(rng, w, h) for (w, h) in ((96, 80), (70, 45))]
    st = hr.default_settings(flags=hr.HR_FLAG_TILE_ELLIPSE)
    pe = oracle.default_params(flags=oracle.TILE_ELLIPSE)
    r, f = gpu_render(hr, sc, cams=cams, export_keys=True, settings=st)
    ranges = f.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = f.keys.cpu().numpy().view(np.uint64)
    vals = f.values.cpu().numpy().view(np.uint32)
    key_base = tile_base = uncut = 0
    for c, cam in enumerate(cams):
        check_view(f, cams, c, oracle.render(sc.gaussians, sc.mesh, cam, params=pe, alts=True))
        k, v, rg = oracle.keys(sc.gaussians, cam, params=pe)
        uncut += len(oracle.keys(sc.gaussians, cam)[0])
        ntl = rg.shape[0]
        np.testing.assert_array_equal(ranges[tile_base:tile_base + ntl] - key_base, rg)
        np.testing.assert_array_equal(keys[key_base:key_base + len(k)] - (np.uint64(tile_base) << np.uint64(32)), k)
        np.testing.assert_array_equal(vals[key_base:key_base + len(k)], v)
        key_base += len(k)
        tile_base += ntl
    say(f"  kept pairs {key_base} of {uncut}")
    assert f.stats_dict()["n_keys"] == key_base and key_base < 0.8 * uncut
    # the same image and T as without culling, and the same gradients
    r0, f0 = gpu_render(hr, sc, cams=cams)
    assert torch.equal(f0.image, f.image) and torch.equal(f0.final_T, f.final_T)
    assert torch.equal(f0.n_blended, f.n_blended)
    gi = torch.randn(3 * r.P, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    ga, gb = r.render_hybrid_backward(gi), r0.render_hybrid_backward(gi)
    torch.cuda.synchronize()
    for k_ in ga:
        x, y = ga[k_].double(), gb[k_].double()
        assert float((x - y).norm()) <= 1e-5 * float(y.norm()) + 1e-12, k_
