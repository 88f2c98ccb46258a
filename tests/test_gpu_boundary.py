"""The boundary above the kernels, on the GPU, against the CPU FP64 oracle:
the loss over several packed images, the hipGraph training step (its loss
and gradients summed over uneven cameras, its capacity overflow handling),
and the torch.autograd.Functions (per-call saved context, loss.backward()).

Scenes are chosen (seeds) so that the oracle tags no ambiguous pixel: the
graph step computes its upstream gradients on the device, so ambiguous
pixels could not be left out of the comparison.
"""
import numpy as np
import pytest

import oracle
from helpers import grad_compare, packed_loss_oracle, say
from paper_2506_06988_amd import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRADS = ("means", "log_scales", "quats", "opacity_logits", "sh", "tex")


def two_camera_room(seed=23, cam_seed=11):
    sc = scenes.small_room(seed, n=3000, faces=1000, tex=32, width=64, height=48, n_cams=1)
    rng = np.random.default_rng(cam_seed)
    cams = [scenes.random_room_camera(rng, w, h) for (w, h) in ((64, 48), (40, 30))]
    trng = np.random.default_rng(seed + 77)
    targets = [trng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    return sc, cams, targets


def test_loss_over_two_uneven_images_matches_oracle_per_image(hr):
    say("case: loss over 2 packed images (37x29, 64x48)")
    rng = np.random.default_rng(3)
    sizes = [(37, 29), (64, 48)]
    ims, Ts, Ims, tris, tgts = [], [], [], [], []
    for (w, h) in sizes:
        ims.append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
        Ts.append(rng.uniform(0, 1, (h, w)).astype(np.float32))
        Ims.append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
        tris.append(np.where(rng.uniform(size=(h, w)) < 0.6, 5, -1).astype(np.int32))
        tgts.append(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
    cat = lambda xs: torch.as_tensor(np.concatenate([x.reshape(-1) for x in xs])).cuda()
    L, gI, gT, gM = hr.hybrid_loss(cat(ims), cat(Ts), cat(Ims), cat(tris), cat(tgts), sizes)
    torch.cuda.synchronize()
    renders = [dict(image=a, final_T=b, mesh_rgb=c, tri_id=d) for a, b, c, d in zip(ims, Ts, Ims, tris)]
    Lr, ups = packed_loss_oracle(oracle, renders, tgts)
    np.testing.assert_allclose(L.item(), Lr, rtol=1e-5)
    for j, got in enumerate((gI, gT, gM)):
        ref = np.concatenate([u[j].reshape(-1) for u in ups])
        np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-4, atol=1e-10)
    # the pairing is per image: the same buffers read as one planar image differ
    L1, gI1, _, _ = hr.hybrid_loss(cat(ims), cat(Ts), cat(Ims), cat(tris), cat(tgts))
    torch.cuda.synchronize()
    assert not torch.equal(gI1, gI) or abs(L1.item() - L.item()) > 1e-6


@pytest.mark.parametrize("variant,batch_bwd", [(0, 0), (8, 128), (8, 32)])
def test_graph_step_matches_oracle_per_camera(hr, variant, batch_bwd):
    say(f"case: hipGraph step on 2 uneven cameras vs oracle, variant {variant} batch_bwd {batch_bwd}")
    sc, cams, targets = two_camera_room()
    renders = [oracle.render(sc.gaussians, sc.mesh, c) for c in cams]
    for c, o in zip(cams, renders):
        assert int((o["amb"] != 0).sum()) == 0, "scene has ambiguous pixels"
    Lr, ups = packed_loss_oracle(oracle, renders, targets)
    ref = None
    for c, o, (gi, gt, gm) in zip(cams, renders, ups):
        b = oracle.backward(sc.gaussians, sc.mesh, c, gi, gt, gm)
        ref = b if ref is None else {k: ref[k] + b[k] for k in GRADS}
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    st = hr.default_settings(variant=variant, batch_bwd=batch_bwd)
    r = hr.Renderer(g, m, cams, st)
    target = torch.as_tensor(np.concatenate([t.reshape(-1) for t in targets])).cuda()
    step = hr.BatchedStep(r, target)
    for rep in range(3):
        stats = step.step()
        # eager work on the default stream between replays
        _ = (step.frame.image * 2).sum().item()
        assert stats["overflow"] == 0 and stats["wait_limit"] == 0
        for c, o in enumerate(renders):
            im, T = [x.cpu().numpy() for x in step.frame.view(c, cams)[:2]]
            assert np.abs(im - o["image"]).max() <= 1e-4 and np.abs(T - o["final_T"]).max() <= 1e-4
        np.testing.assert_allclose(step.loss.item(), Lr, rtol=1e-5)
        for k in GRADS:
            grad_compare(f"{k} (replay {rep})", step.grads[k].cpu().numpy(), ref[k])
    step.close()


def test_timed_backward_matches_the_backward_and_the_oracle(hr):
    say("case: hr_render_hybrid_backward_timed (serial and beside) on 2 cameras vs oracle")
    sc, cams, targets = two_camera_room()
    renders = [oracle.render(sc.gaussians, sc.mesh, c) for c in cams]
    Lr, ups = packed_loss_oracle(oracle, renders, targets)
    ref = None
    for c, o, (gi, gt, gm) in zip(cams, renders, ups):
        b = oracle.backward(sc.gaussians, sc.mesh, c, gi, gt, gm)
        ref = b if ref is None else {k: ref[k] + b[k] for k in GRADS}
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, cams)
    f = r.render_hybrid(sync_check=True)
    target = torch.as_tensor(np.concatenate([t.reshape(-1) for t in targets])).cuda()
    _, gi, gt, gm = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target, r.sizes)
    plain = r.render_hybrid_backward(gi, gt, gm)
    for serial in (True, False):
        t, grads = r.render_hybrid_backward_timed(gi, gt, gm, serial=serial)
        torch.cuda.synchronize()
        say(f"  serial={serial}: " + ", ".join(f"{k} {v:.3f} ms" for k, v in t.items()))
        assert all(v > 0 for v in t.values())
        assert t["backward"] >= t["blend_backward"] and t["backward"] >= t["projection_backward"]
        for k in GRADS:
            a, b = grads[k].cpu().numpy(), plain[k].cpu().numpy()
            # the same kernels; only the order of float atomics may differ
            assert np.abs(a - b).max() <= 1e-5 * max(np.abs(b).max(), 1e-30), k
            grad_compare(f"{k} (timed, serial={serial})", a, ref[k])


def test_graph_step_overflow_is_reported_and_recaptured(hr):
    say("case: hipGraph step captured with a key capacity far too small")
    sc, cams, targets = two_camera_room()
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, cams, key_capacity=500)
    target = torch.as_tensor(np.concatenate([t.reshape(-1) for t in targets])).cuda()
    step = hr.BatchedStep(r, target)
    step.launch()
    with pytest.raises(hr.HRError) as e:
        step.check()
    assert e.value.status == hr.HR_ERR_CAPACITY
    need = step.last_stats["n_keys"]
    say(f"  overflow reported: {need} pairs for a capacity of 500")
    assert step.last_stats["overflow"] == 1 and need > 500
    stats = step.step()
    assert step.recaptures == 1 and r.key_capacity >= need and stats["overflow"] == 0
    # the re-captured step renders the oracle's images
    for c, cam in enumerate(cams):
        o = oracle.render(sc.gaussians, sc.mesh, cam)
        im = step.frame.view(c, cams)[0].cpu().numpy()
        assert np.abs(im - o["image"]).max() <= 1e-4
    # an eager render with the same small capacity and no host sync sets the
    # flag on the device; with the sync it returns HR_ERR_CAPACITY
    r2 = hr.Renderer(g, m, cams, key_capacity=500)
    f2 = r2.new_frame()
    rc = r2._forward(f2, g, None, r2.ws, r2.key_capacity, sync_check=False)
    torch.cuda.synchronize()
    assert rc == hr.HR_OK and f2.stats_dict()["overflow"] == 1
    assert f2.stats_dict()["wait_limit"] == 0
    rc = r2._forward(f2, g, None, r2.ws, r2.key_capacity, sync_check=True)
    assert rc == hr.HR_ERR_CAPACITY and f2.stats_dict()["n_keys"] == need
    step.close()


def _torch_params(g, tex=None):
    ps = [x.clone().requires_grad_(True) for x in (g.means, g.log_scales, g.quats,
                                                   g.opacity_logits, g.sh)]
    return ps + [None if tex is None else tex.clone().requires_grad_(True)]


def test_autograd_loss_backward_matches_oracle(hr):
    say("case: HybridRenderFn + HybridLossFn, loss.backward() on 2 cameras vs oracle")
    sc, cams, targets = two_camera_room()
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, cams)
    ps = _torch_params(g, m.tex)
    target = torch.as_tensor(np.concatenate([t.reshape(-1) for t in targets])).cuda()
    image, T, Im, tri = hr.HybridRenderFn().apply(r, *ps)
    assert not tri.requires_grad and image.requires_grad
    loss = hr.HybridLossFn().apply(image, T, Im, tri, target, r.sizes)
    loss.backward()
    torch.cuda.synchronize()
    renders = [oracle.render(sc.gaussians, sc.mesh, c) for c in cams]
    Lr, ups = packed_loss_oracle(oracle, renders, targets)
    np.testing.assert_allclose(loss.item(), Lr, rtol=1e-5)
    ref = None
    for c, (gi, gt, gm) in zip(cams, ups):
        b = oracle.backward(sc.gaussians, sc.mesh, c, gi, gt, gm)
        ref = b if ref is None else {k: ref[k] + b[k] for k in GRADS}
    for k, p in zip(GRADS, ps):
        grad_compare(k, p.grad.cpu().numpy(), ref[k])


def test_autograd_two_forwards_then_one_summed_backward(hr):
    say("case: two forwards through one renderer, then one backward of their sum")
    sc, cams, targets = two_camera_room(seed=23, cam_seed=14)
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, cams)
    rng = np.random.default_rng(4)
    # the second parameter set: every mean shifted by a few millimetres
    shift = torch.as_tensor(rng.normal(0, 3e-3, (g.n, 3)).astype(np.float32)).cuda()
    pa = _torch_params(g, m.tex)
    pb = _torch_params(g, m.tex)
    with torch.no_grad():
        pb[0] += shift
    up_a = torch.randn(3 * r.P, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    up_b = torch.randn(3 * r.P, device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    ia, _, _, _ = hr.HybridRenderFn().apply(r, *pa)
    ib, _, _, _ = hr.HybridRenderFn().apply(r, *pb)
    assert r.g is g  # the renderer's own Gaussians are untouched
    ((ia * up_a).sum() + (ib * up_b).sum()).backward()
    torch.cuda.synchronize()
    # each against its own eager forward + backward
    for ps, up in ((pa, up_a), (pb, up_b)):
        gd = hr.DevGaussians(*[x.detach().contiguous() for x in ps[:5]], g.sh_degree)
        re = hr.Renderer(gd, m, cams)
        re.render_hybrid()
        ref = re.render_hybrid_backward(up)
        torch.cuda.synchronize()
        for k, p in zip(GRADS, ps):
            a, b = p.grad.double(), ref[k].double()
            assert float((a - b).norm()) <= 1e-5 * float(b.norm()) + 1e-12, k
    # and the first against the oracle (upstream zeroed at ambiguous pixels)
    ups, ref = [], None
    o0 = 0
    for c in cams:
        hw = c.width * c.height
        o = oracle.render(sc.gaussians, sc.mesh, c)
        assert int((o["amb"] != 0).sum()) == 0
        gi = up_a[3 * o0:3 * (o0 + hw)].cpu().numpy().reshape(3, c.height, c.width)
        b = oracle.backward(sc.gaussians, sc.mesh, c, gi, None, None)
        ref = b if ref is None else {k: ref[k] + b[k] for k in GRADS}
        o0 += hw
    for k, p in zip(GRADS, pa):
        grad_compare(k, p.grad.cpu().numpy(), ref[k])


def test_autotune_cache_is_written_and_reused(hr, tmp_path, monkeypatch):
    say("case: autotuner cache (HR_AUTOTUNE_CACHE)")
    import json
    path = tmp_path / "tune.json"
    monkeypatch.setenv("HR_AUTOTUNE_CACHE", str(path))
    sc, cams, targets = two_camera_room()
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, cams)
    f = r.render_hybrid()
    b, v = r.autotune(f, repeats=1)
    gi = torch.randn(3 * r.P, device="cuda", generator=torch.Generator("cuda").manual_seed(8))
    bb, bv = r.autotune_backward(gi, repeats=1)
    d = json.load(open(path))["entries"]
    fk = [k for k in d if k.startswith("fwd|")]
    bk = [k for k in d if k.startswith("bwd|")]
    assert len(fk) == 1 and len(bk) == 1 and "|cams2^1|" in fk[0]
    assert d[fk[0]] == [b, v & 7] and d[bk[0]] == [bb, bv & 8]
    # a hand-edited entry is used as it is, without timing
    d[fk[0]] = [32, 1]
    d[bk[0]] = [64, 8]
    with open(path, "w") as fh:  # the library's layout: one entry per line
        fh.write('{\n  "hr_autotune_cache": 1,\n  "entries": {\n' +
                 ",\n".join(f'    "{k}": [{a}, {c}]' for k, (a, c) in d.items()) + "\n  }\n}\n")
    assert json.load(open(path))["entries"] == d
    ref = [x.clone() for x in (f.image, f.final_T, f.n_contrib, f.n_blended, f.n_processed)]
    r.settings.batch, r.settings.variant, r.settings.batch_bwd = 0, 0, 0
    assert r.autotune(f, repeats=1) == (32, 1)
    torch.cuda.synchronize()
    for x, y in zip(ref, (f.image, f.final_T, f.n_contrib, f.n_blended, f.n_processed)):
        assert torch.equal(x, y)
    assert r.autotune_backward(gi, repeats=1) == (64, 9)
