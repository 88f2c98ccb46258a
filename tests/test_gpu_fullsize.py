"""Parity at the benchmark's full sizes, on sampled windows the oracle can afford.

The GPU renders whole frames exactly as bench.py does; the oracle renders the
same frame restricted to sampled 32x32 windows (its per-pixel result does not
depend on the window). Gradients use a loss restricted to a 32x32 crop, so the
oracle only needs the crop.
"""

import numpy as np
import pytest

import oracle
from helpers import check_pixels, grad_compare, say
from paper_2506_06988_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


def windows(cam, n, rng, size=32):
    out = []
    for _ in range(n):
        x0 = int(rng.integers(0, max(1, (cam.width - size) // 16 + 1))) * 16
        y0 = int(rng.integers(0, max(1, (cam.height - size) // 16 + 1))) * 16
        out.append((x0, y0, min(cam.width, x0 + size), min(cam.height, y0 + size)))
    return out


def check_window(view, orc, win):
    """The window of a full-frame GPU view against the oracle's render of that
    window (made with alts=True); returns (pixels left out, pixels)."""
    x0, y0, x1, y1 = win
    sub = [v[..., y0:y1, x0:x1] for v in view]
    check_window.examined += float(orc["n_processed"].sum())
    hard, soft = check_pixels(sub, orc)
    check_window.by_paths += soft
    return hard, orc["amb"].size


check_window.examined = 0.0
check_window.by_paths = 0

# the benchmark's configurations: tile-ellipse binning with the forward blend
# the autotuner picks there (256 per batch, one-deep staging) and, for the
# training step, the one-wave backward with 128 per batch
TILE_ELLIPSE = 1 << 5  # HR_FLAG_TILE_ELLIPSE
ELLIPSE = dict(flags=TILE_ELLIPSE, batch=256, variant=0)
STEP = dict(flags=TILE_ELLIPSE, batch=256, variant=8, batch_bwd=32)


def run_frames(hr, sc, cams, n_win, seed, settings=None, params=None):
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    st = hr.default_settings(**(settings or {}))
    r = hr.Renderer(g, m, cams, st)
    f = r.render_hybrid()
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    tot_amb = tot = 0
    check_window.examined = 0.0
    check_window.by_paths = 0
    for c, cam in enumerate(cams):
        view = [v.cpu().numpy() for v in f.view(c, cams)]
        for win in windows(cam, n_win, rng):
            orc = oracle.render(sc.gaussians, sc.mesh, cam, window=win, params=params, alts=True)
            a, n = check_window(view, orc, win)
            tot_amb += a
            tot += n
    say(f"{sc.name}: {len(cams)} cameras, settings {settings}: {check_window.by_paths} ambiguous "
        f"px checked by paths, {tot_amb}/{tot} left out; stats {f.stats_dict()}")
    assert tot_amb <= 1e-3 * tot
    return r, f


def pe():
    return oracle.default_params(flags=oracle.TILE_ELLIPSE)


def test_720p_poses(hr):
    say("case: 720p, 300k Gaussians, 4 poses: 3-sigma rectangles, and the one-wave forward")
    sc = scenes.config2()
    run_frames(hr, sc, sc.cameras[:2], 2, 1)
    run_frames(hr, sc, sc.cameras[2:4], 2, 5, settings=dict(flags=TILE_ELLIPSE, batch=128, variant=4),
               params=pe())


def test_1080p_hybrid_and_gaussian_only(hr):
    say("case: 1080p hybrid and Gaussian-only, as benchmarked (tile-ellipse binning)")
    sc = scenes.config5("hybrid")
    run_frames(hr, sc, [sc.cameras[1], sc.cameras[2]], 3, 2, settings=ELLIPSE, params=pe())
    sg = scenes.config5("gaussian_only")
    run_frames(hr, sg, [sg.cameras[1]], 3, 3, settings=dict(flags=TILE_ELLIPSE, batch=64, variant=0),
               params=pe())


def test_sixteen_uneven_cameras_forward(hr):
    say("case: 16 uneven cameras, as benchmarked (tile-ellipse binning, batch 256)")
    sc = scenes.config4()
    run_frames(hr, sc, sc.cameras, 1, 4, settings=ELLIPSE, params=pe())


def test_sixteen_camera_graph_step_gradients_vs_oracle(hr):
    """The benchmark's training step (16 uneven cameras, 1M Gaussians, one
    hipGraph: forward, loss, one-wave backward) against the oracle's gradient
    summed over cameras, for Gaussians whose footprint is small enough that
    the oracle can cover all of it: per such Gaussian and camera, the window of
    its tile rectangle, with the step's own upstream gradients there."""
    say("case: 16-camera graph step, per-Gaussian gradients vs oracle")
    sc = scenes.config4()
    cams = sc.cameras
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, cams, hr.default_settings(**STEP))
    target = torch.as_tensor(np.concatenate([t.reshape(-1) for t in sc.target])).cuda()
    step = hr.BatchedStep(r, target)
    stats = step.step()
    say(f"  step stats {stats}")
    fr = step.frame
    frame_np = {k: getattr(fr, k).cpu().numpy() for k in ("image", "final_T", "n_contrib",
                                                           "n_blended", "n_processed")}
    gi_all = step.g_image.cpu().numpy()
    gt_all = step.g_T.cpu().numpy()
    gm_all = step.g_mesh.cpu().numpy()
    got = {k: step.grads[k].cpu().numpy() for k in ("means", "log_scales", "quats",
                                                      "opacity_logits", "sh")}
    step.close()
    # Gaussians with a gradient, visible in at least two cameras, the smallest
    # footprints (tile rectangles summed over the cameras) first
    n = sc.gaussians.n
    area = np.zeros(n, np.int64)
    seen = np.zeros(n, np.int32)
    projs = []
    for cam in cams:
        pr = oracle.project(sc.gaussians, cam)
        projs.append(pr)
        rc = pr["rect"].astype(np.int64)
        vis = pr["radius"] > 0
        area += np.where(vis, (rc[:, 1] - rc[:, 0]) * (rc[:, 3] - rc[:, 2]), 0)
        seen += vis
    # (every pixel of a Gaussian's windows must have taken the oracle's FP64
    # decisions - equal counts and image - since the step's upstream gradients
    # cannot be zeroed where they differ; small footprints make that likely)
    has_grad = (got["opacity_logits"] != 0) & (np.abs(got["means"]).sum(1) > 0)
    elig = np.nonzero((seen >= 1) & has_grad)[0]
    cand = elig[np.argsort(area[elig] * 4 - np.minimum(seen[elig], 3), kind="stable")][:300]
    say(f"  Gaussians with a gradient: {len(elig)} ({int(((seen >= 2) & has_grad).sum())} seen "
        f"twice or more); footprints of the first candidates {area[cand[:8]].tolist()} tiles")
    offs = [0]
    for cam in cams:
        offs.append(offs[-1] + cam.width * cam.height)
    ref = {k: [] for k in got}
    chosen = []
    for gid in cand:
        acc = {k: 0.0 for k in got}
        ok = True
        for c, cam in enumerate(cams):
            pr = projs[c]
            if pr["radius"][gid] <= 0:
                continue
            rc = pr["rect"][gid]
            win = (int(rc[0]) * 16, int(rc[2]) * 16, min(cam.width, int(rc[1]) * 16),
                   min(cam.height, int(rc[3]) * 16))
            x0, y0, x1, y1 = win
            o = oracle.render(sc.gaussians, sc.mesh, cam, window=win, params=pe())
            H, W, o0 = cam.height, cam.width, offs[c]
            sl = lambda a: a[o0:o0 + H * W].reshape(H, W)[y0:y1, x0:x1]
            im = frame_np["image"][3 * o0:3 * o0 + 3 * H * W].reshape(3, H, W)[:, y0:y1, x0:x1]
            same = (all(np.array_equal(sl(frame_np[k]), o[k])
                        for k in ("n_contrib", "n_blended", "n_processed")) and
                    np.abs(im - o["image"]).max() <= 1e-4 and
                    np.abs(sl(frame_np["final_T"]) - o["final_T"]).max() <= 1e-4)
            if not same:
                ok = False
                break
            gi = gi_all[3 * o0:3 * o0 + 3 * H * W].reshape(3, H, W)[:, y0:y1, x0:x1]
            gt = gt_all[o0:o0 + H * W].reshape(H, W)[y0:y1, x0:x1]
            gm = gm_all[3 * o0:3 * o0 + 3 * H * W].reshape(3, H, W)[:, y0:y1, x0:x1]
            b = oracle.backward(sc.gaussians, sc.mesh, cam, gi, gt, gm, window=win, want_tex=False)
            for k in acc:
                acc[k] = acc[k] + b[k][gid]
        if not ok:
            continue
        for k in got:
            ref[k].append(acc[k])
        chosen.append(gid)
        if len(chosen) >= 8 and int((seen[chosen] >= 2).sum()) >= 3:
            break
    say(f"  Gaussians compared: {chosen}, cameras seeing each: {seen[chosen].tolist()}")
    assert len(chosen) >= 8 and int((seen[chosen] >= 2).sum()) >= 3
    for k in got:
        grad_compare(k, np.stack([got[k][i] for i in chosen]), np.stack(ref[k]))


def _crop_subscene(sc, cam, win):
    """Gaussians whose tile rectangle meets the crop's tiles (the only ones
    that can reach its pixels), in their original order."""
    pr = oracle.project(sc.gaussians, cam)
    x0, y0, x1, y1 = win
    tx0, ty0, tx1, ty1 = x0 // 16, y0 // 16, (x1 + 15) // 16, (y1 + 15) // 16
    r = pr["rect"]
    sel = (pr["radius"] > 0) & (r[:, 0] < tx1) & (r[:, 1] > tx0) & (r[:, 2] < ty1) & (r[:, 3] > ty0)
    return np.nonzero(sel)[0]


def test_1600x1064_gradients_on_a_crop_vs_oracle_and_finite_differences(hr):
    """Forward and backward through the torch.autograd.Functions (render, then
    the loss of Sec. 3.4 on a 32x32 crop, loss.backward()) in the benchmark's
    configuration, against the oracle's analytic gradient and FP64 finite
    differences of its forward. The crop's ambiguous pixels are masked out of
    the loss on both sides (their gradient is then zero)."""
    say("case: 1600x1064, 1M Gaussians, crop gradients through torch.autograd")
    sc = scenes.config3()
    cam = sc.cameras[0]
    g, m = hr.to_device(sc.gaussians, sc.mesh)
    r = hr.Renderer(g, m, [cam], hr.default_settings(**STEP))
    ps = [x.clone().requires_grad_(True) for x in (g.means, g.log_scales, g.quats,
                                                   g.opacity_logits, g.sh, m.tex)]
    image, T, Im, tri = hr.HybridRenderFn().apply(r, *ps)
    torch.cuda.synchronize()
    H, W = cam.height, cam.width
    # a crop with mesh pixels and Gaussians
    rng = np.random.default_rng(33)
    tri_np = tri.view(H, W).cpu().numpy()
    for _ in range(50):
        win = windows(cam, 1, rng)[0]
        x0, y0, x1, y1 = win
        o_nb = oracle.render(sc.gaussians, sc.mesh, cam, window=win, params=pe(), alts=True)
        if (tri_np[y0:y1, x0:x1] >= 0).all() and o_nb["n_blended"].mean() > 2:
            break
    say("crop", win)
    orc = o_nb
    good = orc["amb"] == 0
    im_np = image.detach().view(3, H, W)[:, y0:y1, x0:x1].cpu().numpy()
    T_np = T.detach().view(H, W)[y0:y1, x0:x1].cpu().numpy()
    assert np.abs(im_np - orc["image"])[:, good].max() <= 1e-4
    assert np.abs(T_np - orc["final_T"])[good].max() <= 1e-4
    np.testing.assert_array_equal(tri_np[y0:y1, x0:x1], orc["tri_id"])
    mask_np = (orc["amb"] == 0).astype(np.float32)
    say(f"  ambiguous pixels masked out of the loss: {int((mask_np == 0).sum())}")
    mask = torch.as_tensor(mask_np).cuda()
    tgt_np = sc.target[0][:, y0:y1, x0:x1]
    tgt = torch.as_tensor(np.ascontiguousarray(tgt_np)).cuda()
    crop = lambda t, c: (t.view(c, H, W)[:, y0:y1, x0:x1] if c else t.view(H, W)[y0:y1, x0:x1])
    Ic = (crop(image, 3) * mask).contiguous().reshape(-1)
    Tc = (crop(T, 0) * mask).contiguous().reshape(-1)
    Imc = (crop(Im, 3) * mask).contiguous().reshape(-1)
    tric = crop(tri, 0).contiguous().reshape(-1)
    loss = hr.HybridLossFn().apply(Ic, Tc, Imc, tric, (tgt * mask).reshape(-1),
                                   [(x1 - x0, y1 - y0)])
    loss.backward()
    torch.cuda.synchronize()
    gpu = {k: p.grad.cpu().numpy() for k, p in zip(("means", "log_scales", "quats",
                                                       "opacity_logits", "sh", "tex"), ps)}
    L, gi, gt, gm = oracle.loss(orc["image"] * mask_np, orc["final_T"] * mask_np,
                                orc["mesh_rgb"] * mask_np, orc["tri_id"], tgt_np * mask_np)
    np.testing.assert_allclose(loss.item(), L, rtol=1e-4)
    gi, gt, gm = gi * mask_np, gt * mask_np, gm * mask_np
    ref = oracle.backward(sc.gaussians, sc.mesh, cam, gi.astype(np.float32).astype(np.float64),
                          gt.astype(np.float32).astype(np.float64),
                          gm.astype(np.float32).astype(np.float64), window=win)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "tex"):
        a, b = gpu[k].reshape(-1).astype(np.float64), ref[k].reshape(-1)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        say(f"  {k}: |ref| {np.linalg.norm(b):.3e} rel err {rel:.2e}")
        assert rel <= 1e-3, k

    # FP64 finite differences on the Gaussians that reach the crop
    idx = _crop_subscene(sc, cam, win)
    sub = sc.gaussians.subset(idx)
    p64 = oracle.default_params(flags=oracle.FP64_RECORDS)
    base = dict(means=sub.means.astype(np.float64), log_scales=sub.log_scales.astype(np.float64),
                quats=sub.quats.astype(np.float64), opacity_logits=sub.opacity_logits.astype(np.float64),
                sh=sub.sh.astype(np.float64))

    # the backward's objective: the upstream gradients (zero at ambiguous
    # pixels) held fixed, F = <gi, I_h> + <gt, T> + <gm, I_m> over the crop
    gi64, gt64, gm64 = (x.astype(np.float32).astype(np.float64) for x in (gi, gt, gm))

    def loss_at(over):
        o = oracle.render(sub, sc.mesh, cam, params=p64, window=win, overrides=over)
        F = np.sum(gi64 * o["image"]) + np.sum(gt64 * o["final_T"]) + np.sum(gm64 * o["mesh_rgb"])
        return F, o["trace"]

    # up to 200 sampled scalars of every parameter tensor
    frs = np.random.default_rng(7)
    for name, arr in base.items():
        g_gpu = gpu[name][idx].reshape(-1)
        flat = arr.reshape(-1)
        # sample parameters with a non-negligible gradient
        cand = np.nonzero(np.abs(g_gpu) > 1e-3 * np.abs(g_gpu).max())[0]
        checked = bad = 0
        for j in frs.choice(cand, size=min(len(cand), 200), replace=False):
            h = 1e-6 * max(1.0, abs(flat[j]))
            over = {k: v.copy() for k, v in base.items()}
            over[name].reshape(-1)[j] = flat[j] + h
            lp, tp = loss_at(over)
            over[name].reshape(-1)[j] = flat[j] - h
            lm, tm = loss_at(over)
            if tp != tm:
                continue  # a decision (L1 sign, skip, stop, clamp) flipped
            fd = (lp - lm) / (2 * h)
            checked += 1
            if abs(fd - g_gpu[j]) > 1e-3 * abs(fd) + 1e-6 * np.abs(g_gpu).max():
                bad += 1
        say(f"  {name}: {len(cand)} candidates, FD samples {checked}, outside 1e-3: {bad}")
        assert checked >= min(200, len(cand)) * 0.9 and bad <= 0.01 * checked
    # texels under the crop: F is linear in the texture, so a central
    # difference with a large step is exact
    gtex = gpu["tex"].reshape(-1)
    cand = np.nonzero(gtex != 0)[0]
    tex = sc.mesh.tex
    ok = 0
    sel = frs.choice(cand, size=min(len(cand), 200), replace=False)
    for j in sel:
        t2 = tex.copy()
        v0 = float(t2.reshape(-1)[j])
        hh = 2.0 ** -12
        t2.reshape(-1)[j] = v0 + hh
        lp, tp = loss_at(dict(base, tex=t2))
        t2.reshape(-1)[j] = v0 - hh
        lm, tm = loss_at(dict(base, tex=t2))
        if tp != tm:
            continue
        fd = (lp - lm) / (2 * hh)
        ok += abs(fd - gtex[j]) <= 1e-3 * abs(fd) + 1e-6 * np.abs(gtex).max()
    say(f"  texel FD samples {len(sel)}, within 1e-3: {ok}")
    assert ok >= 0.98 * len(sel) and len(sel) >= 200
