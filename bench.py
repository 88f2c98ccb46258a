"""Throughput of the hybrid mesh-Gaussian rasterizer on one MI355X.

Headline: 1080p hybrid frames/s - forward joint rasterization (mesh z-buffer
and texture, Gaussian projection, depth sort and tile binning, per-tile blend
with the mesh depth stop) of the hybrid room: 600k Gaussians (SH degree 3),
a 200k-triangle room mesh with four 4096x4096 textures, 32 seeded interior
views at 1920x1080. One step renders one view. Also measured in the same run:
  * the blend kernel alone (Gaussian-pixel pairs examined per second, and its
    fraction of the FP32 VALU peak),
  * batched forward + loss + backward views/s: 16 cameras of uneven sizes,
    1M Gaussians, 200k triangles, 2048x2048 textures, one hipGraph per step,
  * the Gaussian-only room (3M Gaussians, no mesh) at 1080p for comparison,
  * the CPU FP64 oracle on a bounded sample of the headline workload.
Inputs are synthetic (seeded) and resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("1080p hybrid frames/s and batched fwd+bwd views/s; "
          "Gaussian-pixel blends/s vs VALU peak")
# VALU lane-operation rate of the MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU lane-operations of the blend (an FMA is one operation, the
# exponential one): per examined (Gaussian, pixel) pair, the offset (2), the
# conic quadratic form (5), exp and the opacity product (2), the alpha and
# depth tests (2); per blended pair, the alpha clamp (1), alpha*T (1), the
# colour update (3), the transmittance update (1) and its test (1). Staging,
# addressing and loop control are not counted.
BLEND_OPS_EXAMINED = 11
BLEND_OPS_BLENDED = 7
# HBM bytes per blend launch over the 32 headline views, by (batch, variant),
# from the FETCH_SIZE and WRITE_SIZE counter passes of `bench.py --pmc-probe`
# (scaled by a 256 MiB copy: FETCH x2, WRITE x1), tile-ellipse binning; valid
# for the blend kernels they were taken with
BLEND_TRAFFIC = {(32, 0): 165.9e6, (32, 1): 166.2e6, (32, 2): 161.0e6, (32, 3): 161.4e6,
                 (64, 0): 166.1e6, (64, 1): 166.8e6, (64, 2): 161.3e6, (64, 3): 162.0e6,
                 (64, 4): 166.4e6, (128, 0): 166.5e6, (128, 1): 167.5e6, (128, 2): 161.7e6,
                 (128, 3): 162.7e6, (128, 4): 166.9e6, (256, 0): 167.3e6, (256, 1): 168.8e6,
                 (256, 2): 162.2e6, (256, 3): 163.8e6}
# every configuration the forward autotuner may choose
BLEND_CONFIGS = [(b, v) for v in range(4) for b in (32, 64, 128, 256)] + [(64, 4), (128, 4)]
# pairs outside the alpha >= alpha_min ellipse are skipped by every pixel:
# binning only the tiles the ellipse reaches leaves every image unchanged
PAIR_CULL = 0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-gaussian-only", action="store_true")
    ap.add_argument("--rect-pairs", action="store_true",
                    help="bin every tile of the 3-sigma rectangle (no tile-ellipse culling)")
    ap.add_argument("--pmc-probe-step", action="store_true",
                    help="for counter runs: one forward + loss + backward of the 16-camera "
                         "step (one-wave backward, batch 128)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for counter runs: every view of the headline workload once (plus one "
                         "extra blend), then 3 copies of a 256 MiB buffer (the scale of the byte "
                         "counters)")
    return ap.parse_args()


def pmc_probe(torch, hr, scenes, dev):
    """One forward of each of the 32 headline views, each followed by one
    blend in every configuration the autotuner may choose, then 3 copies of a
    256 MiB buffer: the dispatches the byte counters are read over, and the
    copy that scales them."""
    sc = scenes.config5("hybrid")
    g, m = hr.to_device(sc.gaussians, sc.mesh, device=dev)
    r = hr.Renderer(g, m, [sc.cameras[0]], settings=hr.default_settings(flags=PAIR_CULL))
    frame = r.new_frame()
    for v in range(len(sc.cameras)):
        r.set_cameras([sc.cameras[v]])
        r.settings.batch, r.settings.variant = 256, 0
        r.render_hybrid(frame, sync_check=True)
        for b, var in BLEND_CONFIGS:
            r.settings.batch, r.settings.variant = b, var
            r.blend_forward(frame)
    torch.cuda.synchronize()
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"pmc probe done: 32 views x {len(BLEND_CONFIGS)} blend configurations, "
        f"copy bytes {src.numel() * 4}")


def pmc_probe_step(torch, hr, scenes, dev):
    s4 = scenes.config4()
    g, m = hr.to_device(s4.gaussians, s4.mesh, device=dev)
    r = hr.Renderer(g, m, s4.cameras, settings=hr.default_settings(flags=PAIR_CULL))
    r.settings.batch, r.settings.variant, r.settings.batch_bwd = 256, 8, 128
    f = r.render_hybrid(sync_check=True)
    target = torch.cat([torch.as_tensor(t.reshape(-1)) for t in s4.target]).to(dev)
    _, gi, gt, gm = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target, r.sizes)
    r.render_hybrid_backward(gi, gt, gm)
    torch.cuda.synchronize()
    log("pmc step probe done")


def timed_frames(torch, r, frame, views, steps, warmup):
    """Renders views round robin; returns seconds per frame (events on the stream)."""
    for k in range(warmup):
        r.set_cameras([views[k % len(views)]])
        r.render_hybrid(frame, sync_check=True)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    for k in range(steps):
        r.set_cameras([views[k % len(views)]])
        r.render_hybrid(frame, sync_check=False)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3 / steps, wall / steps


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for {args.gpus}); with several GPUs each would render its own share "
              f"of the views, so the one-GPU figure is the per-GPU rate.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2506_06988_amd import hr, scenes

    hr.load()
    assert torch.cuda.is_available()
    dev = "cuda:0"
    global PAIR_CULL
    PAIR_CULL = 0 if args.rect_pairs else hr.HR_FLAG_TILE_ELLIPSE
    if args.pmc_probe:
        pmc_probe(torch, hr, scenes, dev)
        return
    if args.pmc_probe_step:
        pmc_probe_step(torch, hr, scenes, dev)
        return

    # ----------------------------------------------------- headline: 1080p
    t = time.perf_counter()
    sc = scenes.config5("hybrid")
    log(f"hybrid scene built in {time.perf_counter() - t:.1f}s: {sc.gaussians.n} Gaussians, "
        f"{sc.mesh.n_faces} faces, textures {sc.mesh.tex.shape}")
    g, m = hr.to_device(sc.gaussians, sc.mesh, device=dev)
    r = hr.Renderer(g, m, [sc.cameras[0]], settings=hr.default_settings(flags=PAIR_CULL))
    frame = r.new_frame()
    # size the key capacity over all views
    for v in range(len(sc.cameras)):
        r.set_cameras([sc.cameras[v]])
        r.render_hybrid(frame, sync_check=True)
    torch.cuda.synchronize()
    # tune the blend on 8 of the views rendered together (one call, the mix
    # of the workload), then use the choice for single-view frames
    tv = sc.cameras[::4]
    rt = hr.Renderer(g, m, tv, settings=hr.default_settings(flags=PAIR_CULL))
    ft = rt.render_hybrid(sync_check=True)
    rt.autotune(ft, repeats=3)
    r.settings.batch, r.settings.variant = rt.settings.batch, rt.settings.variant
    del rt, ft
    torch.cuda.empty_cache()
    log(f"autotuned blend: batch {r.settings.batch} variant {r.settings.variant}")
    sec, wall = timed_frames(torch, r, frame, sc.cameras, args.steps, args.warmup)
    fps = 1.0 / sec
    log(f"1080p hybrid: {sec * 1e3:.3f} ms/frame ({fps:.1f} frames/s), wall {wall * 1e3:.3f} ms")

    # the blend kernel alone over the same 32 views: each view is rendered,
    # then its blend re-run (hr_blend_forward) `nb` times between events on
    # the launch stream; the work is the views' examined and blended pairs
    st = torch.cuda.current_stream()
    nb = 4
    blend_s = 0.0
    pairs = blended = 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for v in range(len(sc.cameras)):
        r.set_cameras([sc.cameras[v]])
        r.render_hybrid(frame)
        r.blend_forward(frame)
        torch.cuda.synchronize()
        stats = frame.stats_dict()
        e0.record(st)
        for _ in range(nb):
            r.blend_forward(frame)
        e1.record(st)
        torch.cuda.synchronize()
        blend_s += e0.elapsed_time(e1) / 1e3
        pairs += nb * stats["n_processed"]
        blended += nb * stats["n_blended"]
    launches = nb * len(sc.cameras)
    ops = pairs * BLEND_OPS_EXAMINED + blended * BLEND_OPS_BLENDED
    achieved = ops / blend_s / 1e12
    blends_per_s = pairs / blend_s
    log(f"blend kernel over {len(sc.cameras)} views: {blend_s / launches * 1e3:.3f} ms/launch, "
        f"{pairs // launches} pairs examined and {blended // launches} blended per launch, "
        f"{blends_per_s:.3e} pairs/s, {achieved:.2f} TOP/s")
    hyb_stats = dict(pairs_examined_per_view=pairs // launches,
                     pairs_blended_per_view=blended // launches)
    tuning = {"batch": int(r.settings.batch), "variant": int(r.settings.variant)}
    del r, frame, g, m
    torch.cuda.empty_cache()

    result = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded room scenes)",
        "config": {"workload": "config5 hybrid: 1920x1080, 600k Gaussians SH3, 200k-triangle room "
                               "mesh, 4x4096^2 textures, 32 views, forward",
                   "gaussians": 600000, "faces": int(sc.mesh.n_faces), "width": 1920,
                   "height": 1080, "views": len(sc.cameras),
                   "pair_binning": "3-sigma rectangle" if args.rect_pairs else "tile-ellipse"},
        "blend_pairs_per_s": blends_per_s,
        "blend_ms_per_launch": round(blend_s / launches * 1e3, 4),
        "blend_stats": hyb_stats,
        "blend_tuning": tuning,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": BLEND_TRAFFIC.get((tuning["batch"], tuning["variant"])),
                     "traffic_unit": "HBM bytes per launch",
                     "kernel": "k_blend_fwd", "ops_per_examined": BLEND_OPS_EXAMINED,
                     "ops_per_blended": BLEND_OPS_BLENDED, "ops_per_launch": ops // launches,
                     "avg_launch_ms": round(blend_s / launches * 1e3, 4)},
    }
    del sc

    # --------------------------------------------------- Gaussian-only room
    if not args.no_gaussian_only:
        sg = scenes.config5("gaussian_only")
        g, _ = hr.to_device(sg.gaussians, None, device=dev)
        r = hr.Renderer(g, None, [sg.cameras[0]], settings=hr.default_settings(flags=PAIR_CULL))
        frame = r.new_frame()
        for v in range(len(sg.cameras)):
            r.set_cameras([sg.cameras[v]])
            r.render_hybrid(frame, sync_check=True)
        r.settings.batch, r.settings.variant = 64, 0
        sec_g, _ = timed_frames(torch, r, frame, sg.cameras, max(8, args.steps // 2), 2)
        log(f"1080p Gaussian-only (3M): {sec_g * 1e3:.3f} ms/frame ({1 / sec_g:.1f} frames/s)")
        result["gaussian_only_frames_per_s"] = round(1.0 / sec_g, 2)
        del r, frame, g, sg
        torch.cuda.empty_cache()

    # --------------------------------------------------- batched fwd + bwd
    if not args.no_batched:
        s4 = scenes.config4()
        g, m = hr.to_device(s4.gaussians, s4.mesh, device=dev)
        r = hr.Renderer(g, m, s4.cameras, settings=hr.default_settings(flags=PAIR_CULL))
        f = r.render_hybrid(sync_check=True)
        torch.cuda.synchronize()
        target = torch.cat([torch.as_tensor(t.reshape(-1)) for t in s4.target]).to(dev)
        r.autotune(f, repeats=2)
        L0, gi0, gt0, _ = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target,
                                          r.sizes)
        r.autotune_backward(gi0, gt0, repeats=2)
        log(f"batched tuning: forward batch {r.settings.batch}, backward batch "
            f"{r.settings.batch_bwd}, variant {r.settings.variant}")
        del L0, gi0, gt0
        step = hr.BatchedStep(r, target)
        for _ in range(2):
            step.launch()
        step.stream.synchronize()
        nst = max(4, args.steps // 8)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(step.stream)
        for _ in range(nst):
            step.launch()
        e1.record(step.stream)
        step.stream.synchronize()
        bsec = e0.elapsed_time(e1) / 1e3 / nst
        views_s = len(s4.cameras) / bsec
        log(f"batched fwd+bwd (16 cams, graph): {bsec * 1e3:.2f} ms/step, {views_s:.1f} views/s, "
            f"loss {step.loss.item():.5f}")
        result["batched_fwd_bwd_views_per_s"] = round(views_s, 2)
        result["batched_tuning"] = {"batch": int(r.settings.batch),
                                    "batch_bwd": int(r.settings.batch_bwd),
                                    "variant": int(r.settings.variant)}
        result["batched_ms_per_step"] = round(bsec * 1e3, 3)
        step.close()
        del step, r, f, g, m, s4
        torch.cuda.empty_cache()

    # ------------------------------------------------------- CPU baseline
    if not args.no_cpu_baseline:
        import oracle
        sc = scenes.config5("hybrid")
        views = sc.cameras
        t_frames = 0.0
        t_spent = 0.0
        for cam in views:
            # a 16x16 and a 480x480 window at the centre give the per-call
            # and the per-pixel cost of this view, extrapolated to 1920x1080
            cx, cy = cam.width // 2, cam.height // 2
            t0 = time.perf_counter()
            oracle.render(sc.gaussians, sc.mesh, cam, window=(cx - 8, cy - 8, cx + 8, cy + 8))
            t_small = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.render(sc.gaussians, sc.mesh, cam, window=(cx - 240, cy - 240, cx + 240, cy + 240))
            t_big = time.perf_counter() - t0
            per_px = max(t_big - t_small, 1e-9) / (480 * 480 - 256)
            t_frames += t_small + per_px * (cam.width * cam.height - 256)
            t_spent += t_small + t_big
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        result["cpu_baseline"] = {
            "value": round(len(views) / t_frames, 5), "unit": "frames/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"oracle (FP64, OpenMP) on all {len(views)} headline views: per view a "
                       f"16x16 and a 480x480 window at the centre ({t_spent:.1f}s in all) give the "
                       f"per-call and per-pixel cost, extrapolated to the 1920x1080 frame")}
        log(f"cpu oracle: {t_spent:.1f}s of samples -> {len(views) / t_frames:.4f} frames/s extrapolated")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
