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
# for the blend-only kernels (no mesh shading) they were taken with
BLEND_TRAFFIC = {(32, 0): 165.9e6, (32, 1): 166.2e6, (32, 2): 161.5e6, (32, 3): 161.7e6,
                 (64, 0): 166.1e6, (64, 1): 166.8e6, (64, 2): 161.4e6, (64, 3): 162.1e6,
                 (64, 4): 166.4e6, (128, 0): 166.5e6, (128, 1): 167.6e6, (128, 2): 161.7e6,
                 (128, 3): 162.7e6, (128, 4): 166.9e6, (256, 0): 167.3e6, (256, 1): 168.9e6,
                 (256, 2): 163.0e6, (256, 3): 163.8e6}
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
    ap.add_argument("--no-720p", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="for traces: only the 16-camera batched step and the single-view "
                         "comparison (prints their figures, not the headline line)")
    ap.add_argument("--rect-pairs", action="store_true",
                    help="bin every tile of the 3-sigma rectangle (no tile-ellipse culling)")
    ap.add_argument("--pmc-probe-step", action="store_true",
                    help="for counter runs: one forward + loss + backward of the 16-camera "
                         "step (one-wave backward, batch 128), then 3 copies of a 256 MiB "
                         "buffer (the scale of the byte counters)")
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
    r.settings.batch, r.settings.variant, r.settings.batch_bwd = 256, 8, 64
    f = r.render_hybrid(sync_check=True)
    target = torch.cat([torch.as_tensor(t.reshape(-1)) for t in s4.target]).to(dev)
    _, gi, gt, gm = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target, r.sizes)
    r.render_hybrid_backward(gi, gt, gm)
    torch.cuda.synchronize()
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"pmc step probe done (then 3 copies of {src.numel() * 4} bytes)")


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


HBM_BYTES_PER_S = 8.0e12


def frame_roofline(stage_ms, counts, blend_stats, n_gauss, sh_degree, faces, pixels):
    """Per stage of a 1080p frame: the algorithmic bytes (or VALU lane-ops)
    the method must move (or compute), the time that takes at the HBM (VALU)
    peak, and that time as a fraction of the measured stage time; the frame's
    roofline time is their sum (the mesh pass counted although it runs
    concurrently on its own stream). The blend stage also shades the mesh
    pixels: its roof is the larger of its lane-ops at the VALU peak and the
    shading's bytes at the HBM peak."""
    K = (sh_degree + 1) ** 2
    nv, nk = counts["n_visible"], counts["n_keys"]
    ex, bl = blend_stats["pairs_examined_per_view"], blend_stats["pairs_blended_per_view"]
    valu = VALU_PEAK_TOPS * 1e12
    work = {
        # per Gaussian its 11 geometry and opacity floats in, its visibility and rank
        # out; per visible one its SH coefficients in, depth key, record and
        # rectangle out (culled Gaussians never need their SH)
        "projection": ("hbm", n_gauss * (4 * 11 + 8) + nv * (4 * 3 * K + 4 + 48 + 8)),
        # 4 LSD passes over the visible (depth key, index) pairs, each read and written
        "depth_sort": ("hbm", nv * 8 * 2 * 4),
        # one 4-byte rank per kept (tile, Gaussian) pair
        "binning": ("hbm", nk * 4),
        # the pairs' lane-ops; the shading: 4 texels (48 bytes) and 20 bytes of
        # outputs per mesh pixel
        "blend": ("alu", ex * BLEND_OPS_EXAMINED + bl * BLEND_OPS_BLENDED),
        # the z-buffer cleared (8 bytes per pixel) and one key per mesh pixel, 80 bytes per face
        "mesh": ("hbm", pixels * 8 + counts["mesh_pixels"] * 8 + faces * 80),
    }
    shade_bytes = counts["mesh_pixels"] * 68
    out, total_roof = {}, 0.0
    for k, (bound, amount) in work.items():
        peak = HBM_BYTES_PER_S if bound == "hbm" else valu
        roof_ms = amount / peak * 1e3
        if k == "blend":
            roof_ms = max(roof_ms, shade_bytes / HBM_BYTES_PER_S * 1e3)
        meas = stage_ms[k]
        total_roof += roof_ms
        out[k] = {"bound": bound, "work": int(amount), "unit": "bytes" if bound == "hbm" else "lane-ops",
                  "roof_ms": round(roof_ms, 5), "measured_ms": round(meas, 5),
                  "frac": round(roof_ms / meas, 4) if meas > 0 else None}
        if k == "blend":
            out[k]["shading_bytes"] = int(shade_bytes)
        if bound == "hbm" and meas > 0:
            out[k]["GB_per_s"] = round(amount / (meas * 1e-3) / 1e9, 1)
    out["frame"] = {"roof_ms": round(total_roof, 5), "measured_ms": round(stage_ms["forward"], 5),
                    "frac": round(total_roof / stage_ms["forward"], 4)}
    return out


# lane-operations of the backward per blended (pixel, Gaussian) pair: the pair's
# exponent, alpha and T recovery (12), colour and alpha gradients (10), the
# running colour behind it (3), the power gradient and its three sums (5)
BWD_OPS_BLENDED = 30
# HBM bytes of the projection backward: per Gaussian its parameters in and
# their gradients out plus the per-Gaussian sums (560 B at SH degree 3), per
# visible (Gaussian, camera) item its 9 accumulated gradients (36 B)
PROJ_BWD_BYTES_PER_G, PROJ_BWD_BYTES_PER_ITEM = 560, 36
# HBM bytes of the texture backward: per mesh pixel its stored footprint (16 B)
# and dL/dI_m (12 B) in; per texel its gradient read and written once (24 B).
# The kernel itself is bound by its atomics (the texels of a workgroup's box
# are summed in LDS first, then added to the gradient with one atomic each)
TEX_BWD_BYTES_PER_PIXEL, TEX_BWD_BYTES_PER_TEXEL = 28, 24


def backward_roofline(stage_ms, n_blended, n_gauss, n_visible, mesh_pixels, texels):
    """Per stage of the backward (timed alone): its algorithmic work, the time
    that takes at the unit's peak, and that time over the measured time."""
    work = {
        "blend_backward": ("alu", n_blended * BWD_OPS_BLENDED, VALU_PEAK_TOPS * 1e12, "lane-ops"),
        "projection_backward": ("hbm", n_gauss * PROJ_BWD_BYTES_PER_G +
                                n_visible * PROJ_BWD_BYTES_PER_ITEM, HBM_BYTES_PER_S, "bytes"),
        "texture_backward": ("hbm", mesh_pixels * TEX_BWD_BYTES_PER_PIXEL +
                             texels * TEX_BWD_BYTES_PER_TEXEL, HBM_BYTES_PER_S, "bytes"),
    }
    out = {}
    for k, (bound, amount, peak, unit) in work.items():
        meas = stage_ms[k]
        roof = amount / peak * 1e3
        out[k] = {"bound": bound, "work": int(amount), "unit": unit, "peak_per_s": peak,
                  "roof_ms": round(roof, 5), "measured_ms": round(meas, 5),
                  "frac": round(roof / meas, 4) if meas > 0 else None}
    return out


def single_view_steps(torch, hr, s4, g, m, settings, target_parts, dev, reps=2):
    """The plain single-view path: each of the 16 cameras rendered, its loss
    taken and its backward run on its own (eager calls, one camera per call),
    with the batched step's settings. Returns milliseconds per 16 views."""
    sizes = sorted({(c.width, c.height) for c in s4.cameras})
    rs, bufs = {}, {}
    for wh in sizes:
        cam0 = next(c for c in s4.cameras if (c.width, c.height) == wh)
        rr = hr.Renderer(g, m, [cam0], settings=hr.hr_settings.from_buffer_copy(settings))
        rs[wh] = (rr, rr.new_frame())
        P = wh[0] * wh[1]
        bufs[wh] = (torch.zeros(1, device=dev), torch.empty(3 * P, device=dev),
                    torch.empty(P, device=dev), torch.empty(3 * P, device=dev),
                    torch.empty(hr.loss_scratch_bytes([wh]), dtype=torch.uint8, device=dev))
    grads = rs[sizes[0]][0]._zero_grads(g)

    def one_pass():
        for c, cam in enumerate(s4.cameras):
            rr, f = rs[(cam.width, cam.height)]
            rr.set_cameras([cam])
            rr.render_hybrid(f, sync_check=False)
            _, gi, gt, gm = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target_parts[c],
                                           out=bufs[(cam.width, cam.height)])
            for t in grads.values():
                t.zero_()
            rr.render_hybrid_backward(gi, gt, gm, grads=grads)

    # size every capacity first (the eager capacity check may regrow)
    for c, cam in enumerate(s4.cameras):
        rr, f = rs[(cam.width, cam.height)]
        rr.set_cameras([cam])
        rr.render_hybrid(f, sync_check=True)
        rs[(cam.width, cam.height)] = (rr, rr.new_frame() if f.image.numel() != 3 * rr.P else f)
    one_pass()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        one_pass()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_frame_rate(oracle, sc, views, half):
    """Seconds of oracle work and the extrapolated 1920x1080 frames/s over
    `views`: per view a 16x16 and a (2 half)^2 window at the centre give the
    per-call and the per-pixel cost."""
    t_frames = t_spent = 0.0
    for cam in views:
        cx, cy = cam.width // 2, cam.height // 2
        t0 = time.perf_counter()
        oracle.render(sc.gaussians, sc.mesh, cam, window=(cx - 8, cy - 8, cx + 8, cy + 8))
        t_small = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.render(sc.gaussians, sc.mesh, cam, window=(cx - half, cy - half, cx + half, cy + half))
        t_big = time.perf_counter() - t0
        per_px = max(t_big - t_small, 1e-9) / ((2 * half) ** 2 - 256)
        t_frames += t_small + per_px * (cam.width * cam.height - 256)
        t_spent += t_small + t_big
    return t_spent, len(views) / t_frames


SINGLE_THREAD_SAMPLE = """
import json, os, sys
sys.path.insert(0, {root!r})
import bench, oracle
from paper_2506_06988_amd import scenes
sc = scenes.config5("hybrid")
spent, fps = bench.oracle_frame_rate(oracle, sc, sc.cameras[:2], 96)
print(json.dumps({{"spent": spent, "fps": fps, "threads": oracle.threads()}}))
"""


def cpu_baseline(scenes):
    """The CPU FP64 oracle on a bounded sample of the headline workload, on all
    the host's cores (median of 3 runs over 16 of the 32 views) and on one
    thread (2 views, in a child process started with OMP_NUM_THREADS=1)."""
    import subprocess
    import oracle
    sc = scenes.config5("hybrid")
    runs, spent = [], 0.0
    for rep in range(3):
        sp, fps = oracle_frame_rate(oracle, sc, sc.cameras[rep % 2::2], 160)
        runs.append(fps)
        spent += sp
    runs.sort()
    env = dict(os.environ, OMP_NUM_THREADS="1")
    child = subprocess.run([sys.executable, "-c", SINGLE_THREAD_SAMPLE.format(root=ROOT)],
                           capture_output=True, text=True, env=env, timeout=600)
    one = json.loads(child.stdout.strip().splitlines()[-1]) if child.returncode == 0 else None
    threads = oracle.threads()
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    log(f"cpu oracle: runs {[round(x, 4) for x in runs]} frames/s on {threads} threads "
        f"({spent:.1f}s); one thread: {one}")
    out = {"value": round(runs[1], 5), "unit": "frames/s", "cores": threads, "kind": "oracle",
           "sample": (f"FP64 oracle (OpenMP, {threads} threads) on the headline workload: per view "
                      f"a 16x16 and a 320x320 window at the centre give the per-call and "
                      f"per-pixel cost, extrapolated to 1920x1080; median of 3 runs over 16 of the "
                      f"32 views ({spent:.1f}s in all)"),
           "runs_frames_per_s": [round(x, 5) for x in runs], "nproc": nproc, "cpu_model": cpu_model()}
    if one is not None:
        out["single_thread"] = {"value": round(one["fps"], 6), "unit": "frames/s",
                                "threads": one["threads"],
                                "sample": "2 views, 16x16 and 192x192 windows, extrapolated"}
    out["other_workloads"] = cpu_other_workloads(scenes, oracle)
    return out


def cpu_other_workloads(scenes, oracle):
    """The oracle on the other workloads, on all the host's threads: full frames
    of the 64x64 quad scene and of the 720p room, 64 tiles (a 128x128 window at
    the centre) of the 1600x1064 and of one 1920x1080 view of the 16-camera
    room, and the gradient over the 32x32 crop of the 1600x1064 room."""
    import numpy as np
    res = {}

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    s1 = scenes.config1()
    c1 = s1.cameras[0]
    res["config1_64x64_frames_per_s"] = round(1.0 / timed(lambda: oracle.render(s1.gaussians, s1.mesh, c1)), 3)
    s2 = scenes.config2()
    c2 = s2.cameras[0]
    res["config2_720p_frames_per_s"] = round(1.0 / timed(lambda: oracle.render(s2.gaussians, s2.mesh, c2)), 4)
    del s2
    s3 = scenes.config3()
    c3 = s3.cameras[0]
    cx, cy = c3.width // 2, c3.height // 2
    win = (cx - 64, cy - 64, cx + 64, cy + 64)
    res["config3_64_tiles_s"] = round(timed(lambda: oracle.render(s3.gaussians, s3.mesh, c3, window=win)), 3)
    rng = np.random.default_rng(7)
    crop = (cx - 16, cy - 16, cx + 16, cy + 16)
    gi = rng.normal(0, 1, (3, 32, 32))
    gt = rng.normal(0, 1, (32, 32))
    gm = rng.normal(0, 1, (3, 32, 32))
    res["config3_crop_32x32_gradient_s"] = round(
        timed(lambda: oracle.backward(s3.gaussians, s3.mesh, c3, gi, gt, gm, window=crop)), 3)
    del s3
    s4 = scenes.config4()
    c4 = max(s4.cameras, key=lambda c: c.width * c.height)
    cx, cy = c4.width // 2, c4.height // 2
    win = (cx - 64, cy - 64, cx + 64, cy + 64)
    res["config4_64_tiles_s"] = round(timed(lambda: oracle.render(s4.gaussians, s4.mesh, c4, window=win)), 3)
    log(f"cpu oracle, other workloads: {res}")
    return res


def batched_step(torch, hr, scenes, dev, args, result):
    """The 16-camera hipGraph training step (forward, loss, backward), then the
    same cameras through the plain single-view path; fills `result`."""
    s4 = scenes.config4()
    g, m = hr.to_device(s4.gaussians, s4.mesh, device=dev)
    r = hr.Renderer(g, m, s4.cameras, settings=hr.default_settings(flags=PAIR_CULL))
    f = r.render_hybrid(sync_check=True)
    torch.cuda.synchronize()
    target = torch.cat([torch.as_tensor(t.reshape(-1)) for t in s4.target]).to(dev)
    r.autotune(f, repeats=2)
    L0, gi0, gt0, _ = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target,
                                      r.sizes)
    r.autotune_backward(gi0, gt0, repeats=5)
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
    # the backward's stages timed one after another (hr_render_hybrid_backward_timed,
    # serial), median of 3, with their roofline fractions
    f = r.render_hybrid(sync_check=True)
    _, gi1, gt1, gm1 = hr.hybrid_loss(f.image, f.final_T, f.mesh_rgb, f.tri_id, target, r.sizes)
    sb = f.stats_dict()
    mesh_px = float((f.tri_id >= 0).sum().item())
    reps = [r.render_hybrid_backward_timed(gi1, gt1, gm1, serial=True)[0] for _ in range(3)]
    bt = {k: sorted(x[k] for x in reps)[1] for k in hr.BWD_STAGES}
    log("step backward stages (alone): " + ", ".join(f"{k} {v:.3f} ms" for k, v in bt.items()))
    result["step_backward_stage_ms"] = {k: round(v, 4) for k, v in bt.items()}
    texels = int(s4.mesh.tex.shape[0] * s4.mesh.tex.shape[1] * s4.mesh.tex.shape[2])
    result["step_backward_roofline"] = backward_roofline(bt, sb["n_blended"], s4.gaussians.n,
                                                         sb["n_visible"], mesh_px, texels)
    log("step backward roofline: " + json.dumps(result["step_backward_roofline"]))
    del gi1, gt1, gm1
    # the plain single-view path on the same GPU: the 16 cameras one by one
    parts = [torch.as_tensor(t.reshape(-1)).to(dev) for t in s4.target]
    sv_ms = single_view_steps(torch, hr, s4, g, m, r.settings, parts, dev)
    log(f"single-view fwd+bwd of the 16 cameras one by one: {sv_ms:.2f} ms "
        f"({len(s4.cameras) / sv_ms * 1e3:.1f} views/s)")
    result["single_view_fwd_bwd_views_per_s"] = round(len(s4.cameras) / sv_ms * 1e3, 2)
    result["batched_vs_single_view"] = round(sv_ms / (bsec * 1e3), 3)
    del step, r, f, g, m, s4, parts
    torch.cuda.empty_cache()


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
    if args.batched_only:
        part = {}
        batched_step(torch, hr, scenes, dev, args, part)
        print(json.dumps(part), flush=True)
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

    # stage times (events between the stages, hr_render_hybrid_timed) and the
    # forward without the mesh pass (the mesh of the same view kept in the
    # workspace, HR_FLAG_MESH_REUSED), over all 32 views
    stage_sum = {k: 0.0 for k in hr.STAGES}
    no_mesh_ms = 0.0
    counts = dict(n_visible=0, n_keys=0, mesh_pixels=0)
    for v in range(len(sc.cameras)):
        r.set_cameras([sc.cameras[v]])
        t = r.render_hybrid_timed(frame)
        for k in stage_sum:
            stage_sum[k] += t[k] / len(sc.cameras)
        st_v = frame.stats_dict()
        counts["n_visible"] += st_v["n_visible"] / len(sc.cameras)
        counts["n_keys"] += st_v["n_keys"] / len(sc.cameras)
        counts["mesh_pixels"] += float((frame.tri_id >= 0).sum().item()) / len(sc.cameras)
        no_mesh_ms += r.render_hybrid_timed(frame, mesh_reused=True)["forward"] / len(sc.cameras)
    log("stage ms per 1080p view: " + ", ".join(f"{k} {v:.4f}" for k, v in stage_sum.items()) +
        f"; forward without the mesh pass {no_mesh_ms:.4f} ms")
    roof = frame_roofline(stage_sum, counts, hyb_stats, n_gauss=sc.gaussians.n,
                          sh_degree=sc.gaussians.sh_degree, faces=sc.mesh.n_faces,
                          pixels=sc.cameras[0].width * sc.cameras[0].height)
    log("frame roofline: " + json.dumps(roof))
    del r, frame
    torch.cuda.empty_cache()
    # throughput with 4 of the views per call (one forward over 4 cameras: the
    # latency-bound sort and binning run once for the 4)
    groups = [sc.cameras[4 * k:4 * k + 4] for k in range(len(sc.cameras) // 4)]
    r4 = hr.Renderer(g, m, groups[0], settings=hr.default_settings(flags=PAIR_CULL))
    r4.settings.batch, r4.settings.variant = tuning["batch"], tuning["variant"]
    f4 = r4.new_frame()
    for grp in groups:
        r4.set_cameras(grp)
        r4.render_hybrid(f4, sync_check=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n4 = max(8, args.steps // 4)
    e0.record(st)
    for k in range(n4):
        r4.set_cameras(groups[k % len(groups)])
        r4.render_hybrid(f4, sync_check=False)
    e1.record(st)
    torch.cuda.synchronize()
    fps4 = 4 * n4 / (e0.elapsed_time(e1) / 1e3)
    log(f"1080p hybrid, 4 views per call: {fps4:.1f} frames/s")
    del r4, f4, g, m
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
        "n_keys_per_view": int(counts["n_keys"]),
        "n_visible_per_view": int(counts["n_visible"]),
        "stage_ms_per_view": {k: round(v, 4) for k, v in stage_sum.items()},
        "frames_per_s_without_mesh_pass": round(1e3 / no_mesh_ms, 2),
        "frames_per_s_4_views_per_call": round(fps4, 2),
        "frame_roofline": roof,
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

    # ------------------------------------------------------- 720p, config 2
    if not args.no_720p:
        s2 = scenes.config2()
        g, m = hr.to_device(s2.gaussians, s2.mesh, device=dev)
        rt = hr.Renderer(g, m, s2.cameras, settings=hr.default_settings(flags=PAIR_CULL))
        ft = rt.render_hybrid(sync_check=True)
        rt.autotune(ft, repeats=3)
        r = hr.Renderer(g, m, [s2.cameras[0]], settings=hr.default_settings(flags=PAIR_CULL))
        r.settings.batch, r.settings.variant = rt.settings.batch, rt.settings.variant
        del rt, ft
        frame = r.new_frame()
        for v in range(len(s2.cameras)):
            r.set_cameras([s2.cameras[v]])
            r.render_hybrid(frame, sync_check=True)
        sec2, _ = timed_frames(torch, r, frame, s2.cameras, max(8, args.steps // 2), 2)
        log(f"720p hybrid (300k Gaussians, 50k faces): {sec2 * 1e3:.3f} ms/frame "
            f"({1 / sec2:.1f} frames/s)")
        result["config2_720p_frames_per_s"] = round(1.0 / sec2, 2)
        del r, frame, g, m, s2
        torch.cuda.empty_cache()

    # --------------------------------------------------- batched fwd + bwd
    if not args.no_batched:
        batched_step(torch, hr, scenes, dev, args, result)

    # ------------------------------------------------------- CPU baseline
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(scenes)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
