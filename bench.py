#!/usr/bin/env python3
"""Binocular 2DGS frame path on one MI355X: stereo frames/s and p99 ms per
stereo frame of the reprojection-and-patch pipeline, next to the sequential
two-pass render (the same full render run for both eyes), with the
affiliated-eye PSNR of the pipeline against the full render.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--workload sphere800]

One step = one stereo frame: dominant render with the depth proxy,
reprojection, hole classification and interpolation, ROI re-rendering of
the affiliated eye.  Frames cycle through the workload's poses; inputs are
resident in HBM before the timed regions.

Two timed regions per method, each of exactly --steps frames between
synchronisations:
  * one frame at a time: frames issued back to back on one stream; p50/p99
    are per-frame GPU times from events recorded around each frame; only
    the dominant-eye blend carries the library's stage events (for the
    roofline's live average).
  * frames in flight (`value`): --inflight contexts, each with its own
    workspace and default-priority stream, frames assigned round robin, as
    a serving loop runs independent frames; throughput = steps / wall time.
    Long tile lists are not split into continuation segments here
    (--inflight-split): the segments shorten one frame's blend by doing
    speculative extra work, which costs throughput when other frames
    already fill the GPU.  One frame at a time keeps the library's
    latency-oriented default split.
The two-pass comparison (the same full render for both eyes) is timed the
same two ways.  The per-stage breakdown comes from a separate, fully
instrumented pass.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

# Paper's two-pass affiliated-eye PSNR against captured images, used as the
# reference noise level of the PSNR-loss stand-in (object-centric / DTU-like
# scenes; unbounded / MipNeRF-360-like scenes).
P_REF = {"cube256": 28.83, "sphere800": 28.83, "unbounded1600": 26.14}
WORKLOAD_TEXT = {
    "cube256": "cube256: 10k surfels uniform in [-1,1]^3, SH0, 256x256 per eye, fx=fy=300, 1 pose, baseline 0.064",
    "sphere800": "sphere800: 300k surfels on a noisy unit sphere shell, SH3, 800x600 per eye, fx=fy=1100, "
                 "16 poses on an orbit of radius 3, baseline 0.064",
    "unbounded1600": "unbounded1600: 1M surfels (70% unit ball, 30% log-uniform shell r=1-20), SH3, 1600x1064 per "
                     "eye, fx=fy=1300, 32 poses on a forward path, baseline 0.064",
}
# Published MI355X peaks.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# HBM bytes of one sphere800 dominant-eye blend stage (capped walk, two
# segment rounds, chain, fix-up), FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0
# (factors from a 512 MiB copy), valid while raster.hip and bgs_api.hip hash
# (sha1 over the two files in that order) to this value.
BLEND_TRAFFIC = {"source_sha1": "d38cf24a846cd3817a9fda718d17bb872d6199f3", "bytes": 120.1e6}
# fp32 operations of one evaluated (pixel, surfel) pair in the blend and the
# extra ones of a contributing pair (an FMA counts as two).
FLOPS_EVAL = 31
FLOPS_USED = 12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sphere800", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--center-roi", type=int, default=1)
    ap.add_argument("--margin", type=int, default=32, help="ROI safety margin m in pixels (the paper fixes 32)")
    ap.add_argument("--edge-bounds", type=int, default=0,
                    help="edge-ROI bounds: 0 = Eq. 6 over all edge samples, 1 = each side's own edge, worst case")
    ap.add_argument("--surfels", type=int, default=0, help="surfel count of the workload's scene (0: its default)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--inflight", type=int, default=4,
                    help="frames in flight for the throughput region: one context and one default-priority stream "
                         "each, frames assigned round robin (the two-pass baseline the same way)")
    ap.add_argument("--inflight-split", default="0,0,128,0,0",
                    help="blend split (cap_dom, cap_roi, seg_len, far_dom, far_roi) of the in-flight region, "
                         "both methods; 0,0 never continues a tile list")
    ap.add_argument("--traffic-probe-stereo", action="store_true",
                    help="no timing: 48 stereo frames of the workload at the default blend split (16 sizing the "
                         "workspace, then 32), for per-kernel rocprofv3 counter runs of the sorts and reprojection")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="no timing: a 512 MiB copy (counter calibration), then 12 dominant-eye renders of the "
                         "workload, for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1 (the frame path shards "
                                   "by frame, see the design notes)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2609_30741_amd import api, synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.traffic_probe:
        traffic_probe(args)
        return
    if args.traffic_probe_stereo:
        traffic_probe_stereo(args)
        return

    t0 = time.time()
    wl_kw = {"n": args.surfels} if args.surfels > 0 else {}
    scene, cams, baseline = synth.WORKLOADS[args.workload](args.seed, **wl_kw)
    affs = [synth.affiliated(c, baseline) for c in cams]
    ds = api.DeviceScene(scene)
    ctx = api.Context(sync=True)
    roi = api.Roi(center_roi=bool(args.center_roi), margin=args.margin, edge_bounds=args.edge_bounds)
    raster = api.Raster()
    log(f"scene {args.workload}: n={scene.n} generated+uploaded in {time.time() - t0:.1f}s")

    # ---- untimed: size the workspace on every pose, quality and pair counts ----
    from paper_2609_30741_amd import metrics
    ps, ss, keys_dom, keys_roi, roi_tiles, n_boxes = [], [], [], [], [], []
    out = None
    full = None
    for i, (cd, ca) in enumerate(zip(cams, affs)):
        out = ctx.render_stereo(ds, cd, ca, raster, roi, out=out)
        st = out["stats"]
        keys_dom.append(st["n_keys_dom"])
        keys_roi.append(st["n_keys_roi"])
        roi_tiles.append(st["n_roi_tiles"])
        n_boxes.append(st["n_boxes"])
        full = ctx.render_dominant(ds, ca, raster, out=full)
        ps.append(api.psnr(out["rgb_aff"], full["rgb"]))
        ss.append(metrics.ssim(out["rgb_aff"].cpu().numpy(), full["rgb"].cpu().numpy()))
    # Reserve 25% headroom over the largest key count so the timed frames
    # never run out of capacity.
    kmax = max(max(keys_dom), max(keys_roi))
    ctx.reserve(scene.n, cams[0].width, cams[0].height, int(kmax * 1.25) + 4096)
    n_tiles = ((cams[0].width + 15) // 16) * ((cams[0].height + 15) // 16)
    mse_ref = 10 ** (-P_REF[args.workload] / 10)
    mses = [10 ** (-p / 10) for p in ps]
    delta_db = float(np.mean([10 * math.log10(1 + m / mse_ref) for m in mses]))
    log(f"quality: PSNR(ours, full) mean {np.mean(ps):.2f} dB min {np.min(ps):.2f}; loss {delta_db:.3f} dB; "
        f"SSIM(ours, full) mean {np.mean(ss):.4f} min {np.min(ss):.4f}; "
        f"keys dom {np.mean(keys_dom):.3g} roi {np.mean(keys_roi):.3g}; roi tiles {np.mean(roi_tiles):.0f}/{n_tiles}")

    ctx.set_count_pairs(True)
    pe_dom, pu_dom, pe_roi, pu_roi, work_dom, work_roi = [], [], [], [], [], []
    for cd, ca in zip(cams, affs):
        out = ctx.render_stereo(ds, cd, ca, raster, roi, out=out)
        st = out["stats"]
        pe_dom.append(st["pairs_eval_dom"])
        pu_dom.append(st["pairs_used_dom"])
        pe_roi.append(st["pairs_eval_roi"])
        pu_roi.append(st["pairs_used_roi"])
        work_dom.append(st["blend_work_dom"])
        work_roi.append(st["blend_work_roi"])
    ctx.set_count_pairs(False)
    wd, wr = np.mean(work_dom, axis=0), np.mean(work_roi, axis=0)
    log(f"blend work dom: walked {wd[0]:.3g} tested {wd[1]:.3g} lane-eff {np.mean(pe_dom) / max(wd[1], 1) / 64:.3f} "
        f"max wave walk {wd[2]:.0f} max list {wd[3]:.0f}; roi: walked {wr[0]:.3g} tested {wr[1]:.3g} "
        f"max wave walk {wr[2]:.0f} max list {wr[3]:.0f}")

    # ---- timed: ours ----
    ctx.set_sync(False)
    n_poses = len(cams)
    for i in range(args.warmup):
        ctx.render_stereo(ds, cams[i % n_poses], affs[i % n_poses], raster, roi, out=out)
    torch.cuda.synchronize()
    # Frames are issued back to back (they are independent): throughput is
    # steps / wall time with the host never waiting on the GPU; each frame's
    # latency is its GPU time between events recorded on its stream around it.
    # Only the dominant-eye blend is timed by the library's stage events here
    # (two event records per frame); the per-stage breakdown comes from a
    # separate pass below, so its events do not slow the timed frames.
    ctx.set_timing(True, stages=["blend_dom"])
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev0[i].record()
        ctx.render_stereo(ds, cams[i % n_poses], affs[i % n_poses], raster, roi, out=out)
        ev1[i].record()
    torch.cuda.synchronize()
    t_ours = time.perf_counter() - t_start
    lat = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    blend_live = ctx.timing_collect()["blend_dom"]
    ctx.set_timing(False)
    status = ctx.poll_status()
    assert status["overflow"] == 0, f"capacity overflow during timing: {status}"

    # ---- timed: sequential two-pass render (no stage events at all) ----
    fo = full
    fd = ctx.render_dominant(ds, cams[0], raster)
    for i in range(args.warmup):
        ctx.render_dominant(ds, cams[i % n_poses], raster, out=fd)
        ctx.render_dominant(ds, affs[i % n_poses], raster, out=fo)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev0[i].record()
        ctx.render_dominant(ds, cams[i % n_poses], raster, out=fd)
        ctx.render_dominant(ds, affs[i % n_poses], raster, out=fo)
        ev1[i].record()
    torch.cuda.synchronize()
    t_two = time.perf_counter() - t_start
    lat2 = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    status = ctx.poll_status()
    assert status["overflow"] == 0, f"capacity overflow during two-pass timing: {status}"

    # ---- timed: throughput with frames in flight on several streams ----
    # Frames are independent, so a serving loop keeps several in flight: K
    # contexts (own workspace, own default-priority stream), frame i on
    # context i mod K.  The two-pass baseline is run the same way.
    K = max(1, args.inflight)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(K - 1)]
    ctxs, outs, fds, fos = [ctx], [out], [fd], [fo]
    for k in range(1, K):
        with torch.cuda.stream(streams[k]):
            c = api.Context(sync=True)
            c.reserve(scene.n, cams[0].width, cams[0].height, int(kmax * 1.25) + 4096)
            o = c.render_stereo(ds, cams[0], affs[0], raster, roi)
            ctxs.append(c)
            outs.append(o)
            fds.append(c.render_dominant(ds, cams[0], raster))
            fos.append(c.render_dominant(ds, affs[0], raster))
            c.set_sync(False)
    split = tuple(int(x) for x in args.inflight_split.split(","))
    for c in ctxs:
        c.set_blend_split(*split)
    torch.cuda.synchronize()

    def inflight_ours(n0, n):
        for i in range(n0, n0 + n):
            k = i % K
            with torch.cuda.stream(streams[k]):
                ctxs[k].render_stereo(ds, cams[i % n_poses], affs[i % n_poses], raster, roi, out=outs[k])

    def inflight_two(n0, n):
        for i in range(n0, n0 + n):
            k = i % K
            with torch.cuda.stream(streams[k]):
                ctxs[k].render_dominant(ds, cams[i % n_poses], raster, out=fds[k])
                ctxs[k].render_dominant(ds, affs[i % n_poses], raster, out=fos[k])

    inflight_ours(0, args.warmup)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    inflight_ours(0, args.steps)
    torch.cuda.synchronize()
    t_ours_k = time.perf_counter() - t_start
    inflight_two(0, args.warmup)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    inflight_two(0, args.steps)
    torch.cuda.synchronize()
    t_two_k = time.perf_counter() - t_start
    for c in ctxs:
        status = c.poll_status()
        assert status["overflow"] == 0, f"capacity overflow during the in-flight timing: {status}"
    ctx.set_blend_split()  # back to the library's default for the stage breakdown

    # ---- per-stage breakdown (every stage timed; not part of the rates) ----
    n_stage = max(20, min(args.steps, 64))
    ctx.set_timing(True)
    for i in range(n_stage):
        ctx.render_stereo(ds, cams[i % n_poses], affs[i % n_poses], raster, roi, out=out)
    torch.cuda.synchronize()
    stages = ctx.timing_collect()
    ctx.set_timing(True)
    for i in range(n_stage):
        ctx.render_dominant(ds, cams[i % n_poses], raster, out=fd)
        ctx.render_dominant(ds, affs[i % n_poses], raster, out=fo)
    torch.cuda.synchronize()
    stages2 = ctx.timing_collect()
    ctx.set_timing(False)

    fps = args.steps / t_ours
    fps2 = args.steps / t_two
    fps_k = args.steps / t_ours_k
    fps2_k = args.steps / t_two_k
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    log("stage ms/frame (ours): " + ", ".join(f"{k}={v:.3f}" for k, v in stage_ms.items()))
    log(f"one frame at a time: ours {fps:.1f} fps p50 {pct(lat, 50):.3f} p99 {pct(lat, 99):.3f} ms; two-pass "
        f"{fps2:.1f} fps p99 {pct(lat2, 99):.3f} ms; reduction {1 - t_ours / t_two:.3f}")
    log(f"{K} frames in flight: ours {fps_k:.1f} fps; two-pass {fps2_k:.1f} fps; reduction {1 - t_ours_k / t_two_k:.3f}")

    # ---- roofline of the dominant kernel (the dominant-eye blend) ----
    blend_ms = blend_live[0] / max(blend_live[1], 1)
    flops = float(np.mean(pe_dom)) * FLOPS_EVAL + float(np.mean(pu_dom)) * FLOPS_USED
    achieved = flops / (blend_ms * 1e-3) / 1e12
    dominant = max(stage_ms, key=lambda k: stage_ms[k])
    roofline = {"kernel": "k_blend (dominant eye)", "bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": blend_traffic() if args.workload == "sphere800" else None, "avg_launch_ms": round(blend_ms, 4),
                "pairs_evaluated_per_launch": int(np.mean(pe_dom)),
                "pairs_contributing_per_launch": int(np.mean(pu_dom)),
                "records_walked_per_launch": int(wd[0]), "records_tested_per_launch": int(wd[1]),
                "longest_wave_walk": int(wd[2]), "longest_tile_list": int(wd[3]),
                "largest_stage": dominant}

    # ---- HBM efficiency of the sort and reprojection stages (algorithmic
    # bytes: one read and one write of every key and value for a sort, 4 B
    # each way when a tile key and its surfel share one word; the 20 B read
    # (colour, depth proxy, alpha) + 21 B written (colour, z, alpha, hole
    # mask) per pixel of a forward warp) ----
    def hbm(stage, nbytes):
        ms = stage_ms[stage]
        gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        return {"stage": stage, "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_launch": int(nbytes), "avg_ms": round(ms, 4)}

    npx = cams[0].width * cams[0].height
    bits = lambda x: max(1, int(math.ceil(math.log2(max(x, 2)))))
    key_b = 8.0 if bits(n_tiles) + bits(scene.n) <= 32 else 16.0
    hbm_stages = [hbm("tile_sort_dom", key_b * np.mean(keys_dom)), hbm("depth_sort_dom", 16.0 * scene.n),
                  hbm("tile_sort_roi", key_b * np.mean(keys_roi)), hbm("reproject", 41.0 * npx)]

    # ---- CPU oracle on a bounded sample (a baseline only) ----
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, scene, cams[0], affs[0], float(np.mean(roi_tiles)) * 256.0)

    result = {
        "metric": "stereo frames/sec + p99 ms/frame on 1 MI355X vs two-pass render at <=1.3dB PSNR loss",
        "value": round(fps_k, 2),
        "unit": "stereo frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_ours_k / args.steps * 1e3, 4),
        # Latency of one frame: GPU time between events around it, frames
        # issued one stream at a time.
        "p50_ms": round(pct(lat, 50), 4),
        "p99_ms": round(pct(lat, 99), 4),
        "inflight": K,
        "blend_split": {"inflight": list(split), "one_frame_at_a_time": "library default"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload] + (f" (surfel count set to {scene.n})" if args.surfels > 0
                                                               else ""),
                   "surfels": int(scene.n),
                   "width": int(cams[0].width), "height": int(cams[0].height), "poses": n_poses,
                   "sh_degree": int(scene.sh_degree), "baseline": baseline, "center_roi": bool(args.center_roi),
                   "margin": roi.margin, "edge_bounds": roi.edge_bounds, "tile": 16, "parallelism": "single GPU"},
        "two_pass": {"value": round(fps2_k, 2), "unit": "stereo frames/s",
                     "ms_per_step": round(t_two_k / args.steps * 1e3, 4),
                     "p50_ms": round(pct(lat2, 50), 4), "p99_ms": round(pct(lat2, 99), 4)},
        "time_reduction_vs_two_pass": round(1 - t_ours_k / t_two_k, 4),
        "one_frame_at_a_time": {"value": round(fps, 2), "two_pass_value": round(fps2, 2),
                                "ms_per_step": round(t_ours / args.steps * 1e3, 4),
                                "two_pass_ms_per_step": round(t_two / args.steps * 1e3, 4),
                                "time_reduction_vs_two_pass": round(1 - t_ours / t_two, 4)},
        "quality": {"psnr_ours_vs_full_db": round(float(np.mean(ps)), 3), "psnr_min_db": round(float(np.min(ps)), 3),
                    "psnr_loss_db": round(delta_db, 4), "p_ref_db": P_REF[args.workload],
                    "ssim_ours_vs_full": round(float(np.mean(ss)), 5), "ssim_min": round(float(np.min(ss)), 5)},
        "frame": {"keys_dom": int(np.mean(keys_dom)), "keys_roi": int(np.mean(keys_roi)),
                  "roi_tile_frac": round(float(np.mean(roi_tiles)) / n_tiles, 4), "boxes": float(np.mean(n_boxes))},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_ms_two_pass": {k: round(v[0] / v[1], 4) for k, v in stages2.items() if v[1]},
        "roofline": roofline,
        "hbm_stages": hbm_stages,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


def traffic_probe(args):
    """Kernels for HBM counter runs: three copies of a 512 MiB fp32 tensor
    (reads and writes of known size, to calibrate FETCH_SIZE/WRITE_SIZE), then
    12 dominant-eye renders of the workload with the library's default blend
    schedule."""
    import torch
    from paper_2609_30741_amd import api, synth

    a = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    scene, cams, _ = synth.WORKLOADS[args.workload](args.seed)
    ds = api.DeviceScene(scene)
    ctx = api.Context(sync=True)
    for c in cams[:4]:
        ctx.render_dominant(ds, c)
    ctx.set_sync(False)
    for c in cams[:8]:
        ctx.render_dominant(ds, c)
    torch.cuda.synchronize()
    log("traffic probe done")


def traffic_probe_stereo(args):
    """Kernels for per-kernel HBM counter runs over whole stereo frames: 16
    frames that size the workspace (synchronous), then 32 frames issued back
    to back, all at the library's default blend split."""
    import torch
    from paper_2609_30741_amd import api, synth

    scene, cams, baseline = synth.WORKLOADS[args.workload](args.seed)
    affs = [synth.affiliated(c, baseline) for c in cams]
    ds = api.DeviceScene(scene)
    ctx = api.Context(sync=True)
    out = None
    for cd, ca in zip(cams, affs):
        out = ctx.render_stereo(ds, cd, ca, out=out)
    ctx.set_sync(False)
    for _ in range(2):
        for cd, ca in zip(cams, affs):
            ctx.render_stereo(ds, cd, ca, out=out)
    torch.cuda.synchronize()
    log("stereo traffic probe done")


def blend_traffic():
    """HBM bytes per dominant-eye blend stage (all its launches) of the bench
    workload, from calibrated FETCH_SIZE and WRITE_SIZE counter runs of
    `bench.py --traffic-probe`; None when the blend kernels or the default
    blend schedule (raster.hip, bgs_api.hip) have changed since the counters
    were taken."""
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2609_30741_amd", "csrc")
    h = hashlib.sha1()
    for f in ("raster.hip", "bgs_api.hip"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return BLEND_TRAFFIC["bytes"] if h.hexdigest() == BLEND_TRAFFIC["source_sha1"] else None


def cpu_baseline(args, scene, cam_dom, cam_aff, roi_px):
    """Time the CPU oracle on a bounded sample of the workload and scale it to
    stereo frames/s: per-pixel rendering rate from a random sample of
    dominant-eye pixels, plus the oracle's reprojection and classification
    on full-size stand-in images (seeded, same size)."""
    from oracle import oracle as O
    from paper_2609_30741_amd import synth

    O.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    W, H = cam_dom.width, cam_dom.height
    rng = np.random.default_rng(11)
    n = 256
    spent = 0.0
    px_total = 0
    while spent < args.cpu_seconds * 0.8:
        pix = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], axis=1).astype(np.int32)
        t = time.perf_counter()
        O.render(scene, cam_dom, pixels=pix, nthreads=threads)
        spent += time.perf_counter() - t
        px_total += n
        n = min(n * 2, 1 << 16)
    rate = px_total / spent
    rgb, dr, a = synth.stage_images(W, H, 0)
    t = time.perf_counter()
    rep = O.reproject(cam_dom, cam_aff, rgb, dr, a)
    O.classify(cam_dom, cam_aff, O.Roi(center_roi=bool(args.center_roi)), rep["depth_range"], rep["rgb"], rep["z"],
               rep["alpha"], rep["hole"])
    t_rc = time.perf_counter() - t
    s_frame = (W * H + roi_px) / rate + t_rc
    log(f"cpu oracle: {rate:.0f} px/s on {threads} threads; reproject+classify {t_rc:.3f}s; {s_frame:.1f} s/frame")
    return {"value": round(1.0 / s_frame, 6), "unit": "stereo frames/s", "cores": threads, "kind": "oracle",
            "sample": f"{px_total} random dominant-eye pixels rendered by the fp64 oracle ({spent:.1f}s, "
                      f"{rate:.0f} px/s) scaled to {W * H} + {int(roi_px)} ROI pixels per frame, plus the oracle's "
                      f"reprojection and classification on full-size seeded stand-in images ({t_rc:.2f}s)",
            "seconds_per_frame": round(s_frame, 3)}


if __name__ == "__main__":
    main()
