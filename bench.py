"""Benchmark: stereo frames/s of the bricked multiresolution ray caster.

Workload (the bricked stereo configuration): a 2048^3 uint16 volume of 400
branching Gaussian tubes over Poisson(200) background, bricked 64^3 with a
one-voxel apron, 6 LOD levels, all 37,449 bricks resident in HBM; a stereo
pair of 1440x1600 per eye (64 mm inter-pupillary distance with the volume's
longest edge = 1 m, head 1.25 m from the centre), step 0.5 voxel of the
selected level, screen-space LOD at 1 pixel, early termination at 0.99,
empty-brick skipping. Inputs are synthetic and seeded.

One step = one sg_render_views call covering both eyes (LOD cut map and ray
casting for every pixel), with the volume already resident in HBM. The
pyramid build, apron fill and transfer-function refresh are one-time per
volume / per transfer function and are timed separately (``setup_ms``).

Prints one JSON line. ``roofline`` covers the ray-casting kernel, timed
with HIP events around its launches; ``cpu_baseline`` is the FP64 oracle on
a random pixel subset of the same frame, on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "samples/s and stereo frames/s, plain vs learned-upsampler path at PSNR≥40 dB"
HBM_PEAK = 8.0e12            # bytes/s, MI355X HBM3E
FP32_PEAK = 157.3e12         # FLOP/s, MI355X FP32 vector (packed FMA)
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9  # VALU lane operations/s (non-packed)
FLOP_PER_SAMPLE = 31         # algorithmic FLOP of one single-channel sample (see flop_per_sample)


def pool_layout(args):
    """The sg_layout of the large volumes' slots."""
    from paper_1804_08197_amd import sg
    return sg.SG_LAYOUT_MICROBLOCK if args.layout == "microblock" else sg.SG_LAYOUT_LINEAR


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload_views():
    import gen
    c = np.array([1024.0, 1024.0, 1024.0])
    head = c + 2560.0 * gen.unit((1.0, 0.7, 0.4))
    ipd = 131.072
    t = math.tan(math.radians(50.0))
    return gen.stereo(head, c, ipd, 1440, 1600, t, 0.9 * t)


PARAMS = {"step": 0.5, "ert": 0.99, "tau": 1.0, "lod": 1, "skip_empty": 1, "bias": 0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--render-only", action="store_true",
                    help="profiling: only warm-up and timed renders (no counting pass, no "
                         "oracle), one line of timings")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="profiling: run a plain device-to-device copy of this many bytes "
                         "3 times (calibrates the HBM byte counters) and exit")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch configuration (no autotuning in set-up)")
    ap.add_argument("--launch", default=None,
                    help="explicit launch configuration kernel,tile,block,stage_bytes,persistent "
                         "(no autotuning); profiles use the one the benchmark chose")
    ap.add_argument("--workload", default="tubes",
                    choices=("tubes", "batched64", "upsampler", "stream", "hmd", "octants",
                             "blobs256", "cells"),
                    help="tubes: the bricked stereo frame (default, the headline); "
                         "blobs256: the plain 256x256 frame of the 128^3 blob volume; "
                         "cells: one resident timepoint of the 3-channel cell series; "
                         "batched64: 64 uneven views of the 128^3 blob volume in one call; "
                         "upsampler: learned-upsampler path vs plain path on the blob scene; "
                         "stream: the 3-channel cell time series played through the "
                         "out-of-core brick cache; hmd: the bricked stereo frame under each "
                         "HMD variant (optical models, lens, clipping, depth limit)")
    ap.add_argument("--stream-timepoints", type=int, default=6,
                    help="stream: timepoints held in the host tier (the movie loops over them)")
    ap.add_argument("--stream-slots", type=int, default=10000,
                    help="stream: GPU cache capacity in bricks (one timepoint has 7,023)")
    ap.add_argument("--train-pairs", type=int, default=20000,
                    help="upsampler: training pairs (random pose and window each)")
    ap.add_argument("--eval-frames", type=int, default=1000,
                    help="upsampler: held-out stereo frames evaluated")
    ap.add_argument("--scene", default="blobs", choices=("blobs", "tubes"),
                    help="upsampler: the 128^3 blob scene (default) or the 2048^3 tube "
                         "volume with the screen-space LOD")
    ap.add_argument("--layout", default="microblock", choices=("microblock", "linear"),
                    help="pool slot layout of the 2048^3 tube and 3-channel cell volumes "
                         "(the 128^3 blob volumes keep linear slots, which the gather "
                         "kernel reads with fewer instructions)")
    ap.add_argument("--no-extras", action="store_true",
                    help="tubes: leave out the further figures the default run adds to its "
                         "line (HMD variants, octant share, upsampler, blobs256, cells, "
                         "batched64, stream)")
    args = ap.parse_args()
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    if args.gpus != 1:
        print("bench.py: the renderer runs on one GPU only (multi-GPU sort-last compositing is "
              "a design, not an implementation); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    if args.workload == "batched64":
        bench_batched(args)
        return
    if args.workload == "upsampler":
        bench_upsampler(args)
        return
    if args.workload == "stream":
        bench_stream(args)
        return
    if args.workload == "hmd":
        bench_hmd(args)
        return
    if args.workload == "octants":
        bench_octants(args)
        return
    if args.workload == "blobs256":
        print(json.dumps(run_blobs256(args, args.cpu_seconds > 0)), flush=True)
        return
    if args.workload == "cells":
        r = run_cells(args, args.cpu_seconds > 0 and not args.render_only)
        if r is not None:
            print(json.dumps(r), flush=True)
        return

    import gen
    from gen.large import TubeVolume, upload_generated
    from paper_1804_08197_amd import sg

    dims, B, levels = gen.TUBES_DIMS, gen.TUBES_BRICK, gen.TUBES_LEVELS
    want_cpu = args.cpu_seconds > 0 and not args.render_only

    t0 = time.time()
    tv = TubeVolume().to_device()
    log("geometry: %d segments in %.1fs" % (tv.n_segments, time.time() - t0))
    h = sg.sg_volume_create(dims, channels=1, dtype=sg.SG_U16, brick=B, levels=levels,
                            layout=pool_layout(args))
    host = np.empty(dims[::-1], dtype=np.uint16) if want_cpu else None
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    upload_generated(h, tv, B, host_out=host, slab_bricks=2, build_lod=False)
    ev[1].record()
    sg.sg_build_lod(h, 0, 0)
    ev[2].record()
    tf = gen.tf_hot()
    sg.sg_set_transfer_function(h, 0, tf, *gen.TUBE_DOMAIN)
    sg.sg_volume_commit(h)
    ev[3].record()
    torch.cuda.synchronize()
    setup = {"generate_upload_ms": ev[0].elapsed_time(ev[1]),
             "build_lod_ms": ev[1].elapsed_time(ev[2]),
             "commit_apron_range_empty_ms": ev[2].elapsed_time(ev[3])}
    log("setup: %s" % json.dumps({k: round(v, 1) for k, v in setup.items()}))

    views = workload_views()
    outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
    npix = sum(v["width"] * v["height"] for v in views)
    launch = sg.sg_get_launch_config(h)
    if args.launch:
        launch = dict(zip(sg.LAUNCH_FIELDS, (int(x) for x in args.launch.split(","))))
        sg.sg_set_launch_config(h, launch)
    elif not args.no_autotune:
        # set-up, untimed: pick the launch configuration on this frame (every
        # configuration renders the same image)
        launch, tuned_ms = sg.sg_autotune(h, views, PARAMS, outs, repeats=5)
        log("autotuned launch %s (%.3f ms)" % (launch, tuned_ms))

    if args.render_only:
        for _ in range(args.warmup):
            sg.sg_render_views(h, views, PARAMS, outs)
        torch.cuda.synchronize()
        sg.sg_set_kernel_timing(h, True)
        for _ in range(args.steps):
            sg.sg_render_views(h, views, PARAMS, outs)
        n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
        print(json.dumps({"renders": n_k, "raycast_kernel_ms": ray_ms / n_k,
                          "cutmap_kernel_ms": cut_ms / n_k}), flush=True)
        sg.sg_volume_destroy(h)
        return

    # counting pass (untimed): samples and distinct 4^3 micro-blocks read
    stats = sg.sg_render_views_stats(h, views, PARAMS, outs)
    samples = stats["total_samples"]
    mb = stats["microblocks"]
    log("samples/frame %d, microblocks %d" % (samples, mb))
    # brick-granular bytes: the non-empty nodes of both views' cuts (the
    # bricks the frame may read, whole, core plus apron)
    cut = set()
    for v in views:
        nodes, empty = sg.sg_get_lod_cut(h, v, PARAMS)
        cut |= set(nodes[~empty].tolist())
    brick_bytes = len(cut) * (B + 2) ** 3 * 2

    for _ in range(args.warmup):
        sg.sg_render_views(h, views, PARAMS, outs)
    torch.cuda.synchronize()
    sg.sg_set_kernel_timing(h, True)
    # per-step HIP events on the stream the renders run on (torch's current
    # stream) give the distribution of step times
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_ev[0].record()
    for i in range(args.steps):
        sg.sg_render_views(h, views, PARAMS, outs)
        step_ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = np.array([step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(args.steps)])
    n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
    sg.sg_set_kernel_timing(h, False)
    assert n_k == args.steps
    ms_step = wall * 1e3 / args.steps
    fps = args.steps / wall
    ray_avg_s = ray_ms / n_k * 1e-3
    log("%.3f ms/step (wall), raycast kernel %.3f ms, cutmap %.4f ms" % (
        ms_step, ray_ms / n_k, cut_ms / n_k))

    traffic = measured_traffic()
    bytes_alg = mb * 64 * 2 + npix * 16
    flops_alg = samples * FLOP_PER_SAMPLE
    hbm = {"bound": "hbm", "achieved": bytes_alg / ray_avg_s / 1e9, "peak": HBM_PEAK / 1e9,
           "unit": "GB/s", "traffic": traffic}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    alu = {"bound": "alu", "achieved": flops_alg / ray_avg_s / 1e12, "peak": FP32_PEAK / 1e12,
           "unit": "TFLOP/s", "traffic": traffic}
    alu["frac"] = alu["achieved"] / alu["peak"]
    roof, other = (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)
    # the VALU lane-operation rate: samples x the measured lane operations
    # per sample (committed counter passes of this kernel) against 256 CUs x
    # 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane operations/s
    rec = profile_record()
    valu = None
    if rec and "valu_lane_ops_per_sample" in rec:
        lane_ops = samples * rec["valu_lane_ops_per_sample"] / ray_avg_s
        valu = {"bound": "valu", "achieved": lane_ops / 1e12, "peak": VALU_LANE_PEAK / 1e12,
                "unit": "T lane-ops/s", "frac": lane_ops / VALU_LANE_PEAK,
                "lane_ops_per_sample": rec["valu_lane_ops_per_sample"]}

    out = {"metric": METRIC, "value": fps, "unit": "stereo frames/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "tubes2048_u16_bricked_stereo_1440x1600",
                      "volume": "2048^3 uint16, 400 branching Gaussian tubes + Poisson(200)",
                      "brick": B, "levels": levels, "layout": args.layout, "views": 2,
                      "width": 1440, "height": 1600,
                      "step_voxels": 0.5, "ert": 0.99, "lod_tau_px": 1.0, "skip_empty": True},
           "samples_per_frame": samples, "samples_per_s": samples * fps,
           "raycast_kernel_ms": ray_ms / n_k, "cutmap_kernel_ms": cut_ms / n_k,
           "step_ms_median": float(np.median(step_ms)),
           "step_ms_p10": float(np.percentile(step_ms, 10)),
           "step_ms_p90": float(np.percentile(step_ms, 90)),
           "microblocks_per_frame": mb, "brick_bytes_per_frame": brick_bytes,
           "cut_nonempty_nodes": len(cut), "roofline": roof, "roofline_other": other,
           "roofline_valu": valu,
           "launch": launch, "setup_ms": setup,
           # instrumented pass of the same frame (staged kernel only)
           "kernel_stats": {
               "node_visits": stats["node_visits"], "slabs": stats["slabs"],
               "staged_bytes": stats["staged_bytes"],
               "lanes_in_node": (stats["node_lanes"] / (64.0 * stats["node_visits"])
                                 if stats["node_visits"] else None),
               "lanes_in_flight": (stats["alive_lanes"] / (64.0 * stats["node_visits"])
                                   if stats["node_visits"] else None),
               "loop_lane_utilisation": (samples / (64.0 * stats["loop_iterations"])
                                         if stats["loop_iterations"] else None),
               "pool_samples": stats["pool_samples"], "slab_retries": stats["slab_retries"]}}

    if want_cpu:
        out["cpu_baseline"] = cpu_baseline(host, tf, views, npix, args.cpu_seconds)
    del host, tv, outs
    if not args.no_extras:
        # the workloads that reuse the resident tube volume, in the same launch
        short = argparse.Namespace(**dict(vars(args), steps=min(args.steps, 10),
                                          warmup=min(args.warmup, 2)))
        for key, fn in (("hmd_variants", lambda: hmd_summary(run_hmd(h, views, launch, short))),
                        ("octant_share", lambda: octant_summary(run_octants(h, views, launch,
                                                                           short)))):
            out[key] = guarded(key, fn)
    sg.sg_volume_destroy(h)
    if not args.no_extras:
        out.update(extras(args))
    print(json.dumps(out), flush=True)


def guarded(key, fn):
    """fn(), or its error as the figure: the headline line stands."""
    import gc

    import torch
    t0 = time.time()
    try:
        r = fn()
    except Exception as e:  # noqa: BLE001 -- reported in the line
        r = {"error": "%s: %s" % (type(e).__name__, e)}
    gc.collect()
    torch.cuda.empty_cache()
    log("%s done in %.1fs" % (key, time.time() - t0))
    return r


def hmd_summary(r):
    """The HMD variants' kernel times and samples for the headline line."""
    return {"workload": r["config"]["workload"], "launch": r["launch"],
            "variants": {k: {"raycast_kernel_ms": v["raycast_kernel_ms"],
                             "samples": v["samples"]} for k, v in r["variants"].items()}}


def octant_summary(r):
    """One GPU's octant share for the headline line."""
    return {"workload": r["config"]["workload"],
            "stereo_frames_per_s_slowest_octant": r["value"], "slowest": r["config"]["slowest"],
            "octant_kernel_ms": {k: v["raycast_kernel_ms"] for k, v in r["octants"].items()},
            "composite_ms_all_parts": r["composite_ms_all_parts"],
            "composite_max_diff_to_whole": r["composite_max_diff_to_whole"]}


def batched_summary(r):
    """The 64-view batch for the headline line."""
    keys = ("value", "unit", "ms_per_step", "views_per_s", "samples_per_batch",
            "default_launch_ms", "autotuned_launch", "autotuned_ms", "graph_replay_ms",
            "raycast_kernel_ms", "roofline")
    return dict({"workload": r["config"]["workload"]}, **{k: r[k] for k in keys})


def stream_summary(r):
    """The time series through the brick cache for the headline line."""
    keys = ("value", "unit", "ms_per_step", "frames_per_timepoint",
            "stereo_frames_per_s_during_playback", "bricks_uploaded_per_timepoint",
            "upload_GB_per_s", "core_voxels_streamed_per_s", "host_to_device_copy_GB_per_s",
            "resident_frame_ms", "resident_samples_per_frame", "evictions")
    return dict({"workload": r["config"]["workload"],
                 "timepoints_in_host_tier": r["config"]["timepoints_in_host_tier"]},
                **{k: r[k] for k in keys})


def extras(args):
    """The default run's further figures, each on its own volume: the
    learned-upsampler path against the plain path (blob scene), the plain
    256x256 blob frame, one resident timepoint of the cell series, the
    64-view batch, and the cell series played through the brick cache (three
    timepoints in the host tier, ten played). A figure that fails is
    reported as its error; the headline stands."""
    short = argparse.Namespace(**dict(vars(args), steps=min(args.steps, 10),
                                      warmup=min(args.warmup, 2),
                                      stream_timepoints=min(args.stream_timepoints, 3)))
    return {key: guarded(key, fn) for key, fn in (
        ("upsampler", lambda: upsampler_summary(run_upsampler(args))),
        ("blobs256", lambda: run_blobs256(args, args.cpu_seconds > 0)),
        ("cells_timepoint", lambda: run_cells(args, args.cpu_seconds > 0)),
        ("batched64", lambda: batched_summary(run_batched(short))),
        ("stream", lambda: stream_summary(run_stream(short))))}


def upsampler_summary(r):
    """The upsampler path's keys for the headline line."""
    return {"workload": r["config"]["workload"], "plain_ms": r["plain_ms"],
            "up_ms": r["upsampler_path_ms"], "speedup": r["speedup_vs_plain"],
            "psnr_mean": r["psnr_upsampled_mean"], "psnr_min": r["psnr_upsampled_min"],
            "bilinear_psnr": r["psnr_bilinear_mean"], "fallback_rate": r["fallback_rate"],
            "frames": r["config"]["eval_frames"], "timed_frames": r["steps"],
            "timed_fallbacks": r["timed_fallbacks"], "delivered_min_psnr": r["delivered_min_psnr"],
            "fallback_threshold_db": r["fallback_threshold_db"], "network_ms": r["network_ms"],
            "network_flag_ms": r["network_flag_ms"],
            "network_mask_built_ms": r["network_mask_built_ms"],
            "train_pairs": r["config"]["train_pairs"],
            "train_seconds": r["train_seconds"], "roofline": r["roofline"]}


def timed_events(fn, steps, warmup):
    """Mean milliseconds of fn over steps calls after warmup calls, from HIP
    events on torch's current stream (the stream the renders run on)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        fn()
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / steps


def rooflines(samples, flop, bytes_alg, kernel_s):
    """(dominant, other) of the FP32 ALU and HBM rooflines of one launch."""
    alu = {"bound": "alu", "achieved": samples * flop / kernel_s / 1e12,
           "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s", "traffic": None}
    hbm = {"bound": "hbm", "achieved": bytes_alg / kernel_s / 1e9, "peak": HBM_PEAK / 1e9,
           "unit": "GB/s", "traffic": None}
    for r in (alu, hbm):
        r["frac"] = r["achieved"] / r["peak"]
    return (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)


def run_blobs256(args, want_cpu):
    """The plain unbricked frame: the 128^3 uint8 blob volume as one brick
    and one level, one 256x256 view (60 degree field of view, eye 2.5
    volume diagonals from the centre), identity ramp over [0, 255], step
    0.5 voxel, early termination at 0.99. A frame is tens of microseconds
    of ray casting, so the figure is launch-bound; it is timed eager and as
    a replayed render graph, and the oracle renders the whole frame."""
    import torch

    import gen
    from paper_1804_08197_amd import sg, upload_volume
    vol = gen.blobs128()
    h = sg.sg_volume_create((128, 128, 128), dtype=sg.SG_U8, brick=128, levels=1)
    upload_volume(h, torch.from_numpy(vol).cuda(), 128)
    tf = gen.tf_identity()
    sg.sg_set_transfer_function(h, 0, tf, 0, 255)
    sg.sg_volume_commit(h)
    views = [gen.blobs128_view()]
    params = {"step": 0.5, "ert": 0.99, "lod": 0, "bias": 0, "skip_empty": 1}
    outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
    npix = sum(v["width"] * v["height"] for v in views)
    launch, _ = sg.sg_autotune(h, views, params, outs, repeats=3)
    stats = sg.sg_render_views_stats(h, views, params, outs)
    samples, mb = stats["total_samples"], stats["microblocks"]
    R = 500
    eager_ms = timed_events(lambda: sg.sg_render_views(h, views, params, outs), R, 20)
    g = sg.RenderGraph(h, views, params, outs)
    graph_ms = timed_events(g.launch, R, 20)
    g.destroy()
    sg.sg_set_kernel_timing(h, True)
    for _ in range(R):
        sg.sg_render_views(h, views, params, outs)
    n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
    sg.sg_set_kernel_timing(h, False)
    ray_s = ray_ms / n_k * 1e-3
    best_ms = min(eager_ms, graph_ms)
    roof, other = rooflines(samples, FLOP_PER_SAMPLE, mb * 64 + npix * 16, ray_s)
    out = {"metric": "frames/s of the plain 256x256 blob frame", "value": 1e3 / best_ms,
           "unit": "frames/s", "n_gpus": 1, "steps": R, "warmup": 20, "ms_per_step": best_ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "blobs128_u8_mono_256x256", "brick": 128, "levels": 1,
                      "step_voxels": 0.5, "ert": 0.99},
           "samples_per_frame": samples, "samples_per_s": samples / (best_ms * 1e-3),
           "eager_ms": eager_ms, "graph_replay_ms": graph_ms,
           "raycast_kernel_ms": ray_ms / n_k, "cutmap_kernel_ms": cut_ms / n_k,
           "microblocks_per_frame": mb, "launch": launch, "roofline": roof,
           "roofline_other": other}
    sg.sg_volume_destroy(h)
    if want_cpu:
        import oracle
        sc = oracle.Scene([vol], 128, 1, [np.asarray(tf, np.float64)], [(0, 255)])
        out["cpu_baseline"] = oracle_whole_frame(sc, views, params, "frames/s")
    return out


def run_cells(args, want_cpu):
    """One timepoint of the 3-channel cell series resident in HBM: 3 x
    1024x1024x512 uint16 (timepoint 0), bricked 64^3 with a one-voxel
    apron, 5 levels, each channel with its own tinted table, additive
    channel blending, stereo 1440x1600 per eye, step 0.5 voxel of the
    selected level, screen-space LOD at 1 pixel, early termination 0.99,
    empty skipping. One step = one sg_render_views call for both eyes."""
    import torch

    import gen
    from gen.large import CellVolume, upload_generated
    from paper_1804_08197_amd import sg
    dims, B, L, C = gen.CELLS_DIMS, gen.CELLS_BRICK, gen.CELLS_LEVELS, 3
    h = sg.sg_volume_create(dims, channels=C, timepoints=1, dtype=sg.SG_U16, brick=B, levels=L,
                            layout=pool_layout(args))
    hosts = []
    t0 = time.time()
    for c in range(C):
        cv = CellVolume(c, 0).to_device()
        host = np.empty(dims[::-1], dtype=np.uint16) if want_cpu else None
        upload_generated(h, cv, B, channel=c, timepoint=0, host_out=host, slab_bricks=4)
        hosts.append(host)
        del cv
    tfs = [gen.tf_tint(tint) for tint in gen.CELL_TINTS]
    for c in range(C):
        sg.sg_set_transfer_function(h, c, tfs[c], *gen.CELL_DOMAIN)
    sg.sg_volume_commit(h)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    views = gen.cells_stereo()
    params = dict(PARAMS)
    outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
    npix = sum(v["width"] * v["height"] for v in views)
    if args.launch:
        launch = dict(zip(sg.LAUNCH_FIELDS, (int(x) for x in args.launch.split(","))))
        sg.sg_set_launch_config(h, launch)
    else:
        launch, _ = sg.sg_autotune(h, views, params, outs, repeats=5)
    if args.render_only:
        for _ in range(args.warmup):
            sg.sg_render_views(h, views, params, outs)
        torch.cuda.synchronize()
        sg.sg_set_kernel_timing(h, True)
        for _ in range(args.steps):
            sg.sg_render_views(h, views, params, outs)
        n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
        print(json.dumps({"renders": n_k, "raycast_kernel_ms": ray_ms / n_k,
                          "cutmap_kernel_ms": cut_ms / n_k}), flush=True)
        sg.sg_volume_destroy(h)
        return None
    stats = sg.sg_render_views_stats(h, views, params, outs)
    samples, mb = stats["total_samples"], stats["microblocks"]
    steps = max(args.steps, 10)
    torch.cuda.synchronize()
    sg.sg_set_kernel_timing(h, True)
    ms = timed_events(lambda: sg.sg_render_views(h, views, params, outs), steps, args.warmup)
    n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
    sg.sg_set_kernel_timing(h, False)
    # the kernel timer also saw the warm-up calls: they render the same frame
    ray_s = ray_ms / n_k * 1e-3
    roof, other = rooflines(samples, flop_per_sample(C), mb * 64 * 2 + npix * 16, ray_s)
    out = {"metric": "stereo frames/s of one resident timepoint of the 3-channel series",
           "value": 1e3 / ms, "unit": "stereo frames/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "cells_3x1024x1024x512_u16_resident_timepoint_stereo_1440x1600",
                      "channels": C, "brick": B, "levels": L, "layout": args.layout,
                      "step_voxels": 0.5, "ert": 0.99, "lod_tau_px": 1.0, "skip_empty": True},
           "samples_per_frame": samples, "samples_per_s": samples * 1e3 / ms,
           "raycast_kernel_ms": ray_ms / n_k, "cutmap_kernel_ms": cut_ms / n_k,
           "microblocks_per_frame": mb, "launch": launch, "roofline": roof,
           "roofline_other": other, "setup_generate_upload_s": setup_s,
           "paper_context": "3D movies of up to 2e7 voxels per volume frame play at 25 volume "
                            "frames/s (Sec 5.4; hardware not stated)"}
    sg.sg_volume_destroy(h)
    if want_cpu:
        import oracle
        sc = oracle.Scene(hosts, B, L, [np.asarray(t, np.float32).astype(np.float64) for t in tfs],
                          [gen.CELL_DOMAIN] * C)
        out["cpu_baseline"] = oracle_pixel_subset(sc, views, params, npix, args.cpu_seconds,
                                                  "stereo frames/s")
    return out


def batched_views():
    """64 views of the 128^3 blob volume: sizes uniform in 512..2048 per
    axis, eyes on a sphere of 1.5..4 volume diagonals, 60 degree vertical
    field of view (seeded)."""
    import gen
    diag = 128 * math.sqrt(3.0)
    return gen.orbit_views((64.0, 64.0, 64.0), (1.5 * diag, 4.0 * diag), 64, 1004,
                           (512, 2048), (512, 2048), tan_top=math.tan(math.radians(30)))


def bench_batched(args):
    print(json.dumps(run_batched(args)), flush=True)


def run_batched(args):
    """64 uneven views in one call: default launch, autotuned launch, and the
    autotuned launch replayed as a render graph."""
    import torch

    import gen
    from paper_1804_08197_amd import sg, upload_volume
    vol = gen.blobs128()
    h = sg.sg_volume_create((128, 128, 128), dtype=sg.SG_U8, brick=128, levels=1)
    upload_volume(h, torch.from_numpy(vol).cuda(), 128)
    sg.sg_set_transfer_function(h, 0, gen.tf_identity(), 0, 255)
    views = batched_views()
    params = {"step": 0.5, "ert": 0.99, "lod": 0, "skip_empty": 1}
    outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
    npix = sum(v["width"] * v["height"] for v in views)
    stats = sg.sg_render_views_stats(h, views, params, outs)
    samples = stats["total_samples"]
    log("batched64: %d views, %.1f Mpx, %d samples" % (len(views), npix / 1e6, samples))

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(steps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    sg.sg_set_launch_config(h, None)
    default_ms = timed(lambda: sg.sg_render_views(h, views, params, outs), args.steps)
    t0 = time.time()
    cfg, tuned_ms = sg.sg_autotune(h, views, params, outs, repeats=2)
    log("autotune: %s %.3f ms (%.1fs)" % (cfg, tuned_ms, time.time() - t0))
    eager_ms = timed(lambda: sg.sg_render_views(h, views, params, outs), args.steps)
    g = sg.RenderGraph(h, views, params, outs)
    graph_ms = timed(g.launch, args.steps)
    g.destroy()
    sg.sg_set_kernel_timing(h, True)
    for _ in range(args.steps):
        sg.sg_render_views(h, views, params, outs)
    n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
    sg.sg_set_kernel_timing(h, False)
    ray_avg_s = ray_ms / n_k * 1e-3
    best_ms = min(eager_ms, graph_ms)
    alu = {"bound": "alu", "achieved": samples * FLOP_PER_SAMPLE / ray_avg_s / 1e12,
           "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s", "traffic": None}
    alu["frac"] = alu["achieved"] / alu["peak"]
    out = {"metric": "samples/s of a 64-view uneven batch in one call", "value": samples / (best_ms * 1e-3),
           "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": best_ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "blobs128_u8_64_uneven_views", "views": len(views),
                      "megapixels": npix / 1e6, "step_voxels": 0.5, "ert": 0.99},
           "views_per_s": len(views) / (best_ms * 1e-3), "samples_per_batch": samples,
           "default_launch_ms": default_ms, "autotuned_launch": cfg, "autotuned_ms": eager_ms,
           "graph_replay_ms": graph_ms, "raycast_kernel_ms": ray_ms / n_k, "roofline": alu}
    sg.sg_volume_destroy(h)
    return out


def upsampler_scene(args):
    """The volume and poses of the upsampler workload. blobs (the default):
    the 128^3 u8 blob volume with two levels, no LOD (target on level 0,
    input on level 1), 60 degree vertical FOV, eyes at 1.5-4 diagonals, IPD
    8.192. tubes: the 2048^3 u16 tube volume with its 6 levels and the
    screen-space LOD at 1 pixel (target = the plain bricked stereo frame;
    the half-resolution input lands one level coarser by itself), the HMD
    frustum (half-FOV 50 degrees), heads at 0.9-1.5 m (1843-3072 voxels),
    IPD 131.072."""
    import torch

    import gen
    from paper_1804_08197_amd import sg, upload_volume
    if args.scene == "blobs":
        vol = gen.blobs128()
        h = sg.sg_volume_create((128, 128, 128), dtype=sg.SG_U8, brick=64, levels=2)
        upload_volume(h, torch.from_numpy(vol).cuda(), 64)
        sg.sg_set_transfer_function(h, 0, gen.tf_identity(), 0, 255)
        diag = 128 * math.sqrt(3.0)
        return {"h": h, "diag": diag, "center": (64.0, 64.0, 64.0),
                "radius": (1.5 * diag, 4.0 * diag), "tan": math.tan(math.radians(30)),
                "ipd": 8.192, "lod": False,
                "workload": "blobs128_u8_stereo_1440x1600_upsampler",
                "input": "720x800 per eye on level 1 with depth"}
    from gen.large import TubeVolume, upload_generated
    dims, B, levels = gen.TUBES_DIMS, gen.TUBES_BRICK, gen.TUBES_LEVELS
    tv = TubeVolume().to_device()
    h = sg.sg_volume_create(dims, channels=1, dtype=sg.SG_U16, brick=B, levels=levels,
                            layout=pool_layout(args))
    upload_generated(h, tv, B, slab_bricks=2, build_lod=False)
    sg.sg_build_lod(h, 0, 0)
    sg.sg_set_transfer_function(h, 0, gen.tf_hot(), *gen.TUBE_DOMAIN)
    sg.sg_volume_commit(h)
    torch.cuda.synchronize()
    return {"h": h, "diag": 2048 * math.sqrt(3.0), "center": (1024.0, 1024.0, 1024.0),
            "radius": (1843.2, 3072.0), "tan": math.tan(math.radians(50)), "ipd": 131.072,
            "lod": True, "workload": "tubes2048_u16_stereo_1440x1600_upsampler",
            "input": "720x800 per eye, screen-space LOD (one level coarser), with depth"}


def bench_upsampler(args):
    print(json.dumps(run_upsampler(args)), flush=True)


def run_upsampler(args):
    """A scene in stereo at 1440x1600 per eye: the plain full-resolution path
    against the learned-upsampler path (half-resolution render one level
    coarser with depth, network, fallback to the plain render when the
    predicted PSNR is below the threshold). Trains the network first on
    pairs the ray caster renders (seed 1005), calibrates the threshold on
    200 frames (seed 3005), evaluates on held-out frames (seed 2005)."""
    import torch

    import gen
    from paper_1804_08197_amd import sg
    from paper_1804_08197_amd import upsample as U
    from paper_1804_08197_amd import upsampler as up
    W, H = 1440, 1600
    t0 = time.time()
    sc = upsampler_scene(args)
    log("scene %s ready in %.1fs" % (args.scene, time.time() - t0))
    h, diag, center, radius, tan_t = sc["h"], sc["diag"], sc["center"], sc["radius"], sc["tan"]
    base = {"step": 0.5, "ert": 0.99, "skip_empty": 1, "tau": 1.0}

    # ---- training (set-up, timed separately)
    t0 = time.time()
    poses = gen.orbit_views(center, radius, args.train_pairs, 1005, W, H, tan_t)
    model = up.Upsampler(max(16 * 128 * 128, 2 * (H // 2) * (W // 2)))
    rng = np.random.default_rng(1005)
    model.set_weights(U.init_params(rng))
    tr = U.Trainer(h, model, diag, base, crop=256, batch=16, lod=sc["lod"])
    steps = max(1, 2 * args.train_pairs // 16)
    losses = []
    for i in range(steps):
        lr = 2e-3 * (0.5 * (1 + math.cos(math.pi * i / steps))) + 1e-5
        loss = tr.step(rng, poses, lr, 1.0, want_loss=(i % 100 == 0 or i == steps - 1))
        if loss is not None:
            losses.append(loss)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    log("trained %d steps (%d pairs per epoch, batch 16) in %.1fs, loss %.3e -> %.3e" % (
        steps, args.train_pairs, train_s, losses[0], losses[-1]))

    path = U.UpsampledPath(h, model, diag, base, W, H, 2, lod=sc["lod"])
    plain = torch.empty(2, H, W, 4, device="cuda")
    p_full = path.p_full
    # set-up, untimed: the launch configuration tuned on the plain path's
    # frame serves both paths (every configuration renders the same image)
    launch, _ = sg.sg_autotune(h, gen.orbit_views(center, radius, 1, 4005, W, H, tan_t,
                                                  stereo_ipd=sc["ipd"])[0], p_full, list(plain),
                               repeats=5)
    log("launch configuration: %s" % launch)
    # the upsampler path's own launches (set-up, untimed; images are the
    # same under every launch): the half-resolution render tuned on its own
    # frame; the gated full-resolution render with 32-pixel workgroup tiles
    # on a direct grid, whose few workgroups end at once when the frame
    # needs no fallback (a persistent grid would first reset its tile
    # queues, one more launch)
    hv = gen.orbit_views(center, radius, 1, 4005, W, H, tan_t, stereo_ipd=sc["ipd"])[0]
    launch_half, _ = sg.sg_autotune(h, path._half_views(hv), path.p_half, list(path.rgba_lo),
                                    repeats=5)
    launch_full = dict(launch, tile=32, block=max(32, launch["block"]), persistent=0)
    log("launch configuration: half %s, gated full %s" % (launch_half, launch_full))
    path.launch_half, path.launch_full = launch_half, launch_full
    launch_up = {"half": launch_half, "full_gated": launch_full}

    def frame_psnr(views):
        sg.sg_render_views(h, views, p_full, list(plain))
        pred = path.predicted_psnr(views)
        mse = float(((path.out[..., :3] - plain[..., :3]) ** 2).mean())
        return pred, (math.inf if mse == 0 else 10 * math.log10(1.0 / mse))

    # ---- calibration of the fallback threshold
    cal = gen.orbit_views(center, radius, 200, 3005, W, H, tan_t, stereo_ipd=sc["ipd"])
    pairs = [frame_psnr(v) for v in cal]
    # the prediction's worst overestimate on the calibration frames, plus a
    # 0.5 dB margin, on top of 40 dB: a frame predicted above the threshold
    # is expected to reach 40 dB
    over = max(0.0, max(p - a for p, a in pairs))
    thr = 40.0 + over + 0.5
    path.threshold_db = thr
    log("fallback threshold (predicted PSNR): %.2f dB" % thr)

    # ---- evaluation on held-out frames
    ev = gen.orbit_views(center, radius, args.eval_frames, 2005, W, H, tan_t,
                         stereo_ipd=sc["ipd"])
    res = [frame_psnr(v) for v in ev]
    actual = np.array([a for _, a in res])
    predicted = np.array([p for p, _ in res])
    accepted = predicted >= thr
    delivered = np.where(accepted, actual, np.inf)
    # bilinear baseline (network output zero): the half-resolution render upsampled
    zero = up.Upsampler(2 * (H // 2) * (W // 2))
    zero.set_weights(np.zeros(up.param_count(), np.float32))
    bl = []
    for v in ev[:200]:
        sg.sg_render_views(h, v, p_full, list(plain))
        sg.sg_render_views(h, [U.half_view(x) for x in v], path.p_half, list(path.rgba_lo),
                           list(path.depth_lo))
        zero.forward(path.rgba_lo, path.depth_lo, diag, path.out)
        mse = float(((path.out[..., :3] - plain[..., :3]) ** 2).mean())
        bl.append(10 * math.log10(1.0 / mse) if mse > 0 else math.inf)
    zero.close()

    # ---- timing: plain path and upsampler path over the held-out frames
    sub = ev[:min(len(ev), 200)]

    def run_plain():
        sg.sg_set_launch_config(h, launch)
        for v in sub:
            sg.sg_render_views(h, v, p_full, list(plain))

    def run_up_host():
        fell = 0
        for v in sub:
            fell += path.render(v)[1]
        return fell

    flags = torch.zeros(len(sub), dtype=torch.int32, device="cuda")
    flag_of = [flags[i:i + 1] for i in range(len(sub))]  # one device flag per frame

    def run_up():
        # the product path: the fallback decision stays on the device
        for v, f in zip(sub, flag_of):
            path.render_device(v, f)

    for fn in (run_plain, run_up_host, run_up):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    run_plain()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t) * 1e3 / len(sub)
    t = time.perf_counter()
    fell_host = run_up_host()
    torch.cuda.synchronize()
    up_host_ms = (time.perf_counter() - t) * 1e3 / len(sub)
    flags.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    run_up()
    torch.cuda.synchronize()
    up_ms = (time.perf_counter() - t) * 1e3 / len(sub)
    fell = int(flags.sum().item())
    # network alone on the last timed frame's input (no render, no host
    # read-back), driven by that render's content mask as the path runs it,
    # and with the mask built by the call itself
    net_ms = timed_events(lambda: model.forward(path.rgba_lo, path.depth_lo, diag, path.out,
                                                content=path.content), 50, 5)
    net_nomask_ms = timed_events(lambda: model.forward(path.rgba_lo, path.depth_lo, diag,
                                                       path.out), 50, 5)
    # the network as the device-decided path runs it, with the fallback decision
    flag1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    flag_ms = timed_events(lambda: model.forward_flag(path.rgba_lo, path.depth_lo, diag, path.out,
                                                      thr, flag1, content=path.content), 50, 5)
    # the network runs only on 16x16 input tiles with a nonzero input pixel
    # within its 4-pixel reach (empty tiles write background): the
    # algorithmic work counts the pixels of those tiles, at 2 x 9 x 32 x
    # (8 + 32 + 32 + 32) flop per input pixel
    nz = (path.rgba_lo != 0).any(-1) | torch.isfinite(path.depth_lo)
    run = torch.nn.functional.max_pool2d(nz.float().unsqueeze(1), 24, 16, 4, ceil_mode=True)
    tiles_run, tiles_all = int(run.sum().item()), run.numel()
    flops = tiles_run * 256 * 2 * 9 * 32 * (8 + 32 + 32 + 32)
    # HBM: the input (rgba + depth, 20 B per pixel) of the tiles that run the
    # network, four output pixels' rgba (64 B) for every input pixel, and
    # the content mask (one byte per 8 x 8 block)
    n_img = path.rgba_lo.shape[0]
    net_bytes = (tiles_run * 256 * 20 + n_img * (H // 2) * (W // 2) * 64
                 + path.content.numel())
    mfma = {"bound": "mfma", "achieved": flops / (net_ms * 1e-3) / 1e12, "peak": 2500.0,
            "unit": "TFLOP/s", "traffic": None}
    hbm = {"bound": "hbm", "achieved": net_bytes / (net_ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
           "unit": "GB/s", "traffic": None}
    for r in (mfma, hbm):
        r["frac"] = r["achieved"] / r["peak"]
    net_roof = (hbm, mfma) if hbm["frac"] >= mfma["frac"] else (mfma, hbm)
    out = {"metric": "stereo frames/s, plain vs learned-upsampler path at PSNR>=40 dB",
           "value": 1e3 / up_ms, "unit": "stereo frames/s", "n_gpus": 1,
           "steps": len(sub), "warmup": 1, "ms_per_step": up_ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16 network, f32 ray caster",
           "data": "synthetic",
           "config": {"workload": sc["workload"], "input": sc["input"],
                      "train_pairs": args.train_pairs, "train_steps": steps,
                      "eval_frames": len(ev)},
           "plain_ms": plain_ms, "plain_fps": 1e3 / plain_ms, "upsampler_path_ms": up_ms,
           "speedup_vs_plain": plain_ms / up_ms, "timed_fallbacks": fell, "launch": launch,
           "launch_upsampler_path": launch_up,
           "upsampler_path_host_decision_ms": up_host_ms,
           "timed_fallbacks_host_decision": int(fell_host),
           "network_ms": net_ms, "network_flag_ms": flag_ms,
           "network_mask_built_ms": net_nomask_ms,
           "network_tiles_run": tiles_run, "network_tiles": tiles_all,
           "network_tflops": flops / (net_ms * 1e-3) / 1e12,
           "roofline": net_roof[0], "roofline_other": net_roof[1],
           "psnr_upsampled_mean": float(np.mean(actual)),
           "psnr_upsampled_min": float(np.min(actual)),
           "psnr_bilinear_mean": float(np.mean(bl)),
           "frac_upsampled_ge_40db": float(np.mean(actual >= 40.0)),
           "fallback_threshold_db": thr, "prediction_overestimate_db": over,
           "fallback_rate": float(1.0 - accepted.mean()),
           "delivered_min_psnr": float(np.min(delivered)),
           "delivered_frac_ge_40db": float(np.mean(delivered >= 40.0)),
           "train_seconds": train_s, "train_loss_first_last": [losses[0], losses[-1]]}
    model.close()
    sg.sg_volume_destroy(h)
    return out


def bench_hmd(args):
    """The bricked stereo frame (tubes2048, both eyes, the launch the
    autotuner picks for the plain frame) under each HMD variant, timed with
    HIP events around the ray-casting kernel: emission-absorption (the plain
    frame), emission-only, maximum intensity, wrapped-space rays (radial lens
    k1 0.22, k2 0.24 about the view centre), a cut plane through the volume
    centre, a region of interest (the central half of every axis), a
    depth-buffer ray limit (a synthetic opaque plane 0.9 m from the head) and
    first-hit depth output. One step = one stereo frame of every variant."""
    from paper_1804_08197_amd import sg
    h = tube_volume(args)
    views = workload_views()
    out = run_hmd(h, views, None, args)
    sg.sg_volume_destroy(h)
    print(json.dumps(out), flush=True)


def tube_volume(args):
    """The 2048^3 tube volume, resident and committed (set-up of the
    workloads that reuse the headline volume)."""
    import torch

    import gen
    from gen.large import TubeVolume, upload_generated
    from paper_1804_08197_amd import sg
    dims, B, levels = gen.TUBES_DIMS, gen.TUBES_BRICK, gen.TUBES_LEVELS
    tv = TubeVolume().to_device()
    h = sg.sg_volume_create(dims, channels=1, dtype=sg.SG_U16, brick=B, levels=levels,
                            layout=pool_layout(args))
    upload_generated(h, tv, B, slab_bricks=2, build_lod=False)
    sg.sg_build_lod(h, 0, 0)
    sg.sg_set_transfer_function(h, 0, gen.tf_hot(), *gen.TUBE_DOMAIN)
    sg.sg_volume_commit(h)
    del tv
    torch.cuda.synchronize()
    return h


def run_hmd(h, views, launch, args):
    """The HMD variants on the tube volume h (launch: the plain frame's
    configuration, or None to tune it here)."""
    import torch

    import gen
    from paper_1804_08197_amd import sg
    outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
    depth = [torch.empty(v["height"], v["width"], device="cuda") for v in views]
    if launch is None:
        launch, _ = sg.sg_autotune(h, views, PARAMS, outs, repeats=5)
    else:
        sg.sg_set_launch_config(h, launch)
    # the synthetic depth buffer: distance along each pixel's ray to a plane
    # 0.9 m (1843.2 voxels) in front of the eye, perpendicular to the view axis
    limits = []
    for v in views:
        W, H = v["width"], v["height"]
        sx = v["tan_left"] + (np.arange(W) + 0.5) / W * (v["tan_right"] - v["tan_left"])
        sy = v["tan_top"] - (np.arange(H) + 0.5) / H * (v["tan_top"] - v["tan_bottom"])
        dist = 1843.2 * np.sqrt(1.0 + sx[None, :] ** 2 + sy[:, None] ** 2)
        limits.append(torch.from_numpy(dist.astype(np.float32)).cuda())
    c = np.array([1024.0, 1024.0, 1024.0])
    n = gen.unit((1.0, 0.7, 0.4))
    lens = (0.22, 0.24, 0.0, 0.0)
    variants = [
        ("emission_absorption", views, dict(PARAMS), None),
        ("emission_only", views, dict(PARAMS, model="eo"), None),
        ("max_intensity", views, dict(PARAMS, model="mip"), None),
        ("wrapped_space_lens", [dict(v, lens=lens) for v in views], dict(PARAMS), None),
        ("cut_plane", views, dict(PARAMS, planes=[(n[0], n[1], n[2], -float(n @ c))]), None),
        ("roi_box", views, dict(PARAMS, roi=(512, 512, 512, 1536, 1536, 1536)), None),
        ("depth_buffer_limit", [dict(v, ray_limit=l) for v, l in zip(views, limits)],
         dict(PARAMS), None),
        ("depth_output", views, dict(PARAMS), depth),
    ]
    res = {}
    for name, vs, p, dep in variants:
        st = sg.sg_render_views_stats(h, vs, p, outs, dep)
        for _ in range(args.warmup):
            sg.sg_render_views(h, vs, p, outs, dep)
        torch.cuda.synchronize()
        sg.sg_set_kernel_timing(h, True)
        for _ in range(args.steps):
            sg.sg_render_views(h, vs, p, outs, dep)
        n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
        sg.sg_set_kernel_timing(h, False)
        res[name] = {"raycast_kernel_ms": ray_ms / n_k, "cutmap_kernel_ms": cut_ms / n_k,
                     "samples": st["total_samples"],
                     "samples_per_s": st["total_samples"] / (ray_ms / n_k * 1e-3)}
        log("%s: %.3f ms, %d samples" % (name, ray_ms / n_k, st["total_samples"]))
    total_ms = sum(r["raycast_kernel_ms"] + r["cutmap_kernel_ms"] for r in res.values())
    base = res["emission_absorption"]
    alu = {"bound": "alu",
           "achieved": base["samples"] * FLOP_PER_SAMPLE / (base["raycast_kernel_ms"] * 1e-3) / 1e12,
           "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s", "traffic": None}
    alu["frac"] = alu["achieved"] / alu["peak"]
    out = {"metric": "stereo frames/s of the bricked frame under each HMD variant",
           "value": 1e3 * len(res) / total_ms, "unit": "stereo frames/s (mean over variants)",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": total_ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "tubes2048_u16_bricked_stereo_1440x1600_hmd_variants",
                      "variants": list(res), "layout": args.layout},
           "variants": res, "launch": launch, "roofline": alu}
    return out


def bench_octants(args):
    """One GPU's share of a sort-last split of the bricked stereo frame: each
    of the eight 1024^3 octants of the tubes volume rendered alone for both
    eyes (the region of interest clips every ray to the octant, so a GPU
    that owned only that octant's bricks would run the same kernel on the
    same samples), timed with HIP events around the ray-casting kernel, in
    the launch the autotuner picks for the whole frame. With eight GPUs the
    frame takes as long as the slowest octant plus the composite, so the
    headline figure is 1 / (slowest octant). One step = every octant once."""
    from paper_1804_08197_amd import sg
    h = tube_volume(args)
    views = workload_views()
    out = run_octants(h, views, None, args)
    sg.sg_volume_destroy(h)
    print(json.dumps(out), flush=True)


def run_octants(h, views, launch, args):
    """One GPU's octant share on the tube volume h (launch: the plain
    frame's configuration, or None to tune it here)."""
    import torch

    import gen
    from paper_1804_08197_amd import sg
    dims = gen.TUBES_DIMS
    if launch is None:
        outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
        launch, _ = sg.sg_autotune(h, views, PARAMS, outs, repeats=5)
        del outs
    else:
        sg.sg_set_launch_config(h, launch)
    half = [d // 2 for d in dims]
    res, boxes, parts = {}, [], []
    for o in range(9):
        if o < 8:
            lo = [half[a] * ((o >> a) & 1) for a in range(3)]
            name = "octant_%d%d%d" % tuple((o >> a) & 1 for a in range(3))
            boxes.append(tuple(lo) + tuple(l + h_ for l, h_ in zip(lo, half)))
            p = dict(PARAMS, roi=boxes[-1])
            outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
            parts.append(outs)
        else:
            name, p = "whole_frame", dict(PARAMS)
            outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
        st = sg.sg_render_views_stats(h, views, p, outs)
        for _ in range(args.warmup):
            sg.sg_render_views(h, views, p, outs)
        torch.cuda.synchronize()
        sg.sg_set_kernel_timing(h, True)
        for _ in range(args.steps):
            sg.sg_render_views(h, views, p, outs)
        n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
        sg.sg_set_kernel_timing(h, False)
        res[name] = {"raycast_kernel_ms": ray_ms / n_k, "cutmap_kernel_ms": cut_ms / n_k,
                     "samples": st["total_samples"]}
        log("%s: %.3f ms, %d samples" % (name, ray_ms / n_k, st["total_samples"]))
    # the local composite of all eight parts of both eyes (sg_composite_over);
    # each part terminates its rays on its own opacity, so the composite
    # differs from the whole frame where early termination cut the whole
    # render short (by at most 1 - ert)
    comp = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for it in range(args.warmup + args.steps):
        if it == args.warmup:
            ev[0].record()
        for i, v in enumerate(views):
            sg.sg_composite_over(v, [pp[i] for pp in parts], boxes, comp[i])
    ev[1].record()
    torch.cuda.synchronize()
    comp_ms = ev[0].elapsed_time(ev[1]) / args.steps
    comp_err = max(float((comp[i] - outs[i]).abs().max()) for i in range(len(views)))
    log("composite of 8 parts, both eyes: %.3f ms, max diff to the whole frame %.2e" % (
        comp_ms, comp_err))
    octs = {k: v for k, v in res.items() if k.startswith("octant")}
    slow = max(octs, key=lambda k: octs[k]["raycast_kernel_ms"])
    slow_ms = octs[slow]["raycast_kernel_ms"] + octs[slow]["cutmap_kernel_ms"]
    step_ms = sum(v["raycast_kernel_ms"] + v["cutmap_kernel_ms"] for v in octs.values())
    alu = {"bound": "alu",
           "achieved": octs[slow]["samples"] * FLOP_PER_SAMPLE
           / (octs[slow]["raycast_kernel_ms"] * 1e-3) / 1e12,
           "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s", "traffic": None}
    alu["frac"] = alu["achieved"] / alu["peak"]
    out = {"metric": "stereo frames/s of one GPU's octant share (slowest of eight)",
           "value": 1e3 / slow_ms, "unit": "stereo frames/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_ms,
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "tubes2048_u16_bricked_stereo_1440x1600_octant_share",
                      "octant": "1024^3", "slowest": slow, "layout": args.layout},
           "octants": res, "samples_octants_sum": sum(v["samples"] for v in octs.values()),
           "composite_ms_all_parts": comp_ms, "composite_max_diff_to_whole": comp_err,
           "launch": launch, "roofline": alu}
    return out


def flop_per_sample(channels):
    """Algorithmic FLOP of one emission-absorption sample, with a linear
    interpolation counted as one multiply-add (2 FLOP): trilinear 7 lerps
    14, table 4 lerps 8, the exponential 1, compositing 8 -- 31 for one
    channel. Each further channel adds its trilinear 14 and table 8 and its
    share of the sum 7 (extinction add, weighted colour); several channels
    add the colour normalisation 4."""
    return FLOP_PER_SAMPLE + 29 * (channels - 1) + (4 if channels > 1 else 0)


def bench_stream(args):
    print(json.dumps(run_stream(args)), flush=True)


def run_stream(args):
    """The 3-channel 1024x1024x512 uint16 cell time series played through the
    out-of-core brick cache (stereo 1440x1600 per eye). The host tier holds
    every brick (core + apron, all levels) of --stream-timepoints timepoints
    in page-locked memory; the GPU cache holds --stream-slots bricks, less
    than two timepoints, so every timepoint of the looping movie arrives
    from the host. One step = one timepoint played to full detail: render
    the stereo frame with what is resident (coarser blocks stand in for
    missing ones), load the blocks the render requested, and repeat until a
    render requests nothing. Also timed: the converged timepoint rendered
    with everything it needs resident (per-timepoint stereo frames/s), and
    a plain page-locked host-to-device copy (the bus rate)."""
    import torch

    import gen
    from gen.large import CellVolume
    from paper_1804_08197_amd import sg
    from paper_1804_08197_amd.container import HostBrickStore
    dims, B, L, C = gen.CELLS_DIMS, gen.CELLS_BRICK, gen.CELLS_LEVELS, 3
    T = args.stream_timepoints
    if T < 3:
        raise SystemExit("bench.py: --stream-timepoints must be at least 3")
    h = sg.sg_volume_create(dims, channels=C, timepoints=T, dtype=sg.SG_U16, brick=B, levels=L,
                            cache_slots=args.stream_slots, layout=pool_layout(args))
    store = HostBrickStore(h, dims, B, L, 2)
    t0 = time.time()
    for t in range(T):
        for c in range(C):
            cv = CellVolume(c, t).to_device()
            store.add(t, c, cv.region((0, 0, 0), dims, device=True))
        torch.cuda.synchronize()
        log("host tier: timepoint %d ready (%.1fs, %.1f GiB page-locked)" % (
            t, time.time() - t0, store.host_bytes() / 2**30))
    setup_s = time.time() - t0
    tfs = [gen.tf_tint(tint) for tint in gen.CELL_TINTS]
    for c in range(C):
        sg.sg_set_transfer_function(h, c, tfs[c], *gen.CELL_DOMAIN)
    for t in range(T):
        store.put_top(t)
    views = gen.cells_stereo()
    params = {"step": 0.5, "ert": 0.99, "tau": 1.0, "lod": 1, "skip_empty": 1, "bias": 0}
    outs = [torch.empty(v["height"], v["width"], 4, device="cuda") for v in views]

    def play(t):
        p = dict(params, timepoint=t)
        frames = nodes = 0
        render_s = 0.0
        while True:
            a = time.perf_counter()
            sg.sg_render_views(h, views, p, outs)
            torch.cuda.synchronize()
            render_s += time.perf_counter() - a
            frames += 1
            n = store.serve_requests()
            nodes += n
            if n == 0:
                return frames, nodes, render_s

    for k in range(args.warmup):
        play(k % T)
    torch.cuda.synchronize()
    info0 = sg.sg_cache_get_info(h)
    bytes0, nodes0 = store.served_bytes, store.served_nodes
    frames = 0
    render_s = 0.0
    per_tp = []
    wall0 = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        f, n, r = play((args.warmup + k) % T)
        per_tp.append((time.perf_counter() - a, f, n))
        frames += f
        render_s += r
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    info = sg.sg_cache_get_info(h)
    up_bytes = store.served_bytes - bytes0
    up_nodes = store.served_nodes - nodes0
    log("stream: %d timepoints in %.3fs, %d frames, %d nodes (%.2f GB) uploaded" % (
        args.steps, wall, frames, up_nodes, up_bytes / 1e9))

    # the last timepoint, converged: its frame with everything it needs resident
    t_last = (args.warmup + args.steps - 1) % T
    p_last = dict(params, timepoint=t_last)
    stats = sg.sg_render_views_stats(h, views, p_last, outs)
    assert len(sg.sg_cache_requests(h)[0]) == 0
    for _ in range(3):
        sg.sg_render_views(h, views, p_last, outs)
    torch.cuda.synchronize()
    sg.sg_set_kernel_timing(h, True)
    a = time.perf_counter()
    R = 10
    for _ in range(R):
        sg.sg_render_views(h, views, p_last, outs)
    torch.cuda.synchronize()
    res_ms = (time.perf_counter() - a) * 1e3 / R
    n_k, cut_ms, ray_ms = sg.sg_get_kernel_timing(h)
    sg.sg_set_kernel_timing(h, False)
    ray_s = ray_ms / n_k * 1e-3
    samples = stats["total_samples"]
    npix = sum(v["width"] * v["height"] for v in views)
    alu = {"bound": "alu", "achieved": samples * flop_per_sample(C) / ray_s / 1e12,
           "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s", "traffic": None}
    alu["frac"] = alu["achieved"] / alu["peak"]
    hbm = {"bound": "hbm", "achieved": (stats["microblocks"] * 64 * 2 + npix * 16) / ray_s / 1e9,
           "peak": HBM_PEAK / 1e9, "unit": "GB/s", "traffic": None}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]

    # the bus: a plain page-locked host-to-device copy of 1 GiB
    src = torch.empty(1 << 30, dtype=torch.uint8, pin_memory=True)
    dst = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(3):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    bus = 3 * (1 << 30) / (time.perf_counter() - a)
    del src, dst

    ms = wall * 1e3 / args.steps
    out = {"metric": "timepoints/s of a 3-channel time series played through the brick cache",
           "value": args.steps / wall, "unit": "timepoints/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "cells_3x1024x1024x512_u16_stream_stereo_1440x1600",
                      "timepoints_in_host_tier": T, "cache_slots": args.stream_slots,
                      "layout": args.layout,
                      "bricks_per_timepoint": sum(int(np.prod(g)) for g in store.grids) * C,
                      "brick": B, "levels": L, "channels": C, "step_voxels": 0.5, "ert": 0.99,
                      "lod_tau_px": 1.0},
           "frames_per_timepoint": frames / args.steps,
           "stereo_frames_per_s_during_playback": frames / wall,
           "render_share_of_step": render_s / wall,
           "bricks_uploaded_per_timepoint": up_nodes * C / args.steps,
           "upload_GB_per_timepoint": up_bytes / args.steps / 1e9,
           "upload_GB_per_s": up_bytes / wall / 1e9,
           "core_voxels_streamed_per_s": up_nodes * C * B ** 3 / wall,
           "host_to_device_copy_GB_per_s": bus / 1e9,
           "step_ms_min_max": [min(x[0] for x in per_tp) * 1e3, max(x[0] for x in per_tp) * 1e3],
           "evictions": info["evictions"] - info0["evictions"],
           "resident_frame_ms": res_ms, "resident_stereo_frames_per_s": 1e3 / res_ms,
           "resident_raycast_kernel_ms": ray_ms / n_k, "resident_samples_per_frame": samples,
           "roofline": alu if alu["frac"] >= hbm["frac"] else hbm,
           "roofline_other": hbm if alu["frac"] >= hbm["frac"] else alu,
           "setup_host_tier_s": setup_s,
           "paper_context": "3D movies of up to 2e7 voxels per volume frame play at 25 volume "
                            "frames/s (Sec 5.4; hardware not stated)"}
    sg.sg_volume_destroy(h)
    return out


def profile_record():
    """The committed rocprofv3 record of the ray-casting kernel (byte counters
    calibrated against a copy of known size, VALU counters), or None once
    the kernel source has changed since it was taken."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "raycast_tubes2048_stereo.traffic.json")
    try:
        rec = json.load(open(rec_path))
        src = open(os.path.join(ROOT, rec["kernel_source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("kernel_source_sha256"):
        return None
    return rec


def measured_traffic():
    """HBM bytes per ray-casting dispatch from the committed FETCH_SIZE /
    WRITE_SIZE passes, or None (see profile_record)."""
    rec = profile_record()
    return rec["traffic_bytes_per_dispatch"] if rec else None


def copy_calibration(nbytes):
    """A plain device-to-device copy of known size: its FETCH_SIZE /
    WRITE_SIZE readings calibrate the byte counters for the roofline."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for _ in range(3):
        ev[0].record()
        b.copy_(a)
        ev[1].record()
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    print(json.dumps({"copy_bytes": n * 4, "ms": times,
                      "GB_per_s_read_plus_write": 2 * n * 4 / (min(times) * 1e-3) / 1e9}),
          flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(host, tf, views, npix, seconds):
    """The FP64 oracle on a seeded random subset of the tube frame's pixels."""
    import gen
    import oracle
    t0 = time.time()
    sc = oracle.Scene([host], gen.TUBES_BRICK, gen.TUBES_LEVELS,
                      [np.asarray(tf, np.float32).astype(np.float64)], [gen.TUBE_DOMAIN])
    log("oracle setup %.1fs" % (time.time() - t0))
    return oracle_pixel_subset(sc, views, PARAMS, npix, seconds, "stereo frames/s")


def oracle_pixel_subset(sc, views, params, npix, seconds, unit):
    """The oracle on uniformly random pixels of every view (seeded), on all
    of this host's threads for about ``seconds``, then on one thread for
    4,096 further pixels per view; each rate is extrapolated to the frame
    by pixel count."""
    import oracle
    cuts = [sc.cut(v, params) for v in views]
    emps = [sc.empty(c) for c in cuts]
    rng = np.random.default_rng(2024)
    threads = oracle.max_threads()
    done_pix, done_samp, spent, n = 0, 0, 0.0, 64
    while spent < seconds and done_pix < npix // 4:
        for i, v in enumerate(views):
            pix = np.stack([rng.integers(0, v["width"], n), rng.integers(0, v["height"], n)], 1)
            t = time.perf_counter()
            r = sc.render(v, params, pixels=pix, cut=cuts[i], empty=emps[i], threads=threads)
            spent += time.perf_counter() - t
            done_pix += n
            done_samp += r["total_samples"]
        n = min(n * 2, 8192)
    frame_s = spent / done_pix * npix
    one_pix, one_samp, one_s = 0, 0, 0.0
    for i, v in enumerate(views):
        pix = np.stack([rng.integers(0, v["width"], 4096), rng.integers(0, v["height"], 4096)], 1)
        t = time.perf_counter()
        r = sc.render(v, params, pixels=pix, cut=cuts[i], empty=emps[i], threads=1)
        one_s += time.perf_counter() - t
        one_pix += len(pix)
        one_samp += r["total_samples"]
    return {"value": 1.0 / frame_s, "unit": unit, "cores": threads,
            "kind": "oracle", "samples_per_s": done_samp / spent,
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": one_pix / (one_s * npix), "unit": unit,
                              "samples_per_s": one_samp / one_s, "pixels": one_pix},
            "sample": "%d uniformly random pixels of %d view(s) (%.1f%% of the frame's pixel "
                      "count), %.1fs of wall time on %d threads, extrapolated to the frame by "
                      "pixel count" % (done_pix, len(views), 100.0 * done_pix / npix, spent,
                                       threads)}


def oracle_whole_frame(sc, views, params, unit):
    """The oracle rendering every pixel of the frame: on all of this host's
    threads, then on one thread."""
    import oracle
    threads = oracle.max_threads()
    res = {}
    for k in (threads, 1):
        t = time.perf_counter()
        samp = sum(sc.render(v, params, threads=k, count=True)["total_samples"] for v in views)
        res[k] = (time.perf_counter() - t, samp)
    (s_all, n_all), (s_one, n_one) = res[threads], res[1]
    return {"value": 1.0 / s_all, "unit": unit, "cores": threads, "kind": "oracle",
            "samples_per_s": n_all / s_all, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": 1.0 / s_one, "unit": unit, "samples_per_s": n_one / s_one},
            "sample": "the whole frame (%d view(s)), %.2fs on %d threads and %.2fs on one"
                      % (len(views), s_all, threads, s_one)}


if __name__ == "__main__":
    main()
