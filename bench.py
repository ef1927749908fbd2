#!/usr/bin/env python3
"""Benchmark of the MI355X ray-based Gaussian splatting renderer.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload all|c1|c2|c3|c4]

The default (all) prints one JSON line with the three parts of the metric:
  value / c1    frames/s at 1080p with 500k Gaussians (64 clusters, SH3), one
                1920x1080 camera at 50 deg FOV on a 16-pose orbit.  A step is
                one orbit: 16 frames, one per pose, each a HIP-graph replay of
                the whole hot path (preprocess, depth sort, scan, emit, tile
                sort, ranges, compositing), so every timed step weights the
                poses equally.
  c2            batched stereo views/s: 3M Gaussians, 4 stereo pairs (8 views,
                2064x2208 per eye x {0.5,1,2} per pair), MIP on; a step renders
                all 8 views in one graph replay at 16x8 tiles (8 plain
                single-view renders reported beside it).
  c3            backward ms/view: 1M Gaussians, 4 views at 1600x1060; a step is
                forward + L1 loss gradient + backward, at the tile shape the
                library's training autotuner picks (--no-autotune: --tile).
Each part carries a roofline object for its compositing kernel (forward for c1
and c2, backward for c3); a leg that fails reports its error in place of its
figures and the line is still printed.
Single legs: --workload c1|c2|c3, and
  c4            6M Gaussians, 16 cameras of uneven size (256..2560 x 256..1440)
                and FOV, autotuned tile shape; a step is forward + L1 loss gradient
                + backward over all 16 views.  Metric: megapixels/s of the step;
                per-view forward latency p50/p99 from device completion clocks.
  --divergence gs  c1 with the linearised divergence of 3DGS (Sec. 3.1) in the same
                pipeline: the same-model speed comparison of GS and RayGS.
  --mip exact   c2 rendered with the exact per-ray MIP (c3 trains through it).

Inputs are resident in HBM before the timed region.  Each roofline covers one
kernel, timed with HIP events on the stream it is launched on; its algorithmic
work comes from the oracle's counts of the same frames
(tests/golden/work_counts_<workload>.json).
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

METRIC = "frames/s at 1080p with 500k Gaussians; batched stereo views/s; backward ms/view"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X vector FP32 (published)
POSES = 16                     # c1 orbit poses per step
# Algorithmic FP32 work of compositing (FMA counts 2, as in the published peak).
# Forward, per fragment (pixel centre inside a projected quad), eq. 16 and eq. 2:
#   delta = p - pi(mu) (2), n = G delta (6), den = k0 + g . delta (4), q = |n|^2 (3),
#   den^2 + q / c^2 (3), D = q / (...) (1), omega = o exp(-D / 2) (3)      -> 22
# per composited fragment, eq. 1: alpha = min(omega, alpha_max), 1 - alpha,
#   T (1 - alpha), T alpha, three colour multiply-adds (6)                  -> 10
FLOP_PER_FRAGMENT = 22
FLOP_PER_CONTRIBUTION = 10
# Backward, per fragment up to the pixel's stop: omega again (22); per
# composited fragment, the adjoint of eq. 1 (T_i = T_i+1 / (1 - alpha): 2,
# g . rgb: 5, dL/dalpha: 4, the running sum S: 2, dL/drgb: 7), through
# alpha and omega to D and o (3), D = q / (den^2 + q / c^2) to q, den, 1/c^2 (8),
# to n, G, g, k0 and pi(mu) (2 + 8 + 4 + 1 + 8) and the 13 record-gradient
# accumulations (13)                                                        -> 65
FLOP_PER_CONTRIBUTION_BWD = 65
# Algorithmic bytes of the other stages (per unit):
PARAM_BYTES = {0: 56, 1: 92, 2: 152, 3: 236}   # Gaussian parameters read once per batch
RECORD_BYTES = 64 + 4 + 8 + 64 + 4             # record, depth key, pixel box, support conic, tile count per visible Gaussian-view
INSTANCE_BYTES = 8                             # (tile id, Gaussian id) written once
PIXEL_BYTES = 20                               # rgb + final T + n_contrib


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="all", choices=["all", "c1", "c2", "c3", "c4"])
    ap.add_argument("--mip", default="approx", choices=["approx", "exact"],
                    help="c2: the approximate MIP of eq. 17 (the paper's renderer) or the exact per-ray MIP; "
                         "c3: exact turns the exact per-ray MIP on (the workload has none)")
    ap.add_argument("--divergence", default="ray", choices=["ray", "gs"],
                    help="c1: the ray-based divergence (the paper's renderer) or the linearised one of 3DGS")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of HIP-graph replays")
    ap.add_argument("--in-flight", type=int, default=1,
                    help="c1: frames in flight for `value` (each its own graph, workspace and stream); the line "
                         "also reports the throughput with 2 and 3 in flight")
    ap.add_argument("--single-flight", action="store_true",
                    help="c1: skip the 2 and 3 frames-in-flight timings (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-steps", type=int, default=32, help="frames of the per-stage timing pass")
    ap.add_argument("--tile", default=None,
                    help="tile shape WxH, each of 8, 16, 32 (default: 8x16 for c1, 16x8 for c2, the autotuner's "
                         "for c3 and c4, 8x16 there with --no-autotune)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="c3, c4: use --tile instead of the training autotuner (for profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for HBM counters)")
    return ap.parse_args()


# Tile shape of each workload when --tile is not given, from sweeps of the
# nine shapes on the benchmark itself: the 1080p frame is fastest at 8x16,
# the stereo batch (views of 1-18 MP) at 16x8 (849 against 823 views/s at
# 8x16).  The training workloads take the autotuner's shape.
DEFAULT_TILE = {"c1": "8x16", "c2": "16x8"}


def tile_of(args, workload):
    return args.tile or DEFAULT_TILE.get(workload, "8x16")


def tile_opts(args, workload):
    tw, th = (int(v) for v in tile_of(args, workload).lower().split("x"))
    return dict(tile_w=tw, tile_h=th)


def work_counts(name):
    path = os.path.join(ROOT, "tests", "golden", f"work_counts_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def to_dev(scene, torch):
    g = {k: torch.from_numpy(np.ascontiguousarray(scene[k])).cuda() for k in
         ("means", "log_scales", "quats", "opacity_logits", "sh")}
    g["sh_degree"] = int(scene["sh_degree"])
    return g


def stage_pass(r, g, cams_seq, opts, ws, outs, frames):
    """Eager renders with per-stage HIP events on the launch stream."""
    import torch

    r.stage_times()  # reset
    r.set_stage_timing(True)
    torch.cuda.synchronize()
    for k in range(frames):
        r.render_into(g, cams_seq(k), outs, ws, opts)
    torch.cuda.synchronize()
    ms, n = r.stage_times()
    r.set_stage_timing(False)
    return {k: v / max(n, 1) for k, v in ms.items()}, n


def pmc_traffic(stage, workload):
    """HBM bytes per launch of a compositing kernel (stage blend: k_blend,
    blend_backward: k_blend_bwd) from the committed counter summary
    (profiles/<stage>_<workload>_pmc_traffic.txt), or None when there is none
    for this workload or the kernel's sources changed since it was taken."""
    kernel = {"blend": "k_blend", "blend_backward": "k_blend_bwd"}.get(stage)
    if kernel is None:
        return None
    from paper_2503_18682_amd.prof_summary import read_traffic

    return read_traffic(os.path.join(ROOT, "profiles", f"{stage}_{workload}_pmc_traffic.txt"), kernel)


def roofline_for(stage, ms, *, flops=None, nbytes=None, traffic=None):
    if stage.startswith("blend"):
        achieved = flops / (ms * 1e-3) / 1e12 if flops else None
        return {"bound": "alu", "kernel": stage, "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS if achieved else None, "traffic": traffic,
                "avg_ms": ms, "algorithmic_flop": flops}
    achieved = nbytes / (ms * 1e-3) / 1e9 if nbytes else None
    return {"bound": "hbm", "kernel": stage, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": traffic, "avg_ms": ms,
            "algorithmic_bytes": nbytes}


def frame_work(wc, views):
    """Oracle fragments and composited fragments summed over `views` (indices
    into the work-count file), or None without a file."""
    if not wc:
        return None
    vs = wc["views"]
    return (float(sum(vs[v]["fragments"] for v in views)), float(sum(vs[v]["contributions"] for v in views)))


def cpu_baseline_c1(scene, cam, opts):
    """The oracle on a bounded sample of one 1080p frame: the full per-Gaussian
    stage plus 8 bands of 6 rows spread over the image, scaled to a frame."""
    import oracle

    threads = os.cpu_count() or 1
    # the per-Gaussian stage alone (no rows), after one untimed call that pays
    # the one-time costs (library load, first touch of the scene's pages);
    # the faster of two calls, so that its noise is not subtracted from the rows
    oracle.render(scene, cam, opts, rows=(0, 0), threads=threads, branches=False)
    t_fixed = float("inf")
    for _ in range(2):
        t = time.perf_counter()
        oracle.render(scene, cam, opts, rows=(0, 0), threads=threads, branches=False)
        t_fixed = min(t_fixed, time.perf_counter() - t)
    H = cam["height"]
    band, rows_done, t_rows = 6, 0, 0.0
    for b in range(8):
        a = int((b + 0.5) * H / 8) - band // 2
        t = time.perf_counter()
        oracle.render(scene, cam, opts, rows=(a, a + band), threads=threads, branches=False)
        t_rows += max(time.perf_counter() - t - t_fixed, 0.0)
        rows_done += band
    frame_s = t_fixed + t_rows * H / rows_done
    return {"value": 1.0 / frame_s, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"pose 0: full per-Gaussian stage + {rows_done} of {H} rows (8 bands), scaled to one frame"}


def bench_c1(args, torch):
    import scenegen
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c1")
    sc, cams, opts = w["scene"], w["cameras"], dict(w["options"], **tile_opts(args, "c1"))
    gs = args.divergence == "gs"
    if gs:
        opts["divergence"] = 1
    n = int(sc["opacity_logits"].shape[0])
    g = to_dev(sc, torch)
    r = R.Renderer(0, opts)
    # size the instance capacity over all poses
    need = 0
    for c in cams:
        _, (buf, ws) = r.render(g, [c], opts, keep_workspace=True)
        need = max(need, r.status(ws)[1])
        del buf
    capacity = int(need * 1.1) + 4096
    log(f"c1: {n} Gaussians, {POSES} poses, max instances {need}, capacity {capacity}")
    br = R.BatchRenderer(r, n, sc["sh_degree"], [cams[0]], capacity, options=opts)
    # frames in flight: each its own plan (workspace, graph, outputs) on its
    # own stream, consecutive poses round robin
    flight = [(br, torch.cuda.current_stream())]
    for _ in range(1, max(args.in_flight, 1 if args.single_flight or args.eager else 3)):
        flight.append((R.BatchRenderer(r, n, sc["sh_degree"], [cams[0]], capacity, options=opts),
                       torch.cuda.Stream()))

    def step(f):
        # one orbit: a frame at each pose
        for k, c in enumerate(cams):
            if args.eager:
                r.render_into(g, [c], br.outs, br.ws, opts)
            else:
                b, st = flight[k % f]
                with torch.cuda.stream(st):
                    b.launch(g, [c])

    def timed(f):
        for _ in range(args.warmup):
            step(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(f)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for b, _ in flight[:f]:
            assert b.status()[0], "instance capacity overflow in the timed region"
        return (t1 - t0) * 1e3 / args.steps

    ms = timed(args.in_flight)
    # throughput with more frames in flight (every frame still runs the whole path)
    pipelined = {} if args.eager or args.single_flight else \
        {str(f): POSES * 1e3 / timed(f) for f in (2, 3) if f != args.in_flight}
    for b, _ in flight[1:]:
        b.close()
    frames = max(POSES, POSES * math.ceil(args.stage_steps / POSES))
    stages, _ = stage_pass(r, g, lambda k: [cams[k % POSES]], opts, br.ws, br.outs, frames)
    fwd = {k: v for k, v in stages.items() if not k.endswith("backward")}
    work = frame_work(work_counts("c1_gs" if gs else "c1"), range(POSES))
    flops = (FLOP_PER_FRAGMENT * work[0] + FLOP_PER_CONTRIBUTION * work[1]) / POSES if work else None
    tag = "c1_1080p_500k_" + tile_of(args, "c1") + ("_gs" if gs else "")
    roof = roofline_for("blend", fwd["blend"], flops=flops, traffic=pmc_traffic("blend", tag))
    # measured ceilings of this device (context for `peak`, which stays the published figure)
    calib = r.calibrate()
    if roof["achieved"]:
        roof["attainable_peak"] = calib["fma_tflops"]
        roof["attainable_frac"] = roof["achieved"] / calib["fma_tflops"]
    res = {
        "metric": METRIC, "value": POSES * 1e3 / ms, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c1: 500k Gaussians (64 clusters, SH3), 1920x1080, 50deg FOV, 16 orbit poses"
                   + (" (linearised GS divergence)" if gs else ""),
                   "n_gaussians": n, "width": 1920, "height": 1080, "tile": tile_of(args, "c1"),
                   "frames_per_step": POSES, "step": "one frame at each of the 16 orbit poses",
                   "frames_in_flight": args.in_flight,
                   "launch": "eager" if args.eager else "hip_graph", "instance_capacity": capacity},
        "roofline": roof,
        "calibration": calib,
        "stages_ms": stages,
        "dominant_stage": max(fwd, key=fwd.get),
        "frames_per_s_in_flight": pipelined,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_c1(sc, cams[0], opts)
    br.close()
    r.close()
    return res


def bench_c2(args, torch):
    import scenegen
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c2")
    sc, cams, opts = w["scene"], w["cameras"], dict(w["options"], **tile_opts(args, "c2"))
    if args.mip == "exact":
        opts["mip"] = 2
    n = int(sc["opacity_logits"].shape[0])
    g = to_dev(sc, torch)
    r = R.Renderer(0, opts)
    _, (buf, ws) = r.render(g, cams, opts, keep_workspace=True)
    need = r.status(ws)[1]
    del buf
    capacity = int(need * 1.1) + 4096
    br = R.BatchRenderer(r, n, sc["sh_degree"], cams, capacity, options=opts)
    for _ in range(args.warmup):
        br.launch(g, cams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        br.launch(g, cams)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert br.status()[0], "instance capacity overflow in the timed region"
    ms = (t1 - t0) * 1e3 / args.steps
    # 8 plain single-view renders
    singles = []
    for c in cams:
        _, (b1, w1) = r.render(g, [c], opts, keep_workspace=True)
        singles.append((b1, w1, r.allocate_outputs([c])))
    torch.cuda.synchronize()
    reps = max(args.steps // 4, 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        for c, (b1, w1, o1) in zip(cams, singles):
            r.render_into(g, [c], o1, w1, opts)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / reps
    del singles
    stages, _ = stage_pass(r, g, lambda k: cams, opts, br.ws, br.outs, max(args.stage_steps // 4, 4))
    fwd = {k: v for k, v in stages.items() if not k.endswith("backward")}
    work = frame_work(work_counts("c2") if args.mip != "exact" else None, range(len(cams)))
    flops = FLOP_PER_FRAGMENT * work[0] + FLOP_PER_CONTRIBUTION * work[1] if work else None
    res = {
        "metric_part": "batched stereo views/s", "value": 8e3 / ms, "unit": "views/s", "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "config": {"workload": "c2: 3M Gaussians, 4 stereo pairs (8 views), MIP on, one HIP-graph replay"
                   + (" (exact per-ray MIP)" if args.mip == "exact" else ""),
                   "views": [[c["width"], c["height"]] for c in cams], "tile": tile_of(args, "c2"),
                   "instance_capacity": capacity},
        "plain_launches_views_per_s": 8e3 / plain_ms,
        "roofline": roofline_for("blend", fwd["blend"], flops=flops,
                                 traffic=pmc_traffic("blend", "c2_stereo_3m_8views_" + tile_of(args, "c2"))),
        "stages_ms": stages,
        "dominant_stage": max(fwd, key=fwd.get),
    }
    br.close()
    r.close()
    return res


def bench_c3(args, torch):
    import scenegen
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c3")
    sc, cams, opts = w["scene"], w["cameras"], dict(w["options"], **tile_opts(args, "c3"))
    if args.mip == "exact":
        opts["mip"] = 2
    n = int(sc["opacity_logits"].shape[0])
    g = to_dev(sc, torch)
    targets = [torch.from_numpy(t).cuda() for t in w["targets"]]
    total = sum(t.numel() for t in targets)
    r = R.Renderer(0, opts)
    outs = r.allocate_outputs(cams)
    tile_from = "--tile"
    if not args.no_autotune:
        # the tile shape of the fastest training step (render + backward), timed
        # by the library's autotuner in a workspace with room for the finest tiles
        fine = dict(opts, tile_w=8, tile_h=8)
        _, (buf, ws) = r.render(g, cams, fine, keep_workspace=True)
        need = r.status(ws)[1]
        del buf, ws
        buf, ws = r.new_workspace(n, cams, int(need * 1.1) + 4096, _lib.RGS_WS_BACKWARD, fine)
        r.render_into(g, cams, outs, ws, fine)
        dls = [torch.sign(o["rgb"] - t) / total for o, t in zip(outs, targets)]
        opts, tune_ms = r.autotune_training(g, cams, ws, outs, dls, reps=3, options=opts)
        tile_from = "rgs_autotune_training"
        log(f"c3: autotuned tile {opts['tile_w']}x{opts['tile_h']} ({tune_ms:.2f} ms per render + backward)")
        del buf, ws, dls
    _, (buf, ws) = r.render(g, cams, opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    need = r.status(ws)[1]
    del buf
    capacity = int(need * 1.1) + 4096
    buf, ws = r.new_workspace(n, cams, capacity, _lib.RGS_WS_BACKWARD, opts)
    grads = {k: torch.zeros_like(g[k]) for k in R.PARAM_KEYS}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step():
        r.render_into(g, cams, outs, ws, opts)
        dls = [torch.sign(o["rgb"] - t) / total for o, t in zip(outs, targets)]
        ev[1].record()
        r.backward(g, cams, outs, dls, ws, opts, grads=grads)
        ev[2].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    bwd = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        ev[2].synchronize()
        bwd += ev[1].elapsed_time(ev[2])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    assert r.status(ws)[0], "instance capacity overflow in the timed region"
    r.stage_times()  # reset
    r.set_stage_timing(True)
    for _ in range(4):
        step()
    torch.cuda.synchronize()
    stages, frames = r.stage_times()
    r.set_stage_timing(False)
    stages = {k: v / max(frames, 1) for k, v in stages.items()}
    work = frame_work(work_counts("c3") if args.mip != "exact" else None, range(len(cams)))
    flops = FLOP_PER_FRAGMENT * work[0] + FLOP_PER_CONTRIBUTION_BWD * work[1] if work else None
    res = {
        "metric_part": "backward ms/view", "value": bwd / args.steps / len(cams), "unit": "backward ms/view",
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False,
        "config": {"workload": "c3: 1M Gaussians (SH3), 4 views 1600x1060, forward + L1 + backward"
                   + (" (exact per-ray MIP)" if args.mip == "exact" else ""),
                   "tile": f"{opts['tile_w']}x{opts['tile_h']}", "tile_from": tile_from,
                   "instance_capacity": capacity},
        "roofline": roofline_for("blend_backward", stages["blend_backward"], flops=flops,
                                 traffic=pmc_traffic("blend_backward",
                                                     f"c3_train_1m_4views_{opts['tile_w']}x{opts['tile_h']}")),
        "stages_ms": stages,
    }
    r.close()
    return res


def line_of(part, res):
    """A single-leg result as a full benchmark line."""
    out = {"metric": METRIC, "value": res["value"], "unit": res["unit"], "n_gpus": 1, "steps": res["steps"],
           "warmup": res["warmup"], "ms_per_step": res["ms_per_step"], "higher_is_better": res["higher_is_better"],
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    out.update({k: v for k, v in res.items() if k not in out})
    out["metric_part"] = part
    return out


def bench_c4(args, torch):
    import scenegen
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c4")
    sc, cams, opts0 = w["scene"], w["cameras"], w["options"]
    n = int(sc["opacity_logits"].shape[0])
    g = to_dev(sc, torch)
    targets = [torch.from_numpy(t).cuda() for t in w["targets"]]
    r = R.Renderer(0, opts0)
    # autotune the tile shape of the whole training step (render + backward) in
    # a workspace with room for the finest tiles
    fine = dict(opts0, tile_w=8, tile_h=8)
    _, (buf, ws) = r.render(g, cams, fine, keep_workspace=True)
    need = r.status(ws)[1]
    del buf, ws
    buf, ws = r.new_workspace(n, cams, int(need * 1.1) + 4096, _lib.RGS_WS_BACKWARD, fine)
    outs = r.allocate_outputs(cams)
    if args.no_autotune:
        opts, tile_from = dict(opts0, **tile_opts(args, "c4")), "--tile"
    else:
        r.render_into(g, cams, outs, ws, fine)
        dls = [torch.sign(o["rgb"] - t) / sum(t.numel() for t in targets) for o, t in zip(outs, targets)]
        opts, tune_ms = r.autotune_training(g, cams, ws, outs, dls, reps=3)
        tile_from = "rgs_autotune_training"
        log(f"c4: autotuned tile {opts['tile_w']}x{opts['tile_h']} ({tune_ms:.2f} ms per render + backward)")
        del dls
    del buf, ws
    _, (buf, ws) = r.render(g, cams, opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    need = r.status(ws)[1]
    del buf, ws
    capacity = int(need * 1.1) + 4096
    buf, ws = r.new_workspace(n, cams, capacity, _lib.RGS_WS_BACKWARD, opts)
    grads = {k: torch.zeros_like(g[k]) for k in R.PARAM_KEYS}
    total = sum(t.numel() for t in targets)
    pixels = sum(c["width"] * c["height"] for c in cams)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step():
        ev[0].record()
        r.render_into(g, cams, outs, ws, opts)
        dls = [torch.sign(o["rgb"] - t) / total for o, t in zip(outs, targets)]
        ev[1].record()
        r.backward(g, cams, outs, dls, ws, opts, grads=grads)
        ev[2].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(args.steps // 8, 20)
    fwd = bwd = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        ev[2].synchronize()
        fwd += ev[0].elapsed_time(ev[1])
        bwd += ev[1].elapsed_time(ev[2])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    assert r.status(ws)[0], "instance capacity overflow in the timed region"
    # per-view forward latency: device clocks of the frame start and of each
    # view's last finished compositing work item, over separate renders
    stamps = torch.zeros(len(cams) + 1, dtype=torch.int64, device="cuda")
    r.set_view_clocks(stamps)
    lat = []
    for _ in range(steps):
        r.render_into(g, cams, outs, ws, opts)
        torch.cuda.synchronize()
        lat.append(r.view_latencies_ms(stamps, len(cams)))
    r.set_view_clocks(None)
    lat = np.asarray(lat)
    r.stage_times()  # reset
    r.set_stage_timing(True)
    for _ in range(4):
        step()
    torch.cuda.synchronize()
    stages, frames = r.stage_times()
    r.set_stage_timing(False)
    stages = {k: v / max(frames, 1) for k, v in stages.items()}
    dom = max(stages, key=stages.get)
    return {
        "metric": METRIC, "value": pixels / 1e6 / (ms * 1e-3), "unit": "megapixels/s (forward + backward)",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4: 6M Gaussians (SH3), 16 uneven cameras, autotuned, forward + L1 + backward",
                   "views": [[c["width"], c["height"]] for c in cams], "megapixels": pixels / 1e6,
                   "tile": [opts["tile_w"], opts["tile_h"]], "tile_from": tile_from,
                   "instance_capacity": capacity},
        "forward_ms": fwd / steps, "backward_ms": bwd / steps,
        "forward_megapixels_per_s": pixels / 1e6 / (fwd / steps * 1e-3),
        "view_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                            "per_view_median": [float(x) for x in np.median(lat, axis=0)],
                            "samples": int(lat.size)},
        "roofline": roofline_for(dom, stages[dom]),
        "stages_ms": stages,
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the renderer has no multi-GPU path "
              "(views would shard across GPUs with no exchange). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "all":
        res = bench_c1(args, torch)
        for key, leg in (("c2", bench_c2), ("c3", bench_c3)):
            torch.cuda.empty_cache()
            try:
                res[key] = leg(args, torch)
            except Exception as e:  # the c1 line is printed whatever a later leg does
                res[key] = {"error": f"{type(e).__name__}: {e}"}
            log(f"{key}: {json.dumps({k: res[key].get(k) for k in ('value', 'unit', 'error')})}")
    elif args.workload == "c1":
        res = bench_c1(args, torch)
    elif args.workload == "c2":
        res = line_of("batched stereo views/s", bench_c2(args, torch))
    elif args.workload == "c3":
        res = line_of("backward ms/view", bench_c3(args, torch))
    else:
        res = bench_c4(args, torch)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
