#!/usr/bin/env python3
"""Benchmark of the MI355X ray-based Gaussian splatting renderer.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c2|c3|c4]

Workloads (synthetic, seeded; see scenegen/scenes.py):
  c1 (default)  500k Gaussians (64 clusters, SH3), one 1920x1080 camera at 50 deg
                FOV cycling over 16 orbit poses; a step renders one frame through
                the whole hot path (preprocess, depth sort, scan, emit, tile sort,
                ranges, compositing) replayed as one HIP graph.  Metric: frames/s.
  c2            3M Gaussians, 4 stereo pairs (8 views, 2064x2208 per eye x
                {0.5,1,2} per pair), MIP on; a step renders all 8 views in one
                graph replay.  Metric: views/s (8 single-view renders reported too).
                --mip exact renders the same frame with the exact per-ray MIP
                (and, for c3, trains through it).
  --divergence gs  c1 with the linearised divergence of 3DGS (Sec. 3.1) in the same
                pipeline: the same-model speed comparison of GS and RayGS.
  c3            1M Gaussians, 4 views at 1600x1060; a step is forward + L1 loss
                gradient + backward.  Metric: backward ms/view.
  c4            6M Gaussians, 16 cameras of uneven size (256..2560 x 256..1440)
                and FOV, autotuned tile shape; a step is forward + L1 loss gradient
                + backward over all 16 views.  Metric: megapixels/s of the step;
                per-view forward latency p50/p99 from device completion clocks.

Prints ONE JSON line.  Inputs are resident in HBM before the timed region.
The roofline object covers the dominant kernel of the step, timed with HIP
events on the stream it is launched on; its algorithmic work comes from the
oracle's counts (tests/golden/work_counts_<workload>.json).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s at 1080p with 500k Gaussians; batched stereo views/s; backward ms/view"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X vector FP32 (published)
# Algorithmic FP32 work of the compositing stage (FMA counts 2):
#   per fragment (pixel centre inside a projected quad): pixel offset (4),
#   quad-plane map (6), den (4), q (3), den^2 + q/c^2 (3), reciprocal (1),
#   D (1), exponent (2), exp2 (1)                                  -> 25
#   per composited fragment: clamp, 1 - a, T (1 - a), T a, colour (3 FMA) -> 10
FLOP_PER_FRAGMENT = 25
FLOP_PER_CONTRIBUTION = 10
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
    ap.add_argument("--steps", type=int, default=160)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="c1", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--mip", default="approx", choices=["approx", "exact"],
                    help="c2: the approximate MIP of eq. 17 (the paper's renderer) or the exact per-ray MIP; "
                         "c3: exact turns the exact per-ray MIP on (the workload has none)")
    ap.add_argument("--divergence", default="ray", choices=["ray", "gs"],
                    help="c1: the ray-based divergence (the paper's renderer) or the linearised one of 3DGS")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of HIP-graph replays")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-steps", type=int, default=32, help="frames of the per-stage timing pass")
    ap.add_argument("--tile", default="8x16", help="tile shape WxH, each of 8, 16, 32")
    ap.add_argument("--no-autotune", action="store_true",
                    help="c4: use --tile instead of the training autotuner (for profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for HBM counters)")
    return ap.parse_args()


def tile_opts(args):
    tw, th = (int(v) for v in args.tile.lower().split("x"))
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
    """HBM bytes per launch of the compositing kernel from the committed
    counter summary (profiles/), or None when there is none for this
    workload or the kernel's sources changed since it was taken."""
    if stage != "blend":
        return None
    from paper_2503_18682_amd.prof_summary import read_traffic

    return read_traffic(os.path.join(ROOT, "profiles", f"blend_{workload}_pmc_traffic.txt"), "k_blend")


def roofline_for(stage, ms, *, flops=None, nbytes=None, traffic=None):
    if stage.startswith("blend"):
        achieved = flops / (ms * 1e-3) / 1e12 if flops else None
        return {"bound": "alu", "kernel": stage, "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS if achieved else None, "traffic": traffic,
                "avg_ms": ms, "algorithmic_flop": flops}
    achieved = nbytes / (ms * 1e-3) / 1e9 if nbytes else None
    return {"bound": "hbm", "kernel": stage, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": None, "avg_ms": ms,
            "algorithmic_bytes": nbytes}


def cpu_baseline_c1(scene, cam, opts):
    """The oracle on a bounded sample of one 1080p frame: the full per-Gaussian
    stage plus 8 bands of 6 rows spread over the image, scaled to a frame."""
    import oracle

    threads = os.cpu_count() or 1
    t = time.perf_counter()
    oracle.render(scene, cam, opts, rows=(0, 0), threads=threads)
    t_fixed = time.perf_counter() - t
    H = cam["height"]
    band, rows_done, t_rows = 6, 0, 0.0
    for b in range(8):
        a = int((b + 0.5) * H / 8) - band // 2
        t = time.perf_counter()
        oracle.render(scene, cam, opts, rows=(a, a + band), threads=threads)
        t_rows += max(time.perf_counter() - t - t_fixed, 0.0)
        rows_done += band
    frame_s = t_fixed + t_rows * H / rows_done
    return {"value": 1.0 / frame_s, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"pose 0: full per-Gaussian stage + {rows_done} of {H} rows (8 bands), scaled to one frame"}


def bench_c1(args, torch):
    import scenegen
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c1")
    sc, cams, opts = w["scene"], w["cameras"], dict(w["options"], **tile_opts(args))
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
    log(f"c1: {n} Gaussians, 16 poses, max instances {need}, capacity {capacity}")
    br = R.BatchRenderer(r, n, sc["sh_degree"], [cams[0]], capacity, options=opts)

    def step(k):
        if args.eager:
            r.render_into(g, [cams[k % 16]], br.outs, br.ws, opts)
        else:
            br.launch(g, [cams[k % 16]])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ok, _ = br.status()
    assert ok, "instance capacity overflow in the timed region"
    ms = (t1 - t0) * 1e3 / args.steps
    stages, frames = stage_pass(r, g, lambda k: [cams[k % 16]], opts, br.ws, br.outs, args.stage_steps)
    wc = work_counts("c1_gs" if gs else "c1")
    fwd = {k: v for k, v in stages.items() if not k.endswith("backward")}
    dom = max(fwd, key=fwd.get)
    flops = nbytes = None
    if wc:
        vs = wc["views"]
        per = [vs[k % 16] for k in range(args.stage_steps)]
        frag = np.mean([v["fragments"] for v in per])
        contrib = np.mean([v["contributions"] for v in per])
        vis = np.mean([v["visible"] for v in per])
        inst = np.mean([v["instances"] for v in per])
        flops = FLOP_PER_FRAGMENT * frag + FLOP_PER_CONTRIBUTION * contrib
        nbytes = {"preprocess": PARAM_BYTES[3] * n + RECORD_BYTES * vis,
                  "tile_sort": 2 * 2 * INSTANCE_BYTES * inst}.get(dom)
    tag = "c1_1080p_500k_" + args.tile + ("_gs" if gs else "")
    roof = roofline_for(dom, fwd[dom], flops=flops, nbytes=nbytes, traffic=pmc_traffic(dom, tag))
    # measured ceilings of this device (context for `peak`, which stays the published figure)
    calib = r.calibrate()
    if roof["unit"] == "TFLOP/s" and roof["achieved"]:
        roof["attainable_peak"] = calib["fma_tflops"]
        roof["attainable_frac"] = roof["achieved"] / calib["fma_tflops"]
    res = {
        "metric": METRIC, "value": 1e3 / ms, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c1: 500k Gaussians (64 clusters, SH3), 1920x1080, 50deg FOV, 16 orbit poses"
                   + (" (linearised GS divergence)" if gs else ""),
                   "n_gaussians": n, "width": 1920, "height": 1080, "tile": args.tile,
                   "launch": "eager" if args.eager else "hip_graph", "instance_capacity": capacity},
        "roofline": roof,
        "calibration": calib,
        "stages_ms": stages,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_c1(sc, cams[0], opts)
    return res


def bench_c2(args, torch):
    import scenegen
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c2")
    sc, cams, opts = w["scene"], w["cameras"], dict(w["options"], **tile_opts(args))
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
    assert br.status()[0]
    ms = (t1 - t0) * 1e3 / args.steps
    # 8 plain single-view renders
    singles = []
    for c in cams:
        _, (b1, w1) = r.render(g, [c], opts, keep_workspace=True)
        singles.append((b1, w1, r.allocate_outputs([c])))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(args.steps // 4, 2)):
        for c, (b1, w1, o1) in zip(cams, singles):
            r.render_into(g, [c], o1, w1, opts)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / max(args.steps // 4, 2)
    stages, _ = stage_pass(r, g, lambda k: cams, opts, br.ws, br.outs, max(args.stage_steps // 4, 4))
    fwd = {k: v for k, v in stages.items() if not k.endswith("backward")}
    dom = max(fwd, key=fwd.get)
    return {
        "metric": METRIC, "value": 8e3 / ms, "unit": "views/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c2: 3M Gaussians, 4 stereo pairs (8 views), MIP on, one HIP-graph replay"
                   + (" (exact per-ray MIP)" if args.mip == "exact" else ""),
                   "views": [[c["width"], c["height"]] for c in cams], "instance_capacity": capacity},
        "plain_launches_views_per_s": 8e3 / plain_ms,
        "roofline": roofline_for(dom, fwd[dom]),
        "stages_ms": stages,
    }


def bench_c3(args, torch):
    import scenegen
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c3")
    sc, cams, opts = w["scene"], w["cameras"], dict(w["options"], **tile_opts(args))
    if args.mip == "exact":
        opts["mip"] = 2
    n = int(sc["opacity_logits"].shape[0])
    g = to_dev(sc, torch)
    targets = [torch.from_numpy(t).cuda() for t in w["targets"]]
    r = R.Renderer(0, opts)
    _, (buf, ws) = r.render(g, cams, opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    need = r.status(ws)[1]
    del buf
    capacity = int(need * 1.1) + 4096
    buf, ws = r.new_workspace(n, cams, capacity, _lib.RGS_WS_BACKWARD, opts)
    outs = r.allocate_outputs(cams)
    grads = {k: torch.zeros_like(g[k]) for k in R.PARAM_KEYS}
    total = sum(t.numel() for t in targets)
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
    steps = max(args.steps // 4, 4)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        ev[2].synchronize()
        bwd += ev[1].elapsed_time(ev[2])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    r.stage_times()  # reset
    r.set_stage_timing(True)
    for _ in range(4):
        step()
    torch.cuda.synchronize()
    stages, frames = r.stage_times()
    r.set_stage_timing(False)
    stages = {k: v / max(frames, 1) for k, v in stages.items()}
    bstages = {k: v for k, v in stages.items() if k.endswith("backward")}
    dom = max(bstages, key=bstages.get)
    return {
        "metric": METRIC, "value": bwd / steps / len(cams), "unit": "backward ms/view", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c3: 1M Gaussians (SH3), 4 views 1600x1060, forward + L1 + backward"
                   + (" (exact per-ray MIP)" if args.mip == "exact" else ""),
                   "instance_capacity": capacity},
        "roofline": roofline_for(dom, bstages[dom]),
        "stages_ms": stages,
    }


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
        opts, tile_from = dict(opts0, **tile_opts(args)), "--tile"
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
    res = {"c1": bench_c1, "c2": bench_c2, "c3": bench_c3, "c4": bench_c4}[args.workload](args, torch)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
