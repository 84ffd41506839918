"""Mapping-iteration benchmark of the HIP rasterizer on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--tile 16x16]

One step = one mapping iteration over the workload's views: forward render
(projection, binning, depth-keyed radix sort, compositing), L1 colour +
0.5 L1 depth loss against a target rendered from perturbed parameters,
backward to the parameters (and Adam where the workload includes it). The
inputs are resident in HBM before the timed region. Prints one JSON line.

--mode graph (default) replays the whole iteration as one HIP graph
(gsr_mapping_iteration); --mode eager issues the entry points one view at a
time (render, loss, backward per view, then Adam). The other mode is timed
too, after the headline, and reported in config for comparison.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mapping iters/sec (fwd+bwd) 640x480, 200k Gaussians; render Mpix/s"
ADAM_WORKLOADS = {"surfaces_1200x680_1M_sh3", "mixed16_2M_sh3"}

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue 39.3e12 FP32 VALU lane
# instructions per second without packed FP32 math (which the library's
# kernels are compiled not to emit). AMD's published 157.3 TFLOP/s FP32 vector
# figure counts a packed FMA (two lanes' FMAs in one instruction) as four
# FLOPs: 256 x 64 x 2 x 2 x 2.4e9.
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_FP32_PUBLISHED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic work per (pixel, Gaussian) pair walked, in two countings.
#  Issue slots (the roofline's unit): one per VALU lane instruction, the
#  transcendentals (exp, rcp) counted as 4 for their quarter issue rate.
#   backward 59: the alpha 20 (exponent in its definition's float order 10,
#     scaling by log2 e 1, exp 4, opacity, clamp and skip tests 5), the reverse
#     step 29 (rcp 4), the wave sums of the ten per-Gaussian moments 10 (63
#     adds per 64 lanes each);
#   backward, row form 50 (one pixel per thread, tiles 16 or 32 wide: each
#     16-lane row is one image row, so the dy factors and the opacity apply
#     to row sums): the alpha 20, the reverse step 23, seven wave sums 7;
#   forward 23: the alpha 20 and the transmittance test and update 3 (the
#     colour and depth accumulation happens once per composited pair).
#  Plain operations (each FP32 operation once, exp and rcp included), for
#  the published FLOP figure: backward 53 (row form 44), forward 20.
OPS_PER_PAIR_BWD = 59.0
OPS_PER_PAIR_BWD_ROW = 50.0
OPS_PER_PAIR_FWD = 23.0
PLAIN_OPS_PER_PAIR_BWD = 53.0
PLAIN_OPS_PER_PAIR_BWD_ROW = 44.0
PLAIN_OPS_PER_PAIR_FWD = 20.0
# The fused launch (forward and backward of every tile in one grid) is
# credited with both per pair walked by the backward; the forward's pairs
# past each pixel's last composited Gaussian are not counted.


def ops_per_pair_for(kernel, tile_w, ppt):
    """(issue slots, plain operations) per pair walked of the blend kernel."""
    row = ppt == 1 and tile_w % 16 == 0
    bwd = OPS_PER_PAIR_BWD_ROW if row else OPS_PER_PAIR_BWD
    pbwd = PLAIN_OPS_PER_PAIR_BWD_ROW if row else PLAIN_OPS_PER_PAIR_BWD
    return {"blend_fwd": (OPS_PER_PAIR_FWD, PLAIN_OPS_PER_PAIR_FWD), "blend_bwd": (bwd, pbwd),
            "blend": (OPS_PER_PAIR_FWD + bwd, PLAIN_OPS_PER_PAIR_FWD + pbwd)}[kernel]


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (profiles/mapping_iteration_<workload>.txt), each scaled by what
# the counter reads for a 256 MiB device copy (FETCH x2.0, WRITE x1.0), for
# the launch configuration profiled there (16x16 tiles, one pixel per
# thread, the default batch depth). An entry is removed whenever its kernel
# changes.
TRAFFIC = {
    ("keyframe_640x480_200k", "blend"): (77.689e6, 84.883e6),   # read, write
    ("batch8_640x480_500k", "blend_bwd"): (639.321e6, 815.010e6),
    ("mixed16_2M_sh3", "blend_bwd"): (1425.186e6, 1915.826e6),
}
PROFILED_CONFIG = (16, 16, 1, 0)   # tile_w, tile_h, pixels per thread, batch depth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="keyframe_640x480_200k")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--ppt", type=int, default=0, help="pixels per thread in the blend kernels (0 = default)")
    ap.add_argument("--batch-depth", type=int, default=0, help="backward batch depth (0 = default)")
    ap.add_argument("--chunk-len", type=int, default=0,
                    help="backward work unit in list positions (0 = automatic, -1 = whole tile lists)")
    ap.add_argument("--max-chunks", type=int, default=0, help="backward chunks per tile (0 = default)")
    ap.add_argument("--depth-sort", type=int, default=0,
                    help="0 = automatic, 1 = per tile after binning, 2 = once over all splats before binning")
    ap.add_argument("--fuse-blend", type=int, default=0,
                    help="graph mode: 0 = automatic, 1 = blend forward and backward in one launch, -1 = two launches")
    ap.add_argument("--tile-order", type=int, default=0,
                    help="0 = automatic, 1 = longest tile lists first, 2 = tile order, 3 = balanced over the CUs")
    ap.add_argument("--backward-schedule", type=int, default=0,
                    help="blend backward: 0 = pixel-parallel, 1 = splat-parallel (whole lists, two blend launches)")
    ap.add_argument("--binning", type=int, default=0,
                    help="instances by tile: 0 = automatic (blocks of tiles where the per-tile depth order "
                         "applies, else a radix sort of tile keys), 1 = counting, 2 = radix sort of tile keys, "
                         "3 = blocks of tiles")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --tile/--ppt/--batch-depth instead of the autotuner's choice")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the achievable-peak probes")
    ap.add_argument("--breakdown", action="store_true", help="print a per-stage time breakdown to stderr")
    ap.add_argument("--mode", choices=["graph", "eager"], default="graph")
    ap.add_argument("--compare-steps", type=int, default=20, help="steps of the other mode (0 = skip)")
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, cams, targets_np, repeats=3, single_row_step=8):
    """The CPU oracle as it stands: one mapping iteration (FP32 brute-force
    forward, L1 loss, FP64 analytic backward) of the workload's first view.
    All cores: the median of `repeats` whole iterations. One thread: the median
    of `repeats` iterations over every single_row_step-th pixel row (forward
    and backward restricted to those rows), extrapolated to the whole view."""
    import numpy as np
    import oracle
    cores = oracle.set_threads(0)
    cam = cams[0]

    def one(window):
        t0 = time.perf_counter()
        r = oracle.render(scene.params, scene.sh_degree, cam, mode="f32", window=window)
        L, grgb, gdep = oracle.l1_loss_and_grad(r["rgb"], r["depth"], targets_np[0][0], targets_np[0][1])
        oracle.backward(scene.params, scene.sh_degree, [cam],
                        [(grgb.astype(np.float32), gdep.astype(np.float32), np.zeros_like(gdep, np.float32))],
                        pinned=True, windows=[window])
        return time.perf_counter() - t0

    t_all = sorted(one(None) for _ in range(repeats))[repeats // 2]
    oracle.set_threads(1)
    win = (0, 0, cam.width, cam.height, single_row_step)
    rows = len(range(0, cam.height, single_row_step))
    t_one = sorted(one(win) for _ in range(repeats))[repeats // 2] * cam.height / rows
    oracle.set_threads(cores)
    return {"value": round(1.0 / t_all, 5), "unit": "iters/s", "cores": cores, "kind": "oracle",
            "single_thread_value": round(1.0 / t_one, 6), "single_thread_extrapolated": True,
            "cpu_model": cpu_model(),
            "sample": f"one mapping iteration (FP32 brute-force forward, L1 loss, FP64 analytic backward) of view 0 "
                      f"of {scene.name}, {cam.width}x{cam.height}, {scene.num} Gaussians; median of {repeats} on "
                      f"{cores} threads ({t_all:.2f} s); one thread: median of {repeats} over every "
                      f"{single_row_step}th pixel row, extrapolated to the view ({t_one:.1f} s)"}


def binning_used(R, num, cams):
    """The binning the library chooses for this rasterizer and workload (its
    rule: blocks of tiles, at most 8x8 and 256 over all views, for the
    per-tile depth order; counting where asked; else the radix sort)."""
    per_tile = R.depth_sort == 1 or (R.depth_sort == 0 and num * len(cams) <= 2 ** 19)
    if per_tile and R.binning == 1:
        return "counting"
    if per_tile and R.binning in (0, 3):
        tiles = [((c.width + R.tile_w - 1) // R.tile_w, (c.height + R.tile_h - 1) // R.tile_h) for c in cams]
        for area in range(7):
            nb = {w: sum(((tx + (1 << w) - 1) >> w) * ((ty + (1 << (area - w)) - 1) >> (area - w))
                         for tx, ty in tiles) for w in range(4) if 0 <= area - w <= 3}
            fits = [w for w, n in nb.items() if n <= 256]
            if fits:
                if area == 0 and R.binning == 0:
                    break                           # single-tile blocks: automatic takes the radix path
                w = min(fits, key=lambda w: (abs(2 * w - area), nb[w]))
                h = area - w
                return f"blocks of {1 << w}x{1 << h} tiles, one pass over block ids, per-tile filter and depth sort"
    return "radix sort of tile keys"


def achievable_peaks():
    """The device's achievable rates from the library's probe kernels
    (include/gsr_peaks.h): HBM copy, FP32 VALU issue, the 2^x rate, LDS reads."""
    import ctypes
    from paper_2509_06433_amd import _lib
    L = _lib.load()
    out = {}
    d = ctypes.c_double()
    for name, fn, args, scale, unit in (
            ("hbm_copy", L.gsr_peak_copy, (2 << 30, 20), 1e-9, "GB/s"),
            ("valu_fp32", L.gsr_peak_valu, (20,), 1e-12, "T lane-instr/s"),
            ("exp2", L.gsr_peak_exp, (20,), 1e-12, "T lane-ops/s"),
            ("lds_read", L.gsr_peak_lds, (20,), 1e-12, "TB/s")):
        rc = fn(*args, None, ctypes.byref(d))
        out[name] = {"value": round(d.value * scale, 3) if rc == 0 else None, "unit": unit}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by view)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import scenes
    from paper_2509_06433_amd.rasterize import Rasterizer

    tw, th = (int(x) for x in args.tile.split("x"))
    scene = scenes.WORKLOADS[args.workload]()
    cams = scene.cameras
    deg = scene.sh_degree
    R = Rasterizer(tile_w=tw, tile_h=th, pixels_per_thread=args.ppt, batch_depth=args.batch_depth,
                   tile_order=args.tile_order, chunk_len=args.chunk_len, max_chunks=args.max_chunks,
                   fuse_blend=args.fuse_blend, depth_sort=args.depth_sort, backward_schedule=args.backward_schedule,
                   binning=args.binning)
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    params = torch.from_numpy(scene.params).to(dev)
    forward_only = scene.target_params is None
    if forward_only:
        targets = None
    else:
        tparams = torch.from_numpy(scene.target_params).to(dev)
        targets = [tuple(t.clone() for t in o) for o in R.render(tparams, deg, cams)]
        del tparams
    outs = R.alloc_images(cams, dev)
    gimgs = [(torch.empty_like(o[0]), torch.empty_like(o[1]), torch.zeros_like(o[2])) for o in outs]
    loss = torch.zeros(1, device=dev)
    grad = torch.zeros_like(params)
    params0 = params.clone()
    use_adam = args.workload in ADAM_WORKLOADS
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    P = params.shape[0]
    lrs = [1.6e-4] * 3 + [5e-3] * 3 + [1e-3] * 4 + [5e-2] + [2.5e-3] * 3 + [1.25e-4] * (P - 14)
    tuned = None
    if not args.no_autotune and not forward_only:
        from paper_2509_06433_amd import autotune
        tuned = autotune.tune(params, deg, cams, targets, 0.5, lrs if use_adam else None,
                              log=(lambda msg: print(msg, file=sys.stderr)) if args.breakdown else None)
        R.close()
        R = Rasterizer(tile_w=tuned["tile_w"], tile_h=tuned["tile_h"], pixels_per_thread=tuned["pixels_per_thread"],
                       batch_depth=tuned["batch_depth"], tile_order=args.tile_order, chunk_len=tuned["chunk_len"],
                       max_chunks=tuned["max_chunks"], fuse_blend=args.fuse_blend, depth_sort=args.depth_sort,
                       backward_schedule=args.backward_schedule, binning=args.binning)
        outs = R.alloc_images(cams, dev)
    from paper_2509_06433_amd import _lib
    adam = dict(m=m, v=v, lr=lrs, beta1=0.9, beta2=0.999, eps=1e-15) if use_adam else None

    def graph_step(it):
        if adam is not None:
            adam["step"] = 1 if it == 1 else 0
        R.mapping_iteration(params, deg, cams, outs, targets, grad, 0.5, loss, adam)

    def eager_step(it):
        grad.zero_()
        for view, cam in enumerate(cams):
            R.render(params, deg, [cam], [outs[view]])
            _lib.gsr_loss_l1(R.handle, [cam], [outs[view]], [targets[view]], [gimgs[view]], 0.5, loss)
            R.render_backward(params, deg, [cam], [gimgs[view]], grad)
        if use_adam:
            R.adam_step(params, grad, m, v, lrs, it)

    def render_step(it):
        R.render(params, deg, cams, outs)

    steps = {"graph": graph_step, "eager": eager_step}
    if forward_only:          # a render-only workload: both modes time the forward
        steps = {"graph": render_step, "eager": render_step}
    # the blend backward, or the fused blend launch when the iteration uses it
    candidates = ["blend_fwd"] if forward_only else ["blend_bwd", "blend"]

    def timed(mode, n_steps, n_warm, profile):
        """Warm up, then time n_steps; returns (ms per step, {stage: (ms, launches)})."""
        fn = steps[mode]
        R.set_profiling(candidates if profile else [])
        it0 = timed.it
        for _ in range(n_warm):
            timed.it += 1
            fn(timed.it - it0)
        torch.cuda.synchronize()
        R.profile(reset=True)
        t0 = time.perf_counter()
        for _ in range(n_steps):
            timed.it += 1
            fn(timed.it - it0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) * 1e3 / max(n_steps, 1), R.profile(reset=True)

    timed.it = 0
    ms_per_step, prof = timed(args.mode, args.steps, args.warmup, True)
    dominant = max(candidates, key=lambda k: prof[k][1])
    dom_ms, dom_n = prof[dominant]
    if args.mode == "graph":
        mst = R.mapping_status()
        if mst["skipped"]:
            print(f"warning: {mst['skipped']} iterations skipped for instance overflow", file=sys.stderr)
    pairs, visible = R.count_work(len(cams))
    dom_avg_ms = dom_ms / max(args.steps, 1)     # one launch per step in graph mode
    traffic_known = ((scene.name, dominant) in TRAFFIC and
                     (R.tile_w, R.tile_h, R.pixels_per_thread or 1, R.batch_depth) == PROFILED_CONFIG)
    ops_per_pair, plain_per_pair = ops_per_pair_for(dominant, R.tile_w, R.pixels_per_thread or 1)
    achieved = ops_per_pair * pairs / (dom_avg_ms * 1e-3) / 1e12
    achieved_plain = plain_per_pair * pairs / (dom_avg_ms * 1e-3) / 1e12

    other = "eager" if args.mode == "graph" else "graph"
    other_ms = None
    if args.compare_steps > 0:
        params.copy_(params0)
        m.zero_()
        v.zero_()
        timed.it = 0
        other_ms, _ = timed(other, args.compare_steps, 2, False)

    # per-stage breakdown (separate, untimed pass)
    params.copy_(params0)
    m.zero_()
    v.zero_()
    R.set_profiling(None)
    for k in range(4):
        steps[args.mode](k + 1)
        if k == 0:
            torch.cuda.synchronize()
            R.profile(reset=True)
    torch.cuda.synchronize()
    stages = {k: ms / 3 for k, (ms, n) in R.profile(reset=True).items() if n}     # ms per step
    R.set_profiling([])
    # the whole forward: the clear, projection, binning, both sorts, ranges, compositing
    front = ["zero", "project", "depth_sort", "scan", "emit", "tile_sort", "ranges", "tile_depth", "blend_fwd"]
    render_ms = sum(stages.get(k, 0.0) for k in front) if "blend_fwd" in stages else 0.0
    render_from = "iteration stages"
    if "blend_fwd" not in stages and "blend" in stages and args.mode == "graph":
        # the fused blend launch gives the forward no time of its own: the
        # render rate comes from a few replays of the same iteration in two
        # blend launches (same kernels up to the forward)
        R2 = Rasterizer(tile_w=R.tile_w, tile_h=R.tile_h, pixels_per_thread=R.pixels_per_thread,
                        batch_depth=R.batch_depth, tile_order=R.tile_order, chunk_len=R.chunk_len,
                        max_chunks=R.max_chunks, fuse_blend=-1, depth_sort=R.depth_sort, binning=R.binning)
        outs2 = R2.alloc_images(cams, dev)
        p2 = params0.clone()
        g2 = torch.zeros_like(p2)
        R2.set_profiling(None)
        for k in range(4):
            R2.mapping_iteration(p2, deg, cams, outs2, targets, g2, 0.5, loss, None)
            if k == 0:
                torch.cuda.synchronize()
                R2.profile(reset=True)
        torch.cuda.synchronize()
        st2 = {k: ms / 3 for k, (ms, n) in R2.profile(reset=True).items() if n}
        render_ms = sum(st2.get(k, 0.0) for k in front)
        render_from = "two-launch replays of the iteration (the fused launch has no forward time of its own)"
        R2.close()
        del outs2, p2, g2
    pix = sum(c.width * c.height for c in cams)
    mpix = pix / (render_ms * 1e-3) / 1e6 if render_ms > 0 else None
    st = R.status()
    if args.breakdown:
        print(json.dumps({"stage_ms": stages, "instances": st["instances"], "pairs": pairs, "visible": visible},
                         indent=1), file=sys.stderr)

    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms_per_step, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": scene.name, "views": len(cams),
                   "resolutions": sorted({f"{c.width}x{c.height}" for c in cams}),
                   "gaussians": scene.num, "sh_degree": deg, "tile": f"{R.tile_w}x{R.tile_h}",
                   "pixels_per_thread": R.pixels_per_thread or 1, "batch_depth": R.batch_depth or "default",
                   "chunk_len": {0: "auto", -1: "whole list"}.get(R.chunk_len, R.chunk_len),
                   "max_chunks": R.max_chunks or "default",
                   "blend_launch": "fused" if dominant == "blend" else "separate",
                   "backward_schedule": ["pixel-parallel", "splat-parallel"][R.backward_schedule],
                   "binning": binning_used(R, scene.num, cams),
                   "autotuned": tuned is not None, "tile_order": ["auto", "longest first", "index", "balanced"][R.tile_order],
                   "adam": use_adam, "mode": args.mode,
                   f"{other}_iters_s": round(1000.0 / other_ms, 3) if other_ms else None,
                   "render_mpix_s": round(mpix, 2) if mpix else None, "render_mpix_s_from": render_from,
                   "instances": st["instances"], "visible_per_view": visible,
                   "stage_ms": {k: round(x, 4) for k, x in stages.items()}},
        "roofline": {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 3),
                     "peak": round(PEAK_VALU_TOPS, 2), "unit": "T issue slots/s (FP32 VALU lane instructions)",
                     "frac": round(achieved / PEAK_VALU_TOPS, 4),
                     "peak_derivation": "256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, non-packed FP32 issue; "
                                        f"{ops_per_pair:g} slots per pair walked (exp and rcp 4 each)",
                     "achieved_plain_tflops": round(achieved_plain, 3),
                     "frac_published": round(achieved_plain / PEAK_FP32_PUBLISHED_TFLOPS, 4),
                     "published_peak": f"{PEAK_FP32_PUBLISHED_TFLOPS} TFLOP/s FP32 vector (packed FMA as 4 FLOPs); "
                                       f"{plain_per_pair:g} plain FP32 ops per pair",
                     "traffic": (round(sum(TRAFFIC[(scene.name, dominant)])) if traffic_known else None),
                     "traffic_read_write": TRAFFIC.get((scene.name, dominant)) if traffic_known else None,
                     "avg_ms": round(dom_avg_ms, 4), "launches": dom_n, "pairs": pairs,
                     "ops_per_pair": ops_per_pair},
    }
    if not args.no_peaks:
        peaks = achievable_peaks()
        out["roofline"]["achievable"] = peaks
        v = peaks["valu_fp32"]["value"]
        if v:
            out["roofline"]["frac_achievable"] = round(achieved / v, 4)
    if not args.no_cpu_baseline and not forward_only:
        tnp = [(t[0].cpu().numpy(), t[1].cpu().numpy()) for t in targets]
        out["cpu_baseline"] = cpu_baseline(scene, cams, tnp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
