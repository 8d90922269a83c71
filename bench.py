#!/usr/bin/env python3
"""Benchmark of the batched mapping step on one MI355X.

Workload (the batched mapping step the paper's renderer runs every
iteration, DROID-Splat Sec. 3.3 and supplementary S1.2): 500k Gaussians with
SH degree 3, 8 keyframes at 1200x680 (f = 600) on a smooth trajectory,
forward + summed L1 RGB + L1 depth loss + backward (all Gaussian gradients and
the pose twists), FP32.  Synthetic scene (seeded, shaped like the paper's
Replica/TUM maps); targets are renders of the unperturbed means.

Reports forward+backward Mpixels/s of the batched launch, the same work as
one launch sequence per frame (batched vs per-frame speedup), per-stage GPU
time from HIP events recorded on the library's stream inside the timed
region, the roofline position of the dominant kernel, and the FP64 CPU
oracle timed on a bounded sample (the keyframes one at a time, at most ~25 s) on the
host cores.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic cost per evaluated (pixel, entry) pair of the compositing
# kernels (FP32 operations counted from the method's arithmetic):
# forward 27 flops + 1 exp, backward 60 flops + 1 exp + 1 rcp.
FLOPS_PER_PAIR = {"composite_fwd": 27.0, "composite_bwd": 60.0}
# 2D surfels, per evaluated (pixel, surfel) pair, counted from the kernels'
# source (an FMA counts 2): the intersection (pixel offsets, h_u, h_v, their
# cross product, a Newton-refined reciprocal, u, v, G, G_lp, depth) is 42
# flops and three exp/rcp; blending with the normal and the distortion sums
# adds 33 in the forward; the backward re-evaluates the intersection and
# adds ~130 (T recovery, the FP64 behind-state, dL/dalpha, the chain through
# p = h_u x h_v and the 18 per-key sums).
SURFEL_FLOPS_PER_PAIR = {"fwd": 75.0, "bwd": 170.0}
PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X fp32 vector (published)
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tile", default="auto", help="WxH or 'auto' (autotuner's choice of tile "
                    "shape and LDS batch)")
    ap.add_argument("--lds-batch", type=int, default=64, help="with --tile WxH: 32, 64 or 128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-frame", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--copy-kernel", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.copy_kernel:
        import torch
        n = args.copy_kernel // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty(n, device="cuda")
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": 3}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU; the rasterizer shards over keyframes "
              "across GPUs only by design (no multi-GPU path is built), so --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_17660_amd import scenes
    from paper_2411_17660_amd.raster import Rasterizer

    t0 = time.time()
    sc = scenes.scene_c3(n=args.n)
    log(f"[bench] scene generated in {time.time() - t0:.1f}s: n={sc.n} frames={sc.n_frames}")
    dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k), np.float32)).cuda()
           for k in ("means", "log_scales", "quats", "opacity", "sh", "poses")}
    gt_means = torch.from_numpy(sc.extra["gt_means"]).cuda()
    P = sc.n_pixels
    F = sc.n_frames
    W, H = sc.cams[0][:2]
    depth_weight = 1.0
    rast = Rasterizer(0)
    # targets: render of the ground-truth means (workload set-up, untimed)
    t_rgb, t_dep, _ = rast.forward(gt_means, dev["log_scales"], dev["quats"], dev["opacity"],
                                   dev["sh"], dev["poses"], sc.cams, 3)
    t_rgb, t_dep = t_rgb.clone(), t_dep.clone()
    torch.cuda.synchronize()
    tune = None
    if args.tile == "auto":
        tile, batch, _, times = rast.autotune(dev["means"], dev["log_scales"], dev["quats"],
                                              dev["opacity"], dev["sh"], dev["poses"], sc.cams,
                                              3, t_rgb, t_dep, depth_weight, reps=3, force=True)
        tune = {f"{w}x{h}/{b}": round(ms, 3) for ((w, h), b), ms in times.items()}
        log(f"[bench] autotune: {tune} -> {tile} x {batch}")
    else:
        tile = tuple(int(v) for v in args.tile.split("x"))
        batch = args.lds_batch

    def buffers(n_frames_px, nF):
        K = (sc.sh_degree + 1) ** 2
        n = sc.n
        return dict(rgb=torch.empty(3 * n_frames_px, device="cuda"),
                    depth=torch.empty(n_frames_px, device="cuda"),
                    alpha=torch.empty(n_frames_px, device="cuda"),
                    loss=torch.empty(1, device="cuda"), means=torch.empty(n, 3, device="cuda"),
                    log_scales=torch.empty(n, 3, device="cuda"),
                    quats=torch.empty(n, 4, device="cuda"), opacity=torch.empty(n, device="cuda"),
                    sh=torch.empty(n, K, 3, device="cuda"), twist=torch.empty(nF, 6, device="cuda"))

    def step(r, cams, poses, trgb, tdep, bufs, cap, timing=False):
        r.step_l1(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                  poses, cams, 3, trgb, tdep, depth_weight, bufs, tile=tile, key_capacity=cap,
                  timing=timing, lds_batch=batch)

    # ---------------- batched: one launch sequence for all 8 frames
    bb = buffers(P, F)
    step(rast, sc.cams, dev["poses"], t_rgb, t_dep, bb, 0)
    torch.cuda.synchronize()
    K = rast.stats()["n_keys"]
    cap = int(K * 1.05) + 1024  # fixed capacity: no host read inside the step
    log(f"[bench] K={K} keys per step; capacity {cap}")
    for _ in range(args.warmup):
        step(rast, sc.cams, dev["poses"], t_rgb, t_dep, bb, cap)
    torch.cuda.synchronize()
    # eager steps with the library's per-stage HIP events (stage times, the
    # roofline's kernel duration)
    rast.timings()  # drop anything recorded so far
    t_eager = median_event_ms(
        lambda: step(rast, sc.cams, dev["poses"], t_rgb, t_dep, bb, cap, timing=True),
        args.steps)
    rast.check_overflow()
    stages = rast.timings()
    loss = bb["loss"].item()
    log(f"[bench] eager batched {t_eager:.3f} ms/step (median), loss {loss:.5f}")

    # the headline: the same step captured as one HIP graph, warmed up, then
    # exactly `steps` replays between two synchronisations, each bracketed by
    # HIP events on the stream it runs on; the median replay is the step time
    t_graph = t_wall = None
    try:
        if args.no_graph:
            raise RuntimeError("graph replay disabled by --no-graph")
        graph = capture(lambda: step(rast, sc.cams, dev["poses"], t_rgb, t_dep, bb, cap))
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_graph = median_event_ms(graph.replay, args.steps, sync=False)
        torch.cuda.synchronize()
        t_wall = (time.perf_counter() - t0) * 1e3 / args.steps
        rast.check_overflow()
        log(f"[bench] graph-replayed batched {t_graph:.3f} ms/step (median of {args.steps}; "
            f"wall mean {t_wall:.3f})")
        del graph
    except Exception as e:  # reported, never silently substituted
        log(f"[bench] graph capture failed: {e!r}")

    # evaluated (pixel, entry) pairs of one forward (separate counting pass)
    rast.forward(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                 dev["poses"], sc.cams, 3, tile=tile, key_capacity=cap, count_pairs=True,
                 lds_batch=batch)
    pairs = rast.stats()["n_pairs"]
    log(f"[bench] evaluated pairs per forward {pairs}")

    # ---------------- per-frame: the same work, one launch sequence per frame
    per_frame = None
    if not args.no_per_frame:
        per_frame = measure_per_frame(sc, dev, t_rgb, t_dep, tile, batch, depth_weight,
                                      args.steps, args.warmup)
        log(f"[bench] per-frame {per_frame}")

    # ---------------- the paper's full rendering loss (L1 + SSIM colour term)
    render = measure_render_loss(rast, sc, dev, bb, t_rgb, t_dep, tile, cap, args.steps)
    median = measure_median(rast, sc, dev, bb, t_rgb, t_dep, tile, cap, args.steps,
                            depth_weight)
    densify = measure_densify(rast, sc, dev, bb, t_rgb, t_dep, tile, cap, depth_weight)
    surfel = measure_surfel(rast, sc, dev, tile, args.steps)

    mpix = P / 1e6
    t_best = t_graph if t_graph is not None else t_eager
    value = mpix / (t_best * 1e-3)
    per_stage = {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]}
    # roofline of the dominant compositing kernel
    dom = max(("composite_fwd", "composite_bwd"), key=lambda k: stages[k][0])
    dur_ms = stages[dom][0] / max(stages[dom][1], 1)
    achieved = pairs * FLOPS_PER_PAIR[dom] / (dur_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                "traffic": measured_traffic(dom, tile),
                "avg_launch_ms": round(dur_ms, 4), "pairs_per_launch": pairs,
                "flops_per_pair": FLOPS_PER_PAIR[dom]}
    achievable = measure_copy(rast)
    sort = sort_roofline(stages, int(K), achievable)
    log(f"[bench] achievable HBM {achievable}; sort {sort}")
    del bb

    c4 = None if args.no_c4 else measure_c4(args.steps, args.warmup)
    c5 = None if args.no_c5 else measure_c5(args.steps)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, args.cpu_threads)

    speedup = speedup_eager = None
    if per_frame is not None:
        pf = per_frame["graph_ms"] if per_frame["graph_ms"] is not None else per_frame["eager_ms"]
        speedup = round(pf / t_best, 4)
        speedup_eager = round(per_frame["eager_ms"] / t_eager, 4)
    out = {
        "metric": "fwd+bwd Mpixels/s at 500k Gaussians; batched vs per-frame speedup",
        "value": round(value, 3), "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_best, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded piecewise-planar scenes shaped like the paper's maps)",
        "config": {"workload": "c3: 500k Gaussians SH3, 8 keyframes 1200x680 f=600, "
                               "fwd + L1 rgb + L1 depth + bwd incl. pose twists",
                   "n_gaussians": sc.n, "frames": F, "resolution": [W, H],
                   "tile": list(tile), "lds_batch": batch, "keys_per_step": int(K)},
        "timing": "median of the per-step HIP-event times of `steps` HIP-graph replays "
                  "after `warmup` untimed ones",
        "autotune_ms_per_tile_and_batch": tune,
        "eager_ms_per_step": round(t_eager, 4),
        "graph_ms_per_step": None if t_graph is None else round(t_graph, 4),
        "graph_wall_mean_ms_per_step": None if t_wall is None else round(t_wall, 4),
        "per_frame": per_frame,
        "batched_vs_per_frame_speedup": speedup,
        "batched_vs_per_frame_speedup_eager": speedup_eager,
        "stage_ms_per_step": per_stage,
        "loss": loss,
        "roofline": roofline,
        "sort": sort,
        "achievable_hbm": achievable,
        "c4": c4,
        "c5": c5,
        "render_loss": render,
        "median_depth": median,
        "densify": densify,
        "surfel": surfel,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def median_event_ms(fn, reps, sync=True):
    """Median over `reps` calls of fn() of the HIP-event time around each call,
    events recorded on the current stream (the one the library and graph
    replays run on)."""
    import torch
    if sync:
        torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def capture(fn):
    """fn() captured as one HIP graph (one eager call on a side stream first,
    so that every workspace buffer exists before the capture)."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def step_buffers(n, K, F, P):
    import torch
    return dict(rgb=torch.empty(3 * P, device="cuda"), depth=torch.empty(P, device="cuda"),
                alpha=torch.empty(P, device="cuda"), loss=torch.empty(1, device="cuda"),
                means=torch.empty(n, 3, device="cuda"), log_scales=torch.empty(n, 3, device="cuda"),
                quats=torch.empty(n, 4, device="cuda"), opacity=torch.empty(n, device="cuda"),
                sh=torch.empty(n, K, 3, device="cuda"), twist=torch.empty(F, 6, device="cuda"))


def per_frame_setup(sc, dev, t_rgb, t_dep, tile, batch, depth_weight):
    """The batch as F single-frame steps on one context (each frame runs its
    own depth sort, scan and tile sort), each at its own fixed key capacity:
    returns the function running all F in sequence."""
    import torch
    from paper_2411_17660_amd.raster import Rasterizer
    rf = Rasterizer(0)
    K = (sc.sh_degree + 1) ** 2
    per, off = [], 0
    for f, cam in enumerate(sc.cams):
        w, h = int(cam[0]), int(cam[1])
        poses_f = dev["poses"][f:f + 1].contiguous()
        tr = t_rgb[3 * off:3 * (off + w * h)]
        td = t_dep[off:off + w * h]
        bf = step_buffers(sc.n, K, 1, w * h)
        rf.step_l1(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                   poses_f, [cam], sc.sh_degree, tr, td, depth_weight, bf, tile=tile,
                   lds_batch=batch)
        torch.cuda.synchronize()
        kf = rf.stats()["n_keys"]
        per.append(([cam], poses_f, tr, td, bf, int(kf * 1.05) + 1024))
        off += w * h

    def run():
        for (c, p, tr, td, bf, kc) in per:
            rf.step_l1(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                       p, c, sc.sh_degree, tr, td, depth_weight, bf, tile=tile, key_capacity=kc,
                       lds_batch=batch)
    return rf, run


def measure_per_frame(sc, dev, t_rgb, t_dep, tile, batch, depth_weight, steps, warmup):
    """Per-frame baseline: the same library called once per frame (F = 1),
    eager and captured as one graph of F steps; median step times."""
    import torch
    rf, run = per_frame_setup(sc, dev, t_rgb, t_dep, tile, batch, depth_weight)
    for _ in range(warmup):
        run()
    eager = median_event_ms(run, steps)
    rf.check_overflow()
    graph_ms = None
    try:
        g = capture(run)
        for _ in range(warmup):
            g.replay()
        graph_ms = median_event_ms(g.replay, steps)
        rf.check_overflow()
        del g
    except Exception as e:
        log(f"[bench] per-frame graph capture failed: {e!r}")
    torch.cuda.synchronize()
    return {"eager_ms": round(eager, 4),
            "graph_ms": None if graph_ms is None else round(graph_ms, 4)}


def measure_copy(rast, nbytes=2 << 30):
    """Achievable HBM: the library's plain 16-byte copy kernel over 2 GiB
    buffers (read 2 GiB + write 2 GiB), median of 10 launches."""
    import torch
    src = torch.ones(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    rast.debug_copy(src, dst)
    ms = median_event_ms(lambda: rast.debug_copy(src, dst), 10)
    assert bool(torch.equal(dst[:1024], src[:1024]))
    del src, dst
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return {"kernel": "copy16 (one 16-byte element per thread)", "buffer_bytes": nbytes,
            "ms": round(ms, 4), "GBps": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_HBM_GBS, 4)}


# Algorithmic HBM bytes per key of the list stages: the sort moves each
# (tile, Gaussian) pair once in and once out (12-byte pairs: 24 B); keygen
# writes the pair (12 B); the ranges read each key once (8 B).
SORT_BYTES_PER_KEY = 24
KEYGEN_BYTES_PER_KEY = 12
RANGES_BYTES_PER_KEY = 8


def sort_roofline(stages, K, achievable):
    def ms(k):
        return stages[k][0] / max(stages[k][1], 1)
    t_sort = ms("tile_sort")
    gbs = SORT_BYTES_PER_KEY * K / (t_sort * 1e-3) / 1e9
    t_all = ms("keygen") + t_sort + ms("ranges")
    b_all = (KEYGEN_BYTES_PER_KEY + SORT_BYTES_PER_KEY + RANGES_BYTES_PER_KEY) * K
    gbs_all = b_all / (t_all * 1e-3) / 1e9
    return {"bound": "hbm", "stage": "tile_sort", "keys": K,
            "algorithmic_bytes_per_key": SORT_BYTES_PER_KEY, "ms": round(t_sort, 4),
            "achieved_GBps": round(gbs, 1), "peak_GBps": PEAK_HBM_GBS,
            "frac": round(gbs / PEAK_HBM_GBS, 4),
            "frac_of_achievable": round(gbs / achievable["GBps"], 4),
            "lists": {"stages": ["keygen", "tile_sort", "ranges"],
                      "algorithmic_bytes_per_key": KEYGEN_BYTES_PER_KEY + SORT_BYTES_PER_KEY +
                      RANGES_BYTES_PER_KEY, "ms": round(t_all, 4),
                      "achieved_GBps": round(gbs_all, 1),
                      "frac": round(gbs_all / PEAK_HBM_GBS, 4),
                      "frac_of_achievable": round(gbs_all / achievable["GBps"], 4)}}


def measure_c4(steps, warmup):
    """C4: 1M Gaussians with Student-t scales, 16 keyframes of mixed
    resolution; the autotuner picks the tile; batched graph replays against
    per-frame launches (eager and graph)."""
    import torch
    from paper_2411_17660_amd import scenes
    from paper_2411_17660_amd.raster import Rasterizer
    t0 = time.time()
    sc = scenes.scene_c4()
    log(f"[bench] c4 scene in {time.time() - t0:.1f}s")
    dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k), np.float32)).cuda()
           for k in ("means", "log_scales", "quats", "opacity", "sh", "poses")}
    gt = torch.from_numpy(sc.extra["gt_means"]).cuda()
    r = Rasterizer(0)
    t_rgb, t_dep, _ = r.forward(gt, dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                                dev["poses"], sc.cams, 3)
    t_rgb, t_dep = t_rgb.clone(), t_dep.clone()
    tile, batch, cap, times = r.autotune(dev["means"], dev["log_scales"], dev["quats"],
                                         dev["opacity"], dev["sh"], dev["poses"], sc.cams, 3,
                                         t_rgb, t_dep, 1.0, reps=2, force=True)
    P = sc.n_pixels
    b = step_buffers(sc.n, 16, sc.n_frames, P)

    def st():
        r.step_l1(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                  dev["poses"], sc.cams, 3, t_rgb, t_dep, 1.0, b, tile=tile, key_capacity=cap,
                  lds_batch=batch)
    st()
    torch.cuda.synchronize()
    keys = int(r.stats()["n_keys"])
    g = capture(st)
    for _ in range(warmup):
        g.replay()
    t_b = median_event_ms(g.replay, steps)
    r.check_overflow()
    del g
    rf, run = per_frame_setup(sc, dev, t_rgb, t_dep, tile, batch, 1.0)
    for _ in range(warmup):
        run()
    t_pf_eager = median_event_ms(run, max(3, steps // 2))
    gp = capture(run)
    for _ in range(warmup):
        gp.replay()
    t_pf = median_event_ms(gp.replay, max(3, steps // 2))
    rf.check_overflow()
    del gp
    res = {"workload": "c4: 1M Gaussians SH3 (Student-t log-scales), 16 keyframes of mixed "
                       "resolution, fwd + L1 rgb + L1 depth + bwd",
           "resolutions": [[int(c[0]), int(c[1])] for c in sc.cams], "pixels": P,
           "keys": keys, "tile": list(tile), "lds_batch": batch,
           "autotune_ms_per_tile_and_batch": {f"{w}x{h}/{b}": round(v, 3)
                                              for ((w, h), b), v in times.items()},
           "ms_per_step": round(t_b, 4), "Mpix_per_s": round(P / 1e6 / (t_b * 1e-3), 3),
           "per_frame_ms": round(t_pf, 4), "per_frame_eager_ms": round(t_pf_eager, 4),
           "batched_vs_per_frame_speedup": round(t_pf / t_b, 4)}
    log(f"[bench] c4 {res}")
    del rf, r
    torch.cuda.synchronize()
    return res


def measure_c5(steps):
    """C5: one mapping iteration (forward + L1 rgb + 0.1 L1 depth + backward +
    fused Adam on means, SH and poses with the pose fold) on 3M Gaussians and
    12 x 1920x1080 keyframes, captured as one graph; median replay time."""
    import torch
    from paper_2411_17660_amd import scenes
    from paper_2411_17660_amd.raster import Rasterizer
    t0 = time.time()
    sc = scenes.scene_c5()
    log(f"[bench] c5 scene in {time.time() - t0:.1f}s")
    dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k), np.float32)).cuda()
           for k in ("means", "log_scales", "quats", "opacity", "sh", "poses")}
    gt = torch.from_numpy(sc.extra["gt_means"]).cuda()
    r = Rasterizer(0)
    t_rgb, t_dep, _ = r.forward(gt, dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                                dev["poses"], sc.cams, 3)
    t_rgb, t_dep = t_rgb.clone(), t_dep.clone()
    n, F, P = sc.n, sc.n_frames, sc.n_pixels
    b = step_buffers(n, 16, F, P)
    state = dict(m_means=torch.zeros(n, 3, device="cuda"), v_means=torch.zeros(n, 3, device="cuda"),
                 m_sh=torch.zeros(n, 16, 3, device="cuda"), v_sh=torch.zeros(n, 16, 3, device="cuda"),
                 m_twist=torch.zeros(F, 6, device="cuda"), v_twist=torch.zeros(F, 6, device="cuda"),
                 step=torch.zeros(1, dtype=torch.int32, device="cuda"))

    def stp(cap):
        r.step_l1(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                  dev["poses"], sc.cams, 3, t_rgb, t_dep, 0.1, b, key_capacity=cap)
    stp(0)
    torch.cuda.synchronize()
    keys = int(r.stats()["n_keys"])
    cap = int(keys * 1.1) + 4096

    def iteration():
        stp(cap)
        r.adam_step(dict(means=dev["means"], sh=dev["sh"], poses=dev["poses"]),
                    dict(means=b["means"], sh=b["sh"], twist=b["twist"]), state)
    g = capture(iteration)
    g.replay()
    t_it = median_event_ms(g.replay, steps)
    r.check_overflow()
    loss = float(b["loss"].item())
    del g
    res = {"workload": "c5: 3M Gaussians SH3, 12 keyframes 1920x1080 f=1000, one mapping "
                       "iteration (fwd + L1 rgb + 0.1 L1 depth + bwd + fused Adam, pose fold)",
           "keys": keys, "iteration_ms": round(t_it, 4),
           "Mpix_per_s": round(P / 1e6 / (t_it * 1e-3), 3), "iterations_timed": steps,
           "adam_steps_taken": int(state["step"].item()), "loss_after": loss}
    log(f"[bench] c5 {res}")
    del r
    torch.cuda.synchronize()
    return res


# Rendering loss with SSIM (11x11 window, FP64 arithmetic), per pixel of the
# batch: the forward reads rendered and target colours (8 B per colour value)
# and writes the map's three FP64 derivatives (24 B); the backward reads
# those and both colours again (32 B) and writes the colour gradient (4 B);
# the depth term reads 8 B and writes 8 B (depth and alpha gradients) more.
# FP64 flops per colour value: 5 window sums x 22 taps + 3 products + ~30 for
# the map (forward), 3 window sums x 22 taps + 6 (backward).
RENDER_LOSS_BYTES_PER_PX = 3 * (32 + 36) + 8 + 16
RENDER_LOSS_FP64_FLOPS_PER_VALUE = 2 * 5 * 22 + 3 + 30 + 2 * 3 * 22 + 6
PEAK_FP64_VECTOR_TFLOPS = 78.6


def measure_render_loss(rast, sc, dev, bb, t_rgb, t_dep, tile, cap, steps):
    """Times gsr_loss_render on the batch's rendered images (HIP events on
    the library's stream) and the mapping step with that loss."""
    import torch
    P, F = sc.n_pixels, sc.n_frames
    out = dict(loss=torch.empty(1, device="cuda"), ssim=torch.empty(F, device="cuda"),
               g_rgb=torch.empty(3 * P, device="cuda"), g_depth=torch.empty(P, device="cuda"),
               g_alpha=torch.empty(P, device="cuda"))
    rast.forward(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                 dev["poses"], sc.cams, 3, tile=tile, key_capacity=cap,
                 out=(bb["rgb"], bb["depth"], bb["alpha"]))
    for _ in range(2):
        rast.loss_render(bb["rgb"], bb["depth"], t_rgb, t_dep, 0.9, 0.2, out=out)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rast.loss_render(bb["rgb"], bb["depth"], t_rgb, t_dep, 0.9, 0.2, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = P * RENDER_LOSS_BYTES_PER_PX
    flops = 3 * P * RENDER_LOSS_FP64_FLOPS_PER_VALUE
    gbs = nbytes / (ms * 1e-3) / 1e9
    tfl = flops / (ms * 1e-3) / 1e12
    # the mapping step with the full loss (forward + loss + backward)
    K = (sc.sh_degree + 1) ** 2
    b = dict(bb, ssim=torch.empty(F, device="cuda"))

    def rstep():
        rast.step_render(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                         dev["poses"], sc.cams, 3, t_rgb, t_dep, b, 0.9, 0.2, tile=tile,
                         key_capacity=cap)
    assert b["sh"].shape[1] == K
    for _ in range(2):
        rstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rstep()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    rast.check_overflow()
    log(f"[bench] render loss {ms:.4f} ms/call ({gbs:.0f} GB/s, {tfl:.2f} FP64 TFLOP/s); "
        f"step with it {t_step * 1e3:.2f} ms")
    return {"lambda1": 0.9, "lambda2": 0.2, "ms_per_call": round(ms, 4),
            "ssim_per_frame": [round(float(v), 6) for v in out["ssim"].cpu()],
            "loss": float(out["loss"].item()),
            "bound": "hbm", "hbm_bytes_per_call": nbytes, "achieved_GBps": round(gbs, 1),
            "peak_GBps": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 4),
            "fp64_flops_per_call": flops, "achieved_fp64_TFLOPs": round(tfl, 3),
            "frac_fp64_peak": round(tfl / PEAK_FP64_VECTOR_TFLOPS, 4),
            "step_ms": round(t_step * 1e3, 4), "step_mpix_per_s": round(P / 1e6 / t_step, 3)}


def measure_median(rast, sc, dev, bb, t_rgb, t_dep, tile, cap, steps, depth_weight):
    """The same L1 step with the median depth (GSR_FLAG_MEDIAN_DEPTH): step
    time and the compositing stages from HIP events on the library's stream."""
    import torch

    def mstep(timing=False):
        rast.step_l1(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                     dev["poses"], sc.cams, 3, t_rgb, t_dep, depth_weight, bb, tile=tile,
                     key_capacity=cap, timing=timing, median=True)
    for _ in range(2):
        mstep()
    torch.cuda.synchronize()
    rast.timings()
    t0 = time.perf_counter()
    for _ in range(steps):
        mstep(timing=True)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    rast.check_overflow()
    st = rast.timings()
    per = {k: round(st[k][0] / max(steps, 1), 4) for k in ("composite_fwd", "composite_bwd")}
    log(f"[bench] median-depth step {t_step * 1e3:.2f} ms, {per}")
    return {"step_ms": round(t_step * 1e3, 4), "step_mpix_per_s": round(sc.n_pixels / 1e6 / t_step, 3),
            "stage_ms_per_step": per}


def _event_ms(fn, reps=20):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def measure_densify(rast, sc, dev, bb, t_rgb, t_dep, tile, cap, depth_weight):
    """The densification kernels on the workload's Gaussians (HIP events on
    the library's stream), against the HBM bytes they must move: ADC
    statistics read, per (Gaussian, frame) record, the tile count (4 B) and
    dL/d(u, v) (16 B) and per Gaussian read-modify-write two floats (16 B);
    MCMC noise reads means, log-scales, quaternion, opacity and the normal
    draw (52 B) and writes the means (12 B); relocation with no dead
    Gaussians reads src (4 B) and writes and reads the 4-byte counter."""
    import torch
    n, F = sc.n, sc.n_frames
    rast.step_l1(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"],
                 dev["poses"], sc.cams, 3, t_rgb, t_dep, depth_weight, bb, tile=tile,
                 key_capacity=cap)
    acc = torch.zeros(n, device="cuda")
    cnt = torch.zeros(n, device="cuda")
    ms_stats = _event_ms(lambda: rast.densify_stats(acc, cnt))
    means = dev["means"].clone()
    eps = torch.randn(n, 3, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    ms_noise = _event_ms(lambda: rast.mcmc_noise(means, dev["log_scales"], dev["quats"],
                                                 dev["opacity"], eps, 1e-9))
    src = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    p = {k: dev[k].clone() for k in ("means", "log_scales", "quats", "opacity", "sh")}
    ms_reloc = _event_ms(lambda: rast.mcmc_relocate(p["means"], p["log_scales"], p["quats"],
                                                    p["opacity"], p["sh"], src, 3))
    b_stats = n * F * 20 + n * 16
    b_noise = n * 64
    b_reloc = n * 12

    def row(ms, b):
        gbs = b / (ms * 1e-3) / 1e9
        return {"ms": round(ms, 4), "hbm_bytes": b, "achieved_GBps": round(gbs, 1),
                "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)}
    out = {"stats": row(ms_stats, b_stats), "mcmc_noise": row(ms_noise, b_noise),
           "mcmc_relocate_no_dead": row(ms_reloc, b_reloc)}
    log(f"[bench] densify kernels {out}")
    return out


def measure_surfel(rast, sc, dev, tile, steps):
    """The 2D surfel variant on the workload's primitives (the same means,
    the first two log-scales, quaternions, opacities and SH), all frames in
    one batch: forward (rgb, depth, alpha, normal, distortion), backward of
    all five outputs, and the normal-consistency term on the rendered maps.
    HIP events on the library's stream.  The normal-consistency kernel moves
    60 B per pixel at least: it reads depth, alpha and the normal (20 B) and
    reads and writes the three gradients (40 B)."""
    import torch
    P = sc.n_pixels
    ls2 = dev["log_scales"][:, :2].contiguous()
    out = [torch.empty(3 * P, device="cuda"), torch.empty(P, device="cuda"),
           torch.empty(P, device="cuda"), torch.empty(3 * P, device="cuda"),
           torch.empty(P, device="cuda")]

    def fwd(cap, **kw):
        rast.forward_surfel(dev["means"], ls2, dev["quats"], dev["opacity"], dev["sh"],
                            dev["poses"], sc.cams, 3, tile=tile, key_capacity=cap, out=out, **kw)
    fwd(0)
    torch.cuda.synchronize()
    keys = int(rast.stats()["n_keys"])
    cap = int(keys * 1.05) + 1024
    fwd(cap, count_pairs=True)
    pairs = int(rast.stats()["n_pairs"])
    gen = torch.Generator("cuda").manual_seed(3)
    ups = [1e-6 * torch.randn(x.numel(), device="cuda", generator=gen) for x in out]
    K = 16
    g = dict(means=torch.empty(sc.n, 3, device="cuda"), log_scales=torch.empty(sc.n, 2, device="cuda"),
             quats=torch.empty(sc.n, 4, device="cuda"), opacity=torch.empty(sc.n, device="cuda"),
             sh=torch.empty(sc.n, K, 3, device="cuda"), twist=torch.empty(sc.n_frames, 6, device="cuda"))
    reps = max(3, min(steps, 10))
    ms_fwd = _event_ms(lambda: fwd(cap), reps)
    fwd(cap)
    ms_bwd = _event_ms(lambda: rast.backward_surfel(*ups, out=g), reps)
    # the compositing kernels alone, from the library's per-stage HIP events
    rast.timings()
    for _ in range(reps):
        fwd(cap, timing=True)
        rast.backward_surfel(*ups, out=g)
    st = rast.timings()
    roof = {}
    for stage, fl in (("composite_fwd", SURFEL_FLOPS_PER_PAIR["fwd"]),
                      ("composite_bwd", SURFEL_FLOPS_PER_PAIR["bwd"])):
        ms = st[stage][0] / max(st[stage][1], 1)
        ach = pairs * fl / (ms * 1e-3) / 1e12
        roof[stage] = {"avg_launch_ms": round(ms, 4), "flops_per_pair": fl,
                       "achieved_TFLOPs": round(ach, 3),
                       "frac": round(ach / PEAK_FP32_VECTOR_TFLOPS, 4)}
    gd, ga, gn = (torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda"),
                  torch.zeros(3 * P, device="cuda"))
    loss = torch.empty(1, device="cuda")
    ms_nc = _event_ms(lambda: rast.normal_consistency(sc.cams, out[1], out[2], out[3], 0.05,
                                                      gd, ga, gn, loss=loss), reps)
    torch.cuda.synchronize()
    ok = bool(torch.isfinite(g["means"]).all()) and float(out[2].max()) > 0.5
    gbs = 60.0 * P / (ms_nc * 1e-3) / 1e9
    res = {"keys_per_forward": keys, "pairs_per_forward": pairs, "forward_ms": round(ms_fwd, 4),
           "backward_ms": round(ms_bwd, 4),
           "fwd_bwd_Mpix_per_s": round(P / 1e6 / ((ms_fwd + ms_bwd) * 1e-3), 3),
           "normal_consistency": {"ms": round(ms_nc, 4), "hbm_bytes": 60 * P,
                                  "achieved_GBps": round(gbs, 1),
                                  "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)},
           "roofline": {"bound": "alu", "unit": "TFLOP/s", "peak": PEAK_FP32_VECTOR_TFLOPS,
                        **roof},
           "finite_and_covered": ok}
    log(f"[bench] surfels {res}")
    return res


# The compositing kernels' source: raster.hip and every header it includes.
COMPOSITING_SOURCES = ("paper_2411_17660_amd/csrc/raster.hip",
                       "paper_2411_17660_amd/csrc/wave_util.h",
                       "paper_2411_17660_amd/csrc/launch.h",
                       "paper_2411_17660_amd/csrc/gsr_device.h",
                       "paper_2411_17660_amd/csrc/host_check.h",
                       "include/gsr.h")


def compositing_sources_sha256(root=None):
    """SHA-256 over the compositing kernels' source files under `root` (the
    repository by default), in the order above."""
    import hashlib
    root = ROOT if root is None else root
    h = hashlib.sha256()
    for rel in COMPOSITING_SOURCES:
        h.update(open(os.path.join(root, rel), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, tile):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (scaled by the copy-kernel calibration), or None when
    the summary covers another kernel or tile shape or the compositing source
    (raster.hip or a header it includes) has changed since the counters were
    taken."""
    import re
    path = os.path.join(ROOT, "profiles", "c3_hbm_traffic_pmc.md")
    if not os.path.exists(path) or tuple(tile) != (16, 16):
        return None
    sha = compositing_sources_sha256(ROOT)
    for line in open(path):
        m = re.search(r"traffic (\w+)<16, 16> bytes_per_launch=(\d+) "
                      r"compositing_sources_sha256=(\w+)", line)
        if m and m.group(1) == kernel + "_kernel" and m.group(3) == sha:
            return int(m.group(2))
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, threads, budget_s=25.0):
    """FP64 oracle, forward + backward of the keyframes one at a time (each
    with all Gaussians) on the host cores, until every frame is done or
    `budget_s` has passed; upstream gradients of the L1 loss's shape
    (+-1/(3HW) per channel, +-1/HW per depth pixel).  Then the first keyframe
    again on one thread."""
    import oracle
    nthreads = threads or min(16, os.cpu_count() or 1)
    log(f"[bench] cpu baseline: oracle, keyframes one at a time, {nthreads} threads")
    rng = np.random.default_rng(0)

    def one(f, nt):
        sf = sc.subset_frames([f])
        r = oracle.forward(sf, threads=nt)
        P = r.P
        G = (rng.choice([-1.0, 1.0], 3 * P) / (3 * P), rng.choice([-1.0, 1.0], P) / P,
             np.zeros(P))
        r.backward(*G)
        return P
    pixels, done, t0 = 0, 0, time.perf_counter()
    for f in range(sc.n_frames):
        pixels += one(f, nthreads)
        done += 1
        dt = time.perf_counter() - t0
        log(f"[bench] cpu baseline: frame {f} done, {dt:.1f}s")
        if dt >= budget_s:
            break
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    p1 = one(0, 1)
    dt1 = time.perf_counter() - t1
    log(f"[bench] cpu baseline: frame 0 on one thread {dt1:.1f}s")
    w, h = int(sc.cams[0][0]), int(sc.cams[0][1])
    return {"value": round(pixels / 1e6 / dt, 5), "unit": "Mpixels/s", "cores": nthreads,
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"{done} of the {sc.n_frames} keyframes ({w}x{h}, all {sc.n} Gaussians "
                      f"each), one at a time, fwd+bwd, FP64",
            "one_thread": {"value": round(p1 / 1e6 / dt1, 5), "unit": "Mpixels/s",
                           "seconds": round(dt1, 2), "sample": "keyframe 0, fwd+bwd, FP64"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
