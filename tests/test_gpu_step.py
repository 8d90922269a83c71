"""The benchmarked call itself: the batched mapping step (forward, summed L1
RGB + L1 depth loss, backward with the pose twists; DROID-Splat Sec. 3.3,
a batch of keyframes per mapping iteration, supplementary S1.2) at a fixed key
capacity, captured in a HIP graph and replayed, through the C-ABI.

Two links close the chain from that call to the FP64 oracle:
  (a) every output of the replayed step (images, loss, every gradient, the
      twists) is bitwise equal to the separate calls gsr_forward (grown key
      buffers), gsr_loss_l1 and gsr_backward;
  (b) the separate calls match the oracle: the loss's upstream gradient equals
      the oracle loss's on every pixel whose decisions are unambiguous, and
      the backward, fed the oracle's upstream with those pixels zeroed,
      matches the oracle's backward of all frames for every Gaussian and
      every twist.
"""
import numpy as np
import pytest

import oracle
from gpu_util import (GRAD_REL, IMG_TOL, assert_grad_close, expand_rgb_mask, gpu_backward,
                      noise_floor, oracle_threads, to_dev)
from paper_2411_17660_amd import scenes

pytestmark = pytest.mark.gpu


def _bufs(sc, dev="cuda"):
    import torch
    P, n, K = sc.n_pixels, sc.n, (sc.sh_degree + 1) ** 2
    return dict(rgb=torch.empty(3 * P, device=dev), depth=torch.empty(P, device=dev),
                alpha=torch.empty(P, device=dev), loss=torch.empty(1, device=dev),
                means=torch.empty(n, 3, device=dev), log_scales=torch.empty(n, 3, device=dev),
                quats=torch.empty(n, 4, device=dev), opacity=torch.empty(n, device=dev),
                sh=torch.empty(n, K, 3, device=dev), twist=torch.empty(sc.n_frames, 6, device=dev))


def _targets(sc, seed):
    """Seeded target images, independent of any render: colours U(0, 1),
    depths U(0.5, 4) with a fifth of the pixels without a target depth."""
    rng = np.random.default_rng(seed)
    P = sc.n_pixels
    t_rgb = rng.uniform(0.0, 1.0, 3 * P).astype(np.float32)
    t_dep = rng.uniform(0.5, 4.0, P).astype(np.float32)
    t_dep[rng.uniform(size=P) < 0.2] = 0.0
    return t_rgb, t_dep


def _sizes(sc):
    return [(int(c[0]), int(c[1])) for c in sc.cams]


def _separate(rast, d, sc, trgb, tdep, wd, tile, batch=0):
    """gsr_forward (grown key buffers) + gsr_loss_l1 + gsr_backward."""
    import torch
    rgb, dep, alp = rast.forward(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                                 d["poses"], sc.cams, sc.sh_degree, sc.background, tile=tile,
                                 lds_batch=batch)
    lo = rast.loss_l1(trgb, tdep, wd)
    g = rast.backward(lo["g_rgb"], lo["g_depth"], lo["g_alpha"])
    torch.cuda.synchronize()
    return dict(rgb=rgb, depth=dep, alpha=alp, loss=lo["loss"], **g), lo


def _check_against_oracle(rast, sc, d, sep, lo, t_rgb, t_dep, wd, tile, label):
    """Link (b): the loss's upstream and the backward against the oracle."""
    import torch
    sizes = _sizes(sc)
    print(f"[step] {label}: oracle forward of {sc.n_frames} frames", flush=True)
    ref = oracle.forward(sc, tile=tile, threads=oracle_threads())
    flags = ref.pixel_info()[0]
    ok = flags == 0
    ok3 = expand_rgb_mask(ok, sizes)
    rgb = sep["rgb"].cpu().numpy()
    dep = sep["depth"].cpu().numpy()
    e_rgb = np.abs(rgb - ref.rgb_flat)[ok3].max(initial=0.0)
    e_dep = np.abs(dep - ref.depth_flat)[ok].max(initial=0.0)
    print(f"[step]   images: max err rgb {e_rgb:.3g} depth {e_dep:.3g}; flagged px "
          f"{int((~ok).sum())} of {ok.size}", flush=True)
    assert e_rgb <= IMG_TOL and e_dep <= IMG_TOL
    L_ref, gr, gd, ga = oracle.loss_l1(ref.rgb_flat, ref.depth_flat, t_rgb, t_dep, wd, sizes)
    # a pixel's sign decision is unambiguous when the oracle's image and the
    # target differ by more than the image tolerance
    amb_rgb = np.abs(ref.rgb_flat - t_rgb) <= IMG_TOL
    amb_dep = (t_dep > 0) & (np.abs(ref.depth_flat - t_dep) <= IMG_TOL)
    keep3 = ok3 & ~amb_rgb
    keep = ok & ~amb_dep
    print(f"[step]   sign-ambiguous values: rgb {int(amb_rgb.sum())}, depth "
          f"{int(amb_dep.sum())}", flush=True)
    g_rgb_gpu = lo["g_rgb"].cpu().numpy().astype(np.float64)
    g_dep_gpu = lo["g_depth"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(g_rgb_gpu[keep3], gr[keep3], rtol=1e-7, atol=0)
    np.testing.assert_allclose(g_dep_gpu[keep], gd[keep], rtol=1e-7, atol=0)
    assert np.all(lo["g_alpha"].cpu().numpy() == 0)
    assert abs(float(lo["loss"].item()) - L_ref) <= 1e-5 * max(1.0, abs(L_ref))
    # the backward of the oracle's upstream with the undecided pixels zeroed,
    # on the forward state of the benchmarked layout
    Gm = (np.where(keep3, gr, 0.0).astype(np.float32), np.where(keep, gd, 0.0).astype(np.float32),
          np.zeros_like(gd, dtype=np.float32))
    rast.forward(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"],
                 sc.cams, sc.sh_degree, sc.background, tile=tile)
    g_gpu = gpu_backward(rast, Gm)
    print(f"[step]   oracle backward", flush=True)
    g_ref = ref.backward(*[x.astype(np.float64) for x in Gm])
    nz = noise_floor(ref, Gm, g_ref)
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        assert_grad_close(f"{label}:{k}", g_gpu[k], g_ref[k], noise=nz[k])
    for f in range(sc.n_frames):
        tw, tr = g_gpu["twist"][f], g_ref["twist"][f]
        bound = GRAD_REL * np.maximum(np.abs(tr), 1e-2 * np.abs(tr).max())
        assert np.all(np.abs(tw - tr) <= bound), (label, f, tw, tr)
    print(f"[step]   twists of {sc.n_frames} frames within the bar", flush=True)


def _bitwise(a, b, label):
    import torch
    for k in ("rgb", "depth", "alpha", "loss", "means", "log_scales", "quats", "opacity", "sh",
              "twist"):
        assert torch.equal(a[k], b[k]), (label, k)


def test_l1_step_equals_forward_loss_backward_and_the_oracle():
    """Small two-frame scene: the one-call step (grown buffers) equals the
    three calls bitwise, and the three calls match the oracle."""
    import torch
    from paper_2411_17660_amd.raster import Rasterizer
    sc = scenes.tiny_scene(seed=8, n=2000, W=120, H=90, f=90.0, n_frames=2)
    rast = Rasterizer(0)
    d = to_dev(sc)
    t_rgb, t_dep = _targets(sc, 8)
    trgb, tdep = torch.from_numpy(t_rgb).cuda(), torch.from_numpy(t_dep).cuda()
    b = _bufs(sc)
    rast.step_l1(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"],
                 sc.cams, sc.sh_degree, trgb, tdep, 0.5, b, background=sc.background)
    torch.cuda.synchronize()
    step = {k: v.clone() for k, v in b.items()}
    sep, lo = _separate(rast, d, sc, trgb, tdep, 0.5, (16, 16))
    _bitwise(step, sep, "small")
    _check_against_oracle(rast, sc, d, sep, lo, t_rgb, t_dep, 0.5, (16, 16), "small")


def test_benchmarked_step_c3():
    """The C3 batch (500k Gaussians, 8 x 1200x680, SH3) in the benchmark's
    launch configuration: the autotuner's tile, its fixed key capacity, the
    step captured once and replayed as a HIP graph."""
    import torch
    from paper_2411_17660_amd.raster import Rasterizer
    sc = scenes.scene_c3()
    rast = Rasterizer(0)
    d = to_dev(sc)
    t_rgb, t_dep = _targets(sc, 33)
    trgb, tdep = torch.from_numpy(t_rgb).cuda(), torch.from_numpy(t_dep).cuda()
    wd = 1.0
    print("[step] c3: autotune", flush=True)
    tile, batch, cap, times = rast.autotune(d["means"], d["log_scales"], d["quats"],
                                            d["opacity"], d["sh"], d["poses"], sc.cams, 3, trgb,
                                            tdep, wd, background=sc.background, reps=1,
                                            force=True)
    print(f"[step] c3: tile {tile} batch {batch} capacity {cap} times {times}", flush=True)
    b = _bufs(sc)

    def step():
        rast.step_l1(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"],
                     sc.cams, 3, trgb, tdep, wd, b, background=sc.background, tile=tile,
                     key_capacity=cap, lds_batch=batch)
    step()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    replays = []
    for rep in range(2):
        for v in b.values():
            v.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        replays.append({k: v.clone() for k, v in b.items()})
    rast.check_overflow()
    del g
    _bitwise(replays[0], replays[1], "c3 replays")
    print("[step] c3: separate calls with grown key buffers", flush=True)
    sep, lo = _separate(rast, d, sc, trgb, tdep, wd, tile, batch)
    _bitwise(replays[1], sep, "c3")
    print("[step] c3: replayed step bitwise equal to forward + loss + backward", flush=True)
    _check_against_oracle(rast, sc, d, sep, lo, t_rgb, t_dep, wd, tile, "c3")


def test_graph_of_steps_with_different_frame_tables():
    """Two steps of one context with different frame tables (sizes and
    intrinsics) captured in one HIP graph: every replay, with eager work of the
    same context between replays, gives each step's eager outputs bitwise.
    The frame table travels as kernel arguments, so each captured forward
    writes its own."""
    import torch
    from paper_2411_17660_amd.raster import Rasterizer
    rast = Rasterizer(0)
    sa = scenes.tiny_scene(seed=31, n=1500, W=96, H=72, f=80.0, n_frames=2)
    sb = scenes.tiny_scene(seed=32, n=1500, W=150, H=100, f=120.0, n_frames=1)
    runs = []
    for sc, seed in ((sa, 1), (sb, 2)):
        d = to_dev(sc)
        t_rgb, t_dep = _targets(sc, 50 + seed)
        trgb, tdep = torch.from_numpy(t_rgb).cuda(), torch.from_numpy(t_dep).cuda()
        runs.append((sc, d, trgb, tdep, _bufs(sc)))

    def step(i, cap):
        sc, d, trgb, tdep, b = runs[i]
        rast.step_l1(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"],
                     sc.cams, sc.sh_degree, trgb, tdep, 0.5, b, background=sc.background,
                     key_capacity=cap)
    caps = []
    eager = []
    for i in range(2):
        step(i, 0)
        torch.cuda.synchronize()
        caps.append(int(rast.stats()["n_keys"]) + 256)
    for i in range(2):
        step(i, caps[i])
        torch.cuda.synchronize()
        eager.append({k: v.clone() for k, v in runs[i][4].items()})

    def both():
        step(0, caps[0])
        step(1, caps[1])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        both()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        both()
    torch.cuda.synchronize()
    for rep in range(3):
        for r in runs:
            for v in r[4].values():
                v.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for i in range(2):
            _bitwise(runs[i][4], eager[i], f"replay {rep} step {i}")
        # eager work of the same context between replays (the other table last)
        step(1, caps[1])
        step(0, caps[0])
        torch.cuda.synchronize()
    rast.check_overflow()
    del g
