"""Parity of the rendering loss with SSIM (HIP, through the C-ABI) against
the FP64 oracle (oracle/ssim.py) on seeded synthetic images.

The kernels evaluate the SSIM map and its adjoint in FP64 from FP32 inputs
and round the results to FP32 once, so the bar is the FP32 rounding of the
outputs: 1e-6 relative per element, plus 1e-10 of the largest gradient
entry for entries the two FP64 evaluations cancel to nearly zero."""
import numpy as np
import pytest

import oracle
from paper_2411_17660_amd import scenes
from gpu_util import to_dev, gpu_forward, assert_grad_close, oracle_threads

pytestmark = pytest.mark.gpu

REL = 1e-6
ABS = 1e-10


def f32(v):
    """The weights cross the C ABI as FP32: the oracle takes those values."""
    return float(np.float32(v))


@pytest.fixture(scope="module")
def rast():
    from paper_2411_17660_amd.raster import Rasterizer
    return Rasterizer(0)


def _dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in arrs]


def _gpu_loss(rast, sizes, imgs, l1, l2):
    import torch
    gpu_forward(rast, scenes.layout_scene(sizes))
    rgb, dep, t_rgb, t_dep = _dev(*imgs)
    out = rast.loss_render(rgb, dep, t_rgb, t_dep, l1, l2)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def _close(name, got, ref, rel=REL, abs_frac=ABS):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    scale = np.abs(ref).max() if ref.size else 0.0
    err = np.abs(got - ref)
    bound = rel * np.abs(ref) + abs_frac * scale
    worst = float((err / (bound + 1e-300)).max()) if ref.size else 0.0
    print(f"[ssim] {name}: max err/bound {worst:.3g}", flush=True)
    assert np.all(err <= bound), f"{name}: worst err/bound {worst}"


def _check(rast, sizes, seed, l1=0.8, l2=0.2, invalid=0.2):
    print(f"[ssim] sizes {sizes} seed {seed} lambda1 {l1} lambda2 {l2}", flush=True)
    imgs = scenes.loss_images(seed, sizes, depth_invalid=invalid)
    got = _gpu_loss(rast, sizes, imgs, l1, l2)
    loss, g_rgb, g_dep, g_alp, ssim = oracle.render_loss(*imgs, f32(l1), f32(l2), sizes)
    _close("loss", got["loss"], [loss])
    _close("ssim", got["ssim"], ssim)
    _close("g_rgb", got["g_rgb"], g_rgb)
    _close("g_depth", got["g_depth"], g_dep)
    assert np.all(got["g_alpha"] == 0.0)


@pytest.mark.parametrize("sizes,seed", [
    ([(100, 70)], 0),
    ([(100, 70), (33, 17), (1, 1), (64, 48), (7, 300)], 1),   # ragged, 1x1, narrow
    ([(32, 16), (31, 15), (65, 33)], 2),                        # one tile, under, over
])
def test_loss_render_matches_oracle(rast, sizes, seed):
    _check(rast, sizes, seed)


@pytest.mark.parametrize("l1,l2", [(1.0, 1.0), (0.9, 0.0), (0.0, 0.5), (0.8, 0.2)])
def test_loss_render_weights(rast, l1, l2):
    _check(rast, [(50, 40), (20, 90)], 3, l1, l2)


def test_loss_render_without_valid_depth(rast):
    _check(rast, [(40, 30), (17, 23)], 4, invalid=1.0)


def test_loss_render_identical_images(rast):
    """I' = I*: SSIM = 1, the L1 terms vanish and so does every gradient."""
    import torch
    sizes = [(70, 45), (9, 9)]
    rgb, dep, t_rgb, t_dep = scenes.loss_images(5, sizes)
    got = _gpu_loss(rast, sizes, (t_rgb, t_dep, t_rgb, t_dep), 0.8, 0.2)
    assert abs(got["loss"][0]) < 1e-6
    assert np.abs(got["ssim"] - 1.0).max() < 1e-6
    ref = oracle.render_loss(t_rgb, t_dep, t_rgb, t_dep, f32(0.8), f32(0.2), sizes)[1]
    assert np.abs(got["g_rgb"]).max() <= max(1e-9, 1e-6 * np.abs(ref).max())
    assert np.all(got["g_depth"] == 0.0)
    torch.cuda.synchronize()


def test_loss_render_rejects_bad_weights(rast):
    from paper_2411_17660_amd.native import GsrError
    sizes = [(16, 16)]
    gpu_forward(rast, scenes.layout_scene(sizes))
    rgb, dep, t_rgb, t_dep = _dev(*scenes.loss_images(6, sizes))
    with pytest.raises(GsrError):
        rast.loss_render(rgb, dep, t_rgb, t_dep, 1.5, 0.2)
    with pytest.raises(GsrError):
        rast.loss_render(rgb, dep, t_rgb, t_dep, 0.5, float("nan"))


def test_loss_render_full_size_sampled_frames(rast):
    """Eight 1200x680 frames (the batched mapping step's layout); the oracle
    evaluates frames 0 and 7, the frames' terms being independent."""
    sizes = [(1200, 680)] * 8
    imgs = scenes.loss_images(7, sizes)
    got = _gpu_loss(rast, sizes, imgs, 0.9, 0.2)
    P = 1200 * 680
    for f in (0, 7):
        print(f"[ssim] full size: oracle on frame {f}", flush=True)
        sl, sl3 = slice(f * P, (f + 1) * P), slice(3 * f * P, 3 * (f + 1) * P)
        sub = (imgs[0][sl3], imgs[1][sl], imgs[2][sl3], imgs[3][sl])
        _, g_rgb, g_dep, _, ssim = oracle.render_loss(*sub, f32(0.9), f32(0.2), [(1200, 680)])
        _close(f"f{f} ssim", got["ssim"][f:f + 1], ssim)
        _close(f"f{f} g_rgb", got["g_rgb"][sl3], g_rgb)
        _close(f"f{f} g_depth", got["g_depth"][sl], g_dep)


def _step_bufs(n, K, F, P):
    import torch
    return dict(rgb=torch.empty(3 * P, device="cuda"), depth=torch.empty(P, device="cuda"),
                alpha=torch.empty(P, device="cuda"), loss=torch.empty(1, device="cuda"),
                ssim=torch.empty(F, device="cuda"), means=torch.empty(n, 3, device="cuda"),
                log_scales=torch.empty(n, 3, device="cuda"), quats=torch.empty(n, 4, device="cuda"),
                opacity=torch.empty(n, device="cuda"), sh=torch.empty(n, K, 3, device="cuda"),
                twist=torch.empty(F, 6, device="cuda"))


def test_step_render_is_forward_loss_backward(rast):
    """The one-call step equals the three calls made one after another."""
    import torch
    sc = scenes.scene_c2(seed=1, n=20_000)
    d = to_dev(sc)
    P, K = sc.n_pixels, (sc.sh_degree + 1) ** 2
    _, _, t_rgb, t_dep = _dev(*scenes.loss_images(8, [c[:2] for c in sc.cams]))
    b = _step_bufs(sc.n, K, sc.n_frames, P)
    rast.step_render(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"],
                     sc.cams, sc.sh_degree, t_rgb, t_dep, b, 0.9, 0.2)
    torch.cuda.synchronize()
    step = {k: v.clone() for k, v in b.items()}
    rgb, dep, _ = rast.forward(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                               d["poses"], sc.cams, sc.sh_degree, sc.background)
    lo = rast.loss_render(rgb, dep, t_rgb, t_dep, 0.9, 0.2)
    g = rast.backward(lo["g_rgb"], lo["g_depth"], lo["g_alpha"])
    torch.cuda.synchronize()
    assert torch.equal(step["rgb"], rgb) and torch.equal(step["loss"], lo["loss"])
    assert torch.equal(step["ssim"], lo["ssim"])
    for k in ("means", "log_scales", "quats", "opacity", "sh", "twist"):
        assert torch.equal(step[k], g[k]), k


def test_step_render_matches_oracle_chain(rast):
    """Forward, loss and backward on each side: the oracle renders, takes
    its own loss of its own images and back-propagates it.  Both renders
    agree to FP32 rounding; the loss's curvature carries that difference
    into the upstream gradients, so the bar adds the response of the
    oracle chain to a perturbation of its images at the same scale."""
    import torch
    sc = scenes.tiny_scene(seed=4, n=120, W=64, H=48, f=48.0, n_frames=2)
    sizes = [c[:2] for c in sc.cams]
    _, _, t_rgb, t_dep = scenes.loss_images(9, sizes)
    ref = oracle.forward(sc, threads=oracle_threads())
    assert int((ref.pixel_info()[0] != 0).sum()) == 0, "a pixel sits on a decision threshold"
    d = to_dev(sc)
    P, K = sc.n_pixels, (sc.sh_degree + 1) ** 2
    td = _dev(t_rgb, t_dep)
    b = _step_bufs(sc.n, K, sc.n_frames, P)
    rast.step_render(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"],
                     sc.cams, sc.sh_degree, td[0], td[1], b, 0.8, 0.2,
                     background=sc.background)
    torch.cuda.synchronize()

    def chain(rgb, dep):
        loss, g_rgb, g_dep, g_alp, _ = oracle.render_loss(rgb, dep, t_rgb, t_dep, f32(0.8),
                                                          f32(0.2), sizes)
        return loss, ref.backward(g_rgb, g_dep, g_alp)

    loss, g_ref = chain(ref.rgb_flat, ref.depth_flat)
    # the renders agree to about 1e-7 absolute (the compositing runs in FP32)
    rng = np.random.default_rng(3)
    jig = lambda a: a + 1e-7 * rng.standard_normal(a.shape)   # noqa: E731
    _, g_pert = chain(jig(ref.rgb_flat), jig(ref.depth_flat))
    assert abs(float(b["loss"].item()) - loss) <= 1e-5 * abs(loss)
    for k, gk in (("means", "means"), ("log_scales", "log_scales"), ("quats", "quats"),
                  ("opacity", "opacity"), ("sh", "sh"), ("twist", "twist")):
        noise = np.abs(np.asarray(g_pert[gk]) - np.asarray(g_ref[gk])).ravel()
        assert_grad_close(f"c1 render step:{k}", b[k].cpu().numpy(), g_ref[gk], noise=noise)


@pytest.mark.parametrize("median", [False, True])
def test_graph_captured_render_step_replays_match_eager(rast, median):
    """The fixed-capacity step with the full loss (and the median depth)
    captured in a HIP graph: every replay, with eager work and
    synchronisations between replays, equals the eager step bitwise."""
    import torch
    from paper_2411_17660_amd.raster import Rasterizer
    sc = scenes.tiny_scene(seed=15, n=3000, W=160, H=96, f=120.0, n_frames=3)
    d = to_dev(sc)
    P, K = sc.n_pixels, (sc.sh_degree + 1) ** 2
    t_rgb, t_dep = _dev(*scenes.loss_images(16, [c[:2] for c in sc.cams])[2:])
    r = Rasterizer(0)
    b = _step_bufs(sc.n, K, sc.n_frames, P)

    def step(cap):
        r.step_render(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"],
                      sc.cams, sc.sh_degree, t_rgb, t_dep, b, 0.8, 0.2, background=sc.background,
                      key_capacity=cap, median=median)
    step(0)
    torch.cuda.synchronize()
    cap = r.stats()["n_keys"] + 64
    step(cap)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in b.items()}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(cap)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(cap)
    torch.cuda.synchronize()
    for rep in range(3):
        for v in b.values():
            v.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for k in eager:
            assert torch.equal(b[k], eager[k]), (rep, k)
        step(cap)
        torch.cuda.synchronize()
    r.check_overflow()
