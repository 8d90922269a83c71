"""The allocation-free L1 loss (gsr_loss_l1_noalloc, for callers that cannot
allocate device memory) through the C-ABI: on two calls in a row, the second
on a smaller batch, its loss and gradients are bitwise those of gsr_loss_l1
on the same forward (the same kernels on the static scratch); the oracle's
L1 loss pins both on the pixels whose sign decisions are unambiguous.  A
forward too large for the static scratch is refused before any launch."""
import numpy as np
import pytest

import oracle
from gpu_util import IMG_TOL, gpu_forward, oracle_threads
from paper_2411_17660_amd import native, scenes

pytestmark = pytest.mark.gpu


def _targets(sc, seed):
    rng = np.random.default_rng(seed)
    P = sc.n_pixels
    t_rgb = rng.uniform(0.0, 1.0, 3 * P).astype(np.float32)
    t_dep = rng.uniform(0.5, 4.0, P).astype(np.float32)
    t_dep[rng.uniform(size=P) < 0.2] = 0.0
    return t_rgb, t_dep


def _outs(P, dev="cuda"):
    import torch
    return dict(loss=torch.full((1,), float("nan"), device=dev),
                g_rgb=torch.full((3 * P,), float("nan"), device=dev),
                g_depth=torch.full((P,), float("nan"), device=dev),
                g_alpha=torch.full((P,), float("nan"), device=dev))


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_loss_matches_loss_l1(order):
    import torch
    from paper_2411_17660_amd.raster import Rasterizer
    rast = Rasterizer(0)
    cases = [scenes.tiny_scene(seed=21, n=3000, W=200, H=150, f=150.0, n_frames=3),
             scenes.tiny_scene(seed=22, n=500, W=64, H=48, f=50.0, n_frames=1)]
    for i, sc in enumerate(cases):
        print(f"[noalloc] call {i}: {sc.n_frames} frames {sc.cams[0][0]}x{sc.cams[0][1]}",
              flush=True)
        _, rgb, dep, _ = gpu_forward(rast, sc)
        t_rgb, t_dep = _targets(sc, 40 + i)
        trgb, tdep = torch.from_numpy(t_rgb).cuda(), torch.from_numpy(t_dep).cuda()
        ref = _outs(sc.n_pixels)
        rast.loss_l1(trgb, tdep, 0.7, out=ref)
        na = _outs(sc.n_pixels)
        rast.loss_l1_noalloc(trgb, tdep, 0.7, na)
        torch.cuda.synchronize()
        for k in ("loss", "g_rgb", "g_depth", "g_alpha"):
            assert torch.equal(ref[k], na[k]), (i, k)
        # the oracle's L1 loss of the GPU images: value, and the gradient where
        # the sign of (image - target) is not within the image tolerance
        sizes = [(int(c[0]), int(c[1])) for c in sc.cams]
        r64, d64 = rgb.cpu().numpy().astype(np.float64), dep.cpu().numpy().astype(np.float64)
        L, gr, gd, _ = oracle.loss_l1(r64, d64, t_rgb, t_dep, 0.7, sizes)
        assert abs(float(na["loss"].item()) - L) <= 1e-5 * max(1.0, abs(L))
        ok_r = np.abs(r64 - t_rgb) > IMG_TOL
        ok_d = ~((t_dep > 0) & (np.abs(d64 - t_dep) <= IMG_TOL))
        np.testing.assert_allclose(na["g_rgb"].cpu().numpy()[ok_r], gr[ok_r], rtol=1e-6, atol=0)
        np.testing.assert_allclose(na["g_depth"].cpu().numpy()[ok_d], gd[ok_d], rtol=1e-6,
                                   atol=0)
        print(f"[noalloc] call {i}: bitwise equal to gsr_loss_l1, loss {L:.6f}", flush=True)


def test_noalloc_refuses_a_batch_beyond_its_scratch():
    import torch
    from paper_2411_17660_amd.raster import Rasterizer
    rast = Rasterizer(0)
    # 12 frames of 4096x2160: 12 * ceil(4096*2160/2048) * 24 + 96 bytes > 1 MiB
    sc = scenes.tiny_scene(seed=23, n=50, W=4096, H=2160, f=2000.0, n_frames=12)
    print("[noalloc] 12 x 4096x2160 forward", flush=True)
    gpu_forward(rast, sc)
    P = sc.n_pixels
    t = torch.zeros(3 * P, device="cuda")
    out = _outs(P)
    with pytest.raises(native.GsrError) as e:
        rast.loss_l1_noalloc(t, t[:P], 1.0, out)
    assert e.value.status == 6  # GSR_ERR_UNSUPPORTED
    assert "1048576" in str(e.value)
    torch.cuda.synchronize()
    assert torch.isnan(out["loss"]).all()  # nothing was launched
