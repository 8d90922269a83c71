"""Parity of the normal-consistency term (gsr_normal_consistency, through the
C-ABI) against the FP64 oracle (oracle/surfel.normal_consistency) and its
autograd.

The kernel evaluates the stencil in FP64 from the FP32 images, so the loss
is held to FP32 rounding of an FP64 sum (1e-6 relative) and each gradient
element, which the kernel adds to a pre-filled FP32 buffer, to the rounding
of that sum: |got - (init + ref)| <= 2^-22 (|init| + |ref|) + 1e-30.
Cases: ragged frame sizes (not multiples of the 64 x 4 block), frames of
2 x 2 and 3 x 3 pixels (no interior, one interior pixel), zero-depth
regions (undefined normals), a mixed batch, and the images of a surfel
render."""
import numpy as np
import pytest

from oracle import surfel as S
from paper_2411_17660_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    from paper_2411_17660_amd.raster import Rasterizer
    return Rasterizer(0)


def _oracle(cams, depth, alpha, normal, weight):
    import torch
    loss = 0.0
    gd, ga, gn = [], [], []
    off = 0
    for cam in cams:
        W, H = int(cam[0]), int(cam[1])
        P = W * H
        D = S.to64(depth[off:off + P].reshape(H, W), True)
        a = S.to64(alpha[off:off + P].reshape(H, W), True)
        n = S.to64(normal[3 * off:3 * (off + P)].reshape(3, H, W), True)
        if W > 2 and H > 2:
            lf, _ = S.normal_consistency(D, a, n, cam)
            lf = weight * lf
            g = torch.autograd.grad(lf, (D, a, n), allow_unused=True)
            g = [np.zeros(x.shape) if gi is None else gi.numpy() for gi, x in zip(g, (D, a, n))]
            loss += float(lf.detach())
        else:
            g = [np.zeros((H, W)), np.zeros((H, W)), np.zeros((3, H, W))]
        gd.append(g[0].ravel())
        ga.append(g[1].ravel())
        gn.append(g[2].ravel())
        off += P
    return loss, np.concatenate(gd), np.concatenate(ga), np.concatenate(gn)


def _run(rast, cams, depth, alpha, normal, weight, seed):
    import torch
    rng = np.random.default_rng(seed)
    init = [rng.normal(size=x.size).astype(np.float32) for x in (depth, alpha, normal)]
    dev = [torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
           for x in (depth, alpha, normal)]
    g = [torch.from_numpy(x.copy()).cuda() for x in init]
    print(f"[normals] frames {[(c[0], c[1]) for c in cams]} weight {weight}", flush=True)
    loss = rast.normal_consistency(cams, *dev, weight, *g)
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in g]
    ref = _oracle(cams, depth.astype(np.float64), alpha.astype(np.float64),
                  normal.astype(np.float64), float(np.float32(weight)))
    L = float(loss.cpu()[0])
    print(f"[normals]   loss {L:.9g} oracle {ref[0]:.9g}", flush=True)
    assert abs(L - ref[0]) <= 1e-6 * abs(ref[0]) + 1e-30
    for name, gi, i0, r in zip(("depth", "alpha", "normal"), got, init, ref[1:]):
        want = i0.astype(np.float64) + r
        bound = 2.0 ** -22 * (np.abs(i0) + np.abs(r)) + 1e-30
        q = float((np.abs(gi - want) / bound).max())
        print(f"[normals]   g_{name}: max err/bound {q:.3g}, max |grad| {np.abs(r).max():.3g}",
              flush=True)
        assert q <= 1.0, name
    return ref


def _images(rng, cams, zero_frac=0.0):
    P = sum(int(c[0]) * int(c[1]) for c in cams)
    depth = (2.0 + 0.3 * rng.normal(size=P)).astype(np.float32)
    if zero_frac:
        depth[rng.uniform(size=P) < zero_frac] = 0.0
    alpha = rng.uniform(0, 1, P).astype(np.float32)
    normal = rng.normal(size=3 * P).astype(np.float32)
    return depth, alpha, normal


@pytest.mark.parametrize("sizes,zero_frac,seed", [
    ([(97, 61)], 0.0, 0), ([(64, 4)], 0.0, 1), ([(130, 70), (33, 17)], 0.1, 2),
    ([(3, 3), (2, 2), (65, 5), (1, 9)], 0.0, 3)])
def test_normal_consistency_matches_oracle(rast, sizes, zero_frac, seed):
    rng = np.random.default_rng(seed)
    cams = [(w, h, 0.8 * max(w, h), 0.9 * max(w, h), w / 2.0 - 0.3, h / 2.0 + 0.2, 0.1)
            for (w, h) in sizes]
    d, a, n = _images(rng, cams, zero_frac)
    _run(rast, cams, d, a, n, 0.05, seed)


def test_normal_consistency_on_rendered_surfels(rast):
    import torch
    from gpu_util import to_dev
    sc = scenes.tiny_scene(seed=31, n=900, W=120, H=80, f=96.0, n_frames=2, sh_degree=1,
                           ls_mean=-2.4, ls_sigma=0.3, opacity_sigma=1.5)
    sc.log_scales = np.ascontiguousarray(sc.log_scales[:, :2])
    d = to_dev(sc)
    rgb, dep, alp, nrm, dst = rast.forward_surfel(d["means"], d["log_scales"], d["quats"],
                                                  d["opacity"], d["sh"], d["poses"], sc.cams,
                                                  sc.sh_degree, sc.background)
    torch.cuda.synchronize()
    assert float(alp.max()) > 0.5
    ref = _run(rast, sc.cams, dep.cpu().numpy(), alp.cpu().numpy(), nrm.cpu().numpy(), 0.1, 4)
    assert ref[0] > 0


def test_plane_with_matching_normals_has_zero_loss(rast):
    rng = np.random.default_rng(5)
    W, H, f = 50, 40, 44.0
    cam = (W, H, f, f, 24.6, 19.3, 0.1)
    nrm = np.array([0.2, -0.3, -1.0])
    nrm /= np.linalg.norm(nrm)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    r = np.stack([(xs - cam[4]) / f, (ys - cam[5]) / f, np.ones_like(xs)])
    D = (-2.0 * abs(nrm[2])) / np.einsum("i,ihw->hw", nrm, r)
    a = rng.uniform(0.3, 1.0, (H, W))
    n_img = a[None] * nrm[:, None, None]
    ref = _run(rast, [cam], D.ravel().astype(np.float32), a.ravel().astype(np.float32),
               n_img.ravel().astype(np.float32), 1.0, 5)
    assert abs(ref[0]) < 1e-5
