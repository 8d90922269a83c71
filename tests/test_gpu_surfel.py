"""Parity of the 2D surfel forward (gsr_forward_surfel, through the C-ABI)
against the PyTorch FP64 surfel oracle (oracle/surfel.py).

Integer artefacts: the kept set and the pixel boxes are equal.  Images (RGB,
depth, alpha, normal) are within 1e-4 absolute on the pixels the oracle
does not flag; a pixel is flagged where some decision sits within the FP32
error of its threshold (alpha near 1/255, with a band widened by the
conditioning 1/sin of the intersection's two planes; T near 1e-4; the 0.99
clamp; or the disk and low-pass terms within 1e-3 of each other)."""
import numpy as np
import pytest

from oracle import surfel as S
from paper_2411_17660_amd import scenes
from gpu_util import IMG_TOL, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    from paper_2411_17660_amd.raster import Rasterizer
    return Rasterizer(0)


def _surfel_scene(seed, n, W, H, f, frames, deg, ls_mean=-2.6):
    sc = scenes.tiny_scene(seed=seed, n=n, W=W, H=H, f=f, n_frames=frames, sh_degree=deg,
                           ls_mean=ls_mean, ls_sigma=0.3, opacity_sigma=1.5)
    sc.log_scales = np.ascontiguousarray(sc.log_scales[:, :2])
    return sc


def _oracle(sc):
    t = S.to64
    return S.render(t(sc.means), t(sc.log_scales), t(sc.quats), t(sc.opacity), t(sc.sh),
                    sc.sh_degree, sc.cams, t(sc.poses), sc.background)


def _check(rast, sc, tile, label):
    import torch
    print(f"[surfel] {label} n={sc.n} F={sc.n_frames} tile={tile}", flush=True)
    d = to_dev(sc)
    rgb, dep, alp, nrm = rast.forward_surfel(d["means"], d["log_scales"], d["quats"],
                                             d["opacity"], d["sh"], d["poses"], sc.cams,
                                             sc.sh_degree, sc.background, tile=tile)
    torch.cuda.synchronize()
    rgb, dep, alp, nrm = (x.cpu().numpy().astype(np.float64) for x in (rgb, dep, alp, nrm))
    L = rast.debug_lists()
    ref = _oracle(sc)
    off = 0
    errs = np.zeros(4)
    flagged = 0
    n = sc.n
    for f, fr in enumerate(ref):
        W, H = int(sc.cams[f][0]), int(sc.cams[f][1])
        P = W * H
        ok = (fr["flags"] == 0).ravel()
        flagged += int((~ok).sum())
        got = [rgb[3 * off:3 * (off + P)].reshape(3, P), dep[off:off + P].reshape(1, P),
               alp[off:off + P].reshape(1, P), nrm[3 * off:3 * (off + P)].reshape(3, P)]
        want = [fr["rgb"].detach().numpy().reshape(3, P), fr["depth"].detach().numpy().reshape(1, P),
                fr["alpha"].detach().numpy().reshape(1, P),
                fr["normal"].detach().numpy().reshape(3, P)]
        for i, (g, w) in enumerate(zip(got, want)):
            errs[i] = max(errs[i], float(np.abs(g - w)[:, ok].max(initial=0.0)))
        # kept set and boxes
        box = fr["box"]
        keep = box[:, 0] >= 0
        nt = L["ntiles"][f * n:(f + 1) * n]
        assert np.array_equal(nt > 0, keep), (label, f)
        sq = L["square"].reshape(-1, 2)[f * n:(f + 1) * n]
        assert np.array_equal(sq[keep, 0] & 0xffff, box[keep, 0])
        assert np.array_equal(sq[keep, 0] >> 16, box[keep, 1])
        assert np.array_equal(sq[keep, 1] & 0xffff, box[keep, 2])
        assert np.array_equal(sq[keep, 1] >> 16, box[keep, 3])
        off += P
    print(f"[surfel]   max err rgb {errs[0]:.3g} depth {errs[1]:.3g} alpha {errs[2]:.3g} "
          f"normal {errs[3]:.3g}; flagged px {flagged} of {off}", flush=True)
    assert np.all(errs <= IMG_TOL), errs
    assert float(alp.max()) > 0.3


@pytest.mark.parametrize("seed,n,frames,deg,W,H,tile", [
    (0, 60, 1, 0, 48, 32, (16, 16)), (1, 300, 2, 3, 97, 61, (8, 8)),
    (2, 800, 3, 1, 130, 70, (32, 8)), (3, 500, 2, 2, 33, 17, (32, 16))])
def test_surfel_forward_matches_oracle(rast, seed, n, frames, deg, W, H, tile):
    sc = _surfel_scene(seed, n, W, H, 0.8 * W, frames, deg)
    _check(rast, sc, tile, f"surfels{seed}")


def test_surfel_forward_larger_scene(rast):
    sc = _surfel_scene(7, 3000, 128, 96, 100.0, 2, 3, ls_mean=-3.0)
    _check(rast, sc, (16, 16), "surfels-3000")


def test_surfel_images_do_not_depend_on_tile_shape(rast):
    import torch
    sc = _surfel_scene(8, 1200, 150, 90, 110.0, 2, 3)
    d = to_dev(sc)
    outs = []
    for tile in ((16, 16), (8, 8), (32, 16)):
        o = rast.forward_surfel(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                                d["poses"], sc.cams, sc.sh_degree, sc.background, tile=tile)
        torch.cuda.synchronize()
        outs.append([x.clone() for x in o])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_backward_after_surfel_forward_is_a_state_error(rast):
    import torch
    from paper_2411_17660_amd.native import GsrError
    sc = _surfel_scene(9, 40, 32, 24, 26.0, 1, 0)
    d = to_dev(sc)
    rast.forward_surfel(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                        d["poses"], sc.cams, sc.sh_degree)
    P = sc.n_pixels
    with pytest.raises(GsrError):
        rast.backward(torch.zeros(3 * P, device="cuda"), torch.zeros(P, device="cuda"),
                      torch.zeros(P, device="cuda"))
