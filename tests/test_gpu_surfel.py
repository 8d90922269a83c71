"""Parity of the 2D surfel forward and backward (gsr_forward_surfel,
gsr_backward_surfel, through the C-ABI) against the PyTorch FP64 surfel
oracle (oracle/surfel.py) and its autograd.

Integer artefacts: the kept set and the pixel boxes are equal.  Images (RGB,
depth, alpha, normal, distortion) are within 1e-4 absolute on the pixels the
oracle does not flag; a pixel is flagged where some decision sits within the
FP32 error of its threshold (ln alpha near ln(1/255) within the FP32 error
of the exponent of the term that sets alpha, which for the disk term grows
with the conditioning 1/sin of the intersection's two planes; T near 1e-4;
the 0.99 clamp; or the disk and low-pass terms within 1e-3 of each other).
Gradients: upstream gradients of all five outputs, zero on flagged pixels
(these include the pixels where a blended disk term has kappa (1 + q) above
32: its FP32 value errs by up to ~5 kappa (1 + q) ulps, and a tilted
surfel's rotation gradient cancels to ~1 % of its per-pixel terms); the bar
of the 3D backward (1e-3 relative with its floors, or 3 times the oracle's
own response to a perturbation), where the perturbation is both a 1e-6
relative jitter of the upstream and a one-ulp rounding of every FP32
operation of the intersection and of the stored surfel, except that a
component's floor is 1e-3 of 5 % (not 1 %) of its parameter group's norm:
a tilted surfel's rotation and scale gradients sum per-pixel terms of the
group's size that cancel, and FP32 arithmetic through an intersection of
conditioning up to ~30 leaves ~1e-5 of the group (measured: 1.3e-5 on a
thin, nearly edge-on surfel, every component of its rotation gradient
alike), which the 1 % floor would not admit."""

SURFEL_BLOCK = 5e-2
import numpy as np
import pytest
import torch

from oracle import surfel as S
from paper_2411_17660_amd import scenes
from gpu_util import IMG_TOL, GRAD_REL, to_dev, perturbed, assert_grad_close

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
    rgb, dep, alp, nrm, dst = rast.forward_surfel(d["means"], d["log_scales"], d["quats"],
                                                  d["opacity"], d["sh"], d["poses"], sc.cams,
                                                  sc.sh_degree, sc.background, tile=tile)
    torch.cuda.synchronize()
    rgb, dep, alp, nrm, dst = (x.cpu().numpy().astype(np.float64)
                               for x in (rgb, dep, alp, nrm, dst))
    L = rast.debug_lists()
    ref = _oracle(sc)
    off = 0
    errs = np.zeros(5)
    flagged = 0
    n = sc.n
    for f, fr in enumerate(ref):
        W, H = int(sc.cams[f][0]), int(sc.cams[f][1])
        P = W * H
        ok = ((fr["flags"] & (0xff ^ S.FLAG_COND)) == 0).ravel()
        flagged += int((~ok).sum())
        got = [rgb[3 * off:3 * (off + P)].reshape(3, P), dep[off:off + P].reshape(1, P),
               alp[off:off + P].reshape(1, P), nrm[3 * off:3 * (off + P)].reshape(3, P),
               dst[off:off + P].reshape(1, P)]
        want = [fr["rgb"].detach().numpy().reshape(3, P), fr["depth"].detach().numpy().reshape(1, P),
                fr["alpha"].detach().numpy().reshape(1, P),
                fr["normal"].detach().numpy().reshape(3, P),
                fr["dist"].detach().numpy().reshape(1, P)]
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
          f"normal {errs[3]:.3g} dist {errs[4]:.3g} (max {dst.max():.3g}); "
          f"flagged px {flagged} of {off}", flush=True)
    assert np.all(errs <= IMG_TOL), errs
    assert float(alp.max()) > 0.3
    assert float(dst.max()) > 1e-3


@pytest.mark.parametrize("seed,n,frames,deg,W,H,tile", [
    (0, 60, 1, 0, 48, 32, (16, 16)), (1, 300, 2, 3, 97, 61, (8, 8)),
    (2, 800, 3, 1, 130, 70, (32, 8)), (3, 500, 2, 2, 33, 17, (32, 16)),
    (4, 400, 2, 3, 75, 43, (16, 8))])
def test_surfel_forward_matches_oracle(rast, seed, n, frames, deg, W, H, tile):
    sc = _surfel_scene(seed, n, W, H, 0.8 * W, frames, deg)
    _check(rast, sc, tile, f"surfels{seed}")


def test_surfel_forward_larger_scene(rast):
    sc = _surfel_scene(7, 3000, 128, 96, 100.0, 2, 3, ls_mean=-3.0)
    _check(rast, sc, (16, 16), "surfels-3000")


def test_surfel_more_frames_than_one_grid_dimension(rast):
    """65,537 copies of one 4 x 4 frame in one batch: the surfel preprocess
    takes the frame from the grid's y dimension and strides past its 65,535
    limit.  Every frame's five maps must equal the single frame's bitwise."""
    one = _surfel_scene(13, 40, 4, 4, 4.0, 1, 3, ls_mean=-1.0)
    F = 65537
    sc = scenes.Scene(one.means, one.log_scales, one.quats, one.opacity, one.sh, one.sh_degree,
                      one.cams * F, np.ascontiguousarray(np.repeat(one.poses, F, axis=0)),
                      one.background)
    print(f"[surfel] one frame, then {F} copies", flush=True)
    outs = []
    for s_ in (one, sc):
        d = to_dev(s_)
        o = rast.forward_surfel(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                                d["poses"], s_.cams, s_.sh_degree, s_.background)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in o])
    assert outs[0][2].max() > 0.1
    for a, b in zip(*outs):
        assert np.array_equal(b.reshape(F, -1), np.tile(a.reshape(1, -1), (F, 1)))


def test_surfel_images_do_not_depend_on_tile_shape(rast):
    import torch
    sc = _surfel_scene(8, 1200, 150, 90, 110.0, 2, 3)
    d = to_dev(sc)
    outs = []
    for tile in ((16, 16), (8, 8), (32, 8), (16, 8), (32, 16)):
        o = rast.forward_surfel(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                                d["poses"], sc.cams, sc.sh_degree, sc.background, tile=tile)
        torch.cuda.synchronize()
        outs.append([x.clone() for x in o])
        assert len(o) == 5
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


def test_surfel_backward_after_3d_forward_is_a_state_error(rast):
    from paper_2411_17660_amd.native import GsrError
    from gpu_util import gpu_forward
    sc = scenes.tiny_scene(seed=10, n=40)
    gpu_forward(rast, sc)
    P = sc.n_pixels
    z = lambda k: torch.zeros(k, device="cuda")             # noqa: E731
    rast.sh_degree = sc.sh_degree
    with pytest.raises(GsrError):
        rast.backward_surfel(z(3 * P), z(P), z(P), z(3 * P), z(P))


def _upstream(seed, sc, flags):
    """Upstream gradients of (rgb, depth, alpha, normal, dist), FP32, zero on
    the flagged pixels."""
    rng = np.random.default_rng(seed)
    P = sc.n_pixels
    sizes = [(int(c[0]), int(c[1])) for c in sc.cams]
    keep = (flags == 0).astype(np.float32)
    offs = np.cumsum([0] + [w * h for w, h in sizes])[:-1]
    keep3 = np.concatenate([np.tile(keep[o:o + w * h], 3) for o, (w, h) in zip(offs, sizes)])
    g = [rng.normal(size=3 * P) * keep3, rng.normal(size=P) * keep, rng.normal(size=P) * keep,
         rng.normal(size=3 * P) * keep3, 5.0 * rng.normal(size=P) * keep]
    return [x.astype(np.float32) for x in g]


NAMES = ("means", "log_scales", "quats", "opacity", "sh", "twist")


def _oracle_grads(sc, jitter=None):
    """Oracle autograd of sum_o <G_o, output_o> (grads(G) -> per-parameter
    arrays); with `jitter` (a seed) the render rounds each FP32 operation of
    the intersection and the stored surfel by a random ulp."""
    t = S.to64
    params = [t(sc.means, True), t(sc.log_scales, True), t(sc.quats, True), t(sc.opacity, True),
              t(sc.sh, True), t(np.zeros((sc.n_frames, 6)), True)]
    gen = None if jitter is None else torch.Generator().manual_seed(jitter)
    out = S.render(*params[:5], sc.sh_degree, sc.cams, t(sc.poses), sc.background,
                   twist=params[5], jitter=gen)
    flags = np.concatenate([fr["flags"].ravel() for fr in out])
    maps = [torch.cat([fr["rgb"].reshape(-1) for fr in out]),
            torch.cat([fr["depth"].reshape(-1) for fr in out]),
            torch.cat([fr["alpha"].reshape(-1) for fr in out]),
            torch.cat([fr["normal"].reshape(-1) for fr in out]),
            torch.cat([fr["dist"].reshape(-1) for fr in out])]

    def grads(Gs, retain):
        loss = sum((m * torch.from_numpy(np.asarray(g, np.float64))).sum()
                   for m, g in zip(maps, Gs))
        return [x.numpy() for x in torch.autograd.grad(loss, params, retain_graph=retain)]
    return flags, maps, grads


def _check_backward(rast, sc, tile, seed, label):
    flags, _, grads = _oracle_grads(sc)
    G = _upstream(seed, sc, flags)
    g_ref = grads(G, True)
    dG = [p - np.asarray(g, np.float64) for p, g in zip(perturbed(G), G)]
    noise = [np.abs(x) for x in grads(dG, False)]
    _, _, grads_j = _oracle_grads(sc, jitter=seed)
    noise = [np.maximum(a, np.abs(b - r)) for a, b, r in zip(noise, grads_j(G, False), g_ref)]
    d = to_dev(sc)
    rast.forward_surfel(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                        d["poses"], sc.cams, sc.sh_degree, sc.background, tile=tile)
    g = rast.backward_surfel(*[torch.from_numpy(x).cuda() for x in G])
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    print(f"[surfel] backward {label} n={sc.n} F={sc.n_frames} tile={tile}: "
          f"flagged {int((flags != 0).sum())} of {flags.size}", flush=True)
    for k, r, nz in zip(NAMES[:5], g_ref[:5], noise[:5]):
        assert_grad_close(f"surfel {label}:{k}", got[k], r, noise=nz, block=SURFEL_BLOCK)
    tr = g_ref[5]
    bound = np.maximum(GRAD_REL * np.maximum(np.abs(tr), 1e-2 * np.abs(tr).max()),
                       3.0 * noise[5])
    err = np.abs(got["twist"] - tr)
    print(f"[surfel]   twist max err/bound {float((err / bound).max()):.3g}", flush=True)
    assert np.all(err <= bound)


@pytest.mark.parametrize("seed,n,frames,deg,W,H,tile", [
    (20, 40, 1, 0, 40, 30, (16, 16)), (21, 150, 2, 3, 61, 45, (8, 8)),
    (22, 250, 2, 1, 70, 50, (32, 8)), (23, 120, 1, 2, 33, 17, (32, 16)),
    (24, 700, 1, 3, 96, 64, (16, 16)), (25, 200, 2, 1, 57, 39, (16, 8))])
def test_surfel_backward_matches_oracle_autograd(rast, seed, n, frames, deg, W, H, tile):
    sc = _surfel_scene(seed, n, W, H, 0.8 * W, frames, deg)
    _check_backward(rast, sc, tile, seed, f"surfels{seed}")


def _large_facing_scene(seed, n=30, W=320, H=240, frames=2):
    """Round disks, nearly face-on, large enough that each covers most of the
    image: records with hundreds of keys."""
    sc = _surfel_scene(seed, n, W, H, 0.8 * W, frames, 1, ls_mean=-0.8)
    sc.log_scales = np.ascontiguousarray(np.repeat(sc.log_scales[:, :1], 2, 1))
    rng = np.random.default_rng(seed + 1000)
    sc.quats = np.concatenate([np.ones((n, 1)), 0.1 * rng.normal(size=(n, 3))],
                              1).astype(np.float32)
    return sc


def test_surfel_backward_large_disks_many_tiles(rast):
    """Backward parity where every record spans hundreds of tiles, so that
    the per-record reduction walks its longest lists."""
    sc = _large_facing_scene(26)
    _check_backward(rast, sc, (16, 16), 26, "large-disks")
    nt = rast.debug_lists()["ntiles"]
    print(f"[surfel] large-disks: tiles per record max {int(nt.max())}, "
          f"mean {float(nt[nt > 0].mean()):.1f}", flush=True)
    assert int(nt.max()) >= 200


def test_surfel_objective_chain_matches_oracle(rast):
    """The surfel objective end to end: rendering loss with SSIM (lambda1 0.8,
    lambda2 0.2) + 0.05 x normal consistency + 100 x the mean depth
    distortion of each frame, forward, losses and backward on each side.  On
    the GPU through the C ABI: gsr_forward_surfel, gsr_loss_render,
    gsr_normal_consistency (adding to the loss's depth and alpha gradients),
    a constant distortion upstream, gsr_backward_surfel.  The oracle renders,
    takes its loss terms of its own maps and back-propagates them.  The
    renders agree to FP32 rounding, which the terms' curvature carries into
    the upstream gradients, so the bar adds the oracle chain's response to a
    1e-7 jitter of its maps, and to a one-ulp rounding of each FP32
    operation of the intersection.  The scene has no flagged pixel (its
    surfels face the camera within ~20 degrees, so no intersection is
    ill-conditioned)."""
    import oracle
    sc = _facing_scene(85)
    sizes = [(int(c[0]), int(c[1])) for c in sc.cams]
    _, _, t_rgb, t_dep = scenes.loss_images(12, sizes)
    l1, l2, wn, wd = 0.8, 0.2, 0.05, 100.0
    f32 = lambda v: float(np.float32(v))                          # noqa: E731
    t = S.to64
    params = [t(sc.means, True), t(sc.log_scales, True), t(sc.quats, True), t(sc.opacity, True),
              t(sc.sh, True), t(np.zeros((sc.n_frames, 6)), True)]
    out = S.render(*params[:5], sc.sh_degree, sc.cams, t(sc.poses), sc.background,
                   twist=params[5])
    assert sum(int((fr["flags"] != 0).sum()) for fr in out) == 0
    maps = [torch.cat([fr[k].reshape(-1) for fr in out])
            for k in ("rgb", "depth", "alpha", "normal", "dist")]

    def upstream(m):
        """Image-space gradients of the objective at maps m (numpy FP64) and
        its value."""
        rgb, dep, alp, nrm, dst = m
        loss, g_rgb, g_dep, g_alp, _ = oracle.render_loss(rgb, dep, t_rgb, t_dep, f32(l1),
                                                          f32(l2), sizes)
        g_nrm = np.zeros_like(nrm)
        g_dst = np.zeros_like(dst)
        off = 0
        for cam, (w, h) in zip(sc.cams, sizes):
            P = w * h
            D = t(dep[off:off + P].reshape(h, w), True)
            A = t(alp[off:off + P].reshape(h, w), True)
            N = t(nrm[3 * off:3 * (off + P)].reshape(3, h, w), True)
            ln, _ = S.normal_consistency(D, A, N, cam)
            gD, gA, gN = torch.autograd.grad(f32(wn) * ln, (D, A, N))
            loss += f32(wn) * float(ln.detach()) + f32(wd) * float(dst[off:off + P].mean())
            g_dep[off:off + P] += gD.numpy().ravel()
            g_alp[off:off + P] += gA.numpy().ravel()
            g_nrm[3 * off:3 * (off + P)] = gN.numpy().ravel()
            g_dst[off:off + P] = f32(wd) / P
            off += P
        return loss, [g_rgb, g_dep, g_alp, g_nrm, g_dst]

    def grads(G, retain):
        s = sum((mp * torch.from_numpy(np.asarray(g, np.float64))).sum()
                for mp, g in zip(maps, G))
        return [x.numpy() for x in torch.autograd.grad(s, params, retain_graph=retain)]

    m64 = [mp.detach().numpy() for mp in maps]
    loss_ref, G = upstream(m64)
    g_ref = grads(G, True)
    rng = np.random.default_rng(3)
    _, Gj = upstream([a + 1e-7 * rng.standard_normal(a.shape) for a in m64])
    noise = [np.abs(x) for x in grads([a - b for a, b in zip(Gj, G)], False)]
    # and the response to a one-ulp jitter of the intersection vectors
    _, _, grads_j = _oracle_grads(sc, jitter=85)
    noise = [np.maximum(a, np.abs(b - r)) for a, b, r in zip(noise, grads_j(G, False), g_ref)]

    d = to_dev(sc)
    rgb, dep, alp, nrm, dst = rast.forward_surfel(d["means"], d["log_scales"], d["quats"],
                                                  d["opacity"], d["sh"], d["poses"], sc.cams,
                                                  sc.sh_degree, sc.background)
    tr, td = (torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in (t_rgb, t_dep))
    lr = rast.loss_render(rgb, dep, tr, td, l1, l2)
    g_nrm = torch.zeros_like(nrm)
    ln = rast.normal_consistency(sc.cams, dep, alp, nrm, wn, lr["g_depth"], lr["g_alpha"], g_nrm)
    g_dst = torch.cat([torch.full((w * h,), f32(wd) / (w * h), device="cuda") for w, h in sizes])
    g = rast.backward_surfel(lr["g_rgb"], lr["g_depth"], lr["g_alpha"], g_nrm, g_dst)
    torch.cuda.synchronize()
    off, loss_gpu = 0, float(lr["loss"].item()) + float(ln.item())
    for (w, h) in sizes:
        loss_gpu += f32(wd) * float(dst[off:off + w * h].double().mean())
        off += w * h
    print(f"[surfel] objective {loss_gpu:.9g} oracle {loss_ref:.9g}", flush=True)
    assert abs(loss_gpu - loss_ref) <= 1e-5 * abs(loss_ref)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    for k, r, nz in zip(NAMES[:5], g_ref[:5], noise[:5]):
        assert_grad_close(f"surfel objective:{k}", got[k], r, noise=nz, block=SURFEL_BLOCK)
    tw = g_ref[5]
    bound = np.maximum(GRAD_REL * np.maximum(np.abs(tw), 1e-2 * np.abs(tw).max()),
                       3.0 * noise[5])
    assert np.all(np.abs(got["twist"] - tw) <= bound)


def _facing_scene(seed, n=25):
    """A two-frame surfel scene whose rotations are near the identity (disks
    facing the camera within ~20 degrees)."""
    sc = _surfel_scene(seed, n, 40, 30, 34.0, 2, 1, ls_mean=-2.3)
    rng = np.random.default_rng(seed + 1000)
    sc.quats = np.concatenate([np.ones((n, 1)), 0.2 * rng.normal(size=(n, 3))],
                              1).astype(np.float32)
    return sc


def test_surfel_pair_count_matches_oracle(rast):
    """GSR_FLAG_COUNT_PAIRS on the surfel forward counts the (pixel, surfel)
    pairs whose box test passes before the pixel stops, exactly as the
    oracle does, on a scene with no flagged pixel (where both take the same
    stop decisions); counting leaves the images unchanged."""
    sc = _facing_scene(85)
    ref = _oracle(sc)
    assert sum(int((fr["flags"] != 0).sum()) for fr in ref) == 0
    d = to_dev(sc)
    args = (d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"], d["poses"], sc.cams,
            sc.sh_degree, sc.background)
    plain = [x.clone() for x in rast.forward_surfel(*args)]
    counted = rast.forward_surfel(*args, count_pairs=True)
    torch.cuda.synchronize()
    n = int(rast.stats()["n_pairs"])
    want = sum(fr["pairs"] for fr in ref)
    print(f"[surfel] pairs {n} oracle {want}", flush=True)
    assert n == want and n > 0
    for a, b in zip(plain, counted):
        assert torch.equal(a, b)


def test_surfel_graph_captured_step_replays_match_eager():
    """The surfel forward and backward at a fixed key capacity (no host read)
    captured in a HIP graph: every replay, with eager work and
    synchronisations between replays, equals the eager pass bitwise (images,
    distortion and every gradient)."""
    from paper_2411_17660_amd.raster import Rasterizer
    sc = _surfel_scene(13, 2000, 160, 96, 120.0, 3, 3)
    d = to_dev(sc)
    P, n, K, F = sc.n_pixels, sc.n, (sc.sh_degree + 1) ** 2, sc.n_frames
    gen = torch.Generator("cuda").manual_seed(13)
    ups = [torch.randn(k, device="cuda", generator=gen) for k in (3 * P, P, P, 3 * P, P)]
    imgs = [torch.empty(k, device="cuda") for k in (3 * P, P, P, 3 * P, P)]
    grads = dict(means=torch.empty(n, 3, device="cuda"), log_scales=torch.empty(n, 2, device="cuda"),
                 quats=torch.empty(n, 4, device="cuda"), opacity=torch.empty(n, device="cuda"),
                 sh=torch.empty(n, K, 3, device="cuda"), twist=torch.empty(F, 6, device="cuda"))
    r = Rasterizer(0)

    def step(cap):
        r.forward_surfel(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                         d["poses"], sc.cams, sc.sh_degree, sc.background, key_capacity=cap,
                         out=imgs)
        r.backward_surfel(*ups, out=grads)
    step(0)
    torch.cuda.synchronize()
    cap = r.stats()["n_keys"] + 64
    step(cap)
    torch.cuda.synchronize()
    eager = [x.clone() for x in imgs] + [v.clone() for v in grads.values()]
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
        for v in imgs + list(grads.values()):
            v.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        got = imgs + list(grads.values())
        for i, (a, b) in enumerate(zip(got, eager)):
            assert torch.equal(a, b), (rep, i)
        step(cap)
        torch.cuda.synchronize()
    r.check_overflow()
    assert float(imgs[2].max()) > 0.5


def _run_surfel(rast, sc, **kw):
    d = to_dev(sc)
    outs = rast.forward_surfel(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                               d["poses"], sc.cams, sc.sh_degree, sc.background, **kw)
    torch.cuda.synchronize()
    rast._inputs = d
    return [x.clone() for x in outs]


def _zero_upstream(sc):
    P = sc.n_pixels
    return [torch.randn(k, device="cuda") for k in (3 * P, P, P, 3 * P, P)]


def test_surfel_empty_scene(rast):
    """n = 0: background, zero depth, alpha, normal and distortion; the
    backward writes only the (zero) twist."""
    sc = _surfel_scene(30, 1, 40, 30, 32.0, 2, 1)
    sc = scenes.Scene(sc.means[:0], sc.log_scales[:0], sc.quats[:0], sc.opacity[:0], sc.sh[:0],
                      1, sc.cams, sc.poses, (0.25, 0.5, 0.75))
    rgb, dep, alp, nrm, dst = _run_surfel(rast, sc)
    P = 40 * 30
    r = rgb.cpu().numpy().reshape(2, 3, P)
    for c in range(3):
        assert np.all(r[:, c] == np.float32(sc.background[c]))
    for x in (dep, alp, nrm, dst):
        assert torch.all(x == 0)
    g = rast.backward_surfel(*_zero_upstream(sc))
    torch.cuda.synchronize()
    assert g["means"].shape == (0, 3) and torch.all(g["twist"] == 0)


def test_surfel_everything_culled(rast):
    """Every surfel behind every camera: no keys, background images, zero
    gradients everywhere."""
    sc = _surfel_scene(31, 150, 48, 32, 38.0, 2, 2)
    sc.means[:, 2] = -5.0
    rgb, dep, alp, nrm, dst = _run_surfel(rast, sc)
    assert rast.stats()["n_keys"] == 0
    assert torch.all(alp == 0) and torch.all(dst == 0) and torch.all(nrm == 0)
    g = rast.backward_surfel(*_zero_upstream(sc))
    torch.cuda.synchronize()
    for k, v in g.items():
        assert torch.all(v == 0), k


def test_surfel_fixed_capacity_and_overflow(rast):
    """A fixed key capacity equal to the key count gives the grown images
    bitwise; a third of it overflows, which gsr_check_overflow reports
    (GSR_ERR_CAPACITY) and then clears; the backward after the overflow
    stays finite (overflowed surfels' keys never reach the kernels)."""
    from paper_2411_17660_amd import native
    sc = _surfel_scene(32, 800, 96, 64, 76.8, 2, 1)
    a = _run_surfel(rast, sc)
    K = rast.stats()["n_keys"]
    b = _run_surfel(rast, sc, key_capacity=K)
    rast.check_overflow()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    _run_surfel(rast, sc, key_capacity=max(1, K // 3))
    g = rast.backward_surfel(*_zero_upstream(sc))
    torch.cuda.synchronize()
    for k, v in g.items():
        assert torch.isfinite(v).all(), k
    with pytest.raises(native.GsrError) as ei:
        rast.check_overflow()
    assert ei.value.status == 2
    rast.check_overflow()
