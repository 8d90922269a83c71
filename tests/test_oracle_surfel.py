"""Pins of the 2DGS surfel oracle (oracle/surfel.py) against facts other
than itself (no GPU).

- SH colour: the basis equals the 3D oracle's (itself pinned to scipy);
- a surfel facing the camera: the ray-disk intersection has the closed
  form u = ((x - c_x) z / f_x - mu_x) / s_u, the depth is z and the normal
  (0, 0, -1); alpha is sigma max(G, G_lp) in closed form;
- any pose and rotation: (u, v) and the depth equal a ray-plane
  intersection computed geometrically (ray K^-1 (x, y, 1), the disk's plane
  through its centre with its normal, coordinates along its axes);
- an edge-on surfel: the object-space Gaussian vanishes off its line and the
  screen-space low-pass exp(-|x - c|^2) sets alpha;
- layered "over" of two surfels and their order; zero opacity; permutation;
- autograd against central differences (torch.autograd.gradcheck).
Sources: DROID-Splat Sec. 3.3 (2D surfels compared in tab:renderer) and the
2DGS method it cites.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import surfel as S

A_MAX = S.A_MAX


def _render(means, ls, quats, opac, sh, deg, cams, poses, bg=(0.0, 0.0, 0.0), twist=None):
    t = lambda a: S.to64(a)                                       # noqa: E731
    return S.render(t(means), t(ls), t(quats), t(opac), t(sh), deg, cams, t(poses), bg,
                    twist=twist)


def _ident(F=1):
    return np.repeat(np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None], F, 0)


def test_sh_colour_matches_3d_oracle_basis():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    sh = rng.normal(size=(50, 16, 3))
    got = S._sh_colour(S.to64(sh), 3, S.to64(d)).numpy()
    Y = np.stack([oracle.sh_basis(3, d[i]) for i in range(50)])
    want = np.maximum(np.einsum("nk,nkc->nc", Y, sh) + 0.5, 0.0)
    assert np.abs(got - want).max() < 1e-14


def test_fronto_parallel_closed_form():
    W, H, f, cx, cy = 48, 36, 40.0, 23.7, 17.2
    mu = np.array([[0.1, -0.05, 2.0]])
    ls = np.log(np.array([[0.08, 0.05]]))
    o = np.array([1.2])
    sh = np.full((1, 1, 3), 0.4)
    out = _render(mu, ls, [[1, 0, 0, 0]], o, sh, 0, [(W, H, f, f, cx, cy, 0.2)], _ident())[0]
    sig = 1 / (1 + math.exp(-1.2))
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    u = ((xs - cx) * 2.0 / f - 0.1) / 0.08
    v = ((ys - cy) * 2.0 / f + 0.05) / 0.05
    G = np.exp(-0.5 * (u * u + v * v))
    c = (f * 0.1 / 2.0 + cx, -f * 0.05 / 2.0 + cy)
    Glp = np.exp(-((xs - c[0]) ** 2 + (ys - c[1]) ** 2))
    a = np.minimum(A_MAX, sig * np.maximum(G, Glp))
    a = np.where(a >= S.A_MIN, a, 0.0)
    box = out["box"][0]
    inb = (xs >= box[0]) & (xs <= box[1]) & (ys >= box[2]) & (ys <= box[3])
    a = np.where(inb, a, 0.0)
    assert np.abs(out["alpha"].numpy() - a).max() < 1e-13
    obj = (G >= Glp) & (a > 0)
    assert np.abs(out["depth"].numpy()[obj] - 2.0 * a[obj]).max() < 1e-13
    nz = out["normal"].numpy()
    assert np.abs(nz[2] + a).max() < 1e-13 and np.abs(nz[:2]).max() < 1e-15
    # the box holds every pixel where alpha >= 1/255
    full = np.minimum(A_MAX, sig * np.maximum(G, Glp))
    assert not np.any((full >= S.A_MIN) & ~inb)


def _rot(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ray_plane_intersection_any_pose(seed):
    rng = np.random.default_rng(seed)
    W, H, f, cx, cy = 40, 30, 32.0, 20.3, 14.6
    Rp = _rot(rng.normal(size=4) * [3, 0.2, 0.2, 0.2])
    tp = rng.normal(0, 0.1, 3)
    pose = np.concatenate([Rp, tp[:, None]], 1)[None]
    mc = np.array([rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), rng.uniform(1.5, 2.5)])
    mu = Rp.T @ (mc - tp)
    q = rng.normal(size=4)
    q[0] += 2.0                      # mostly facing the camera
    ls = np.log(rng.uniform(0.06, 0.12, 2))
    out = _render(mu[None], ls[None], q[None], [3.0], np.full((1, 1, 3), 0.3), 0,
                  [(W, H, f, f, cx, cy, 0.2)], pose)[0]
    R = Rp @ _rot(q)
    tu, tv, tw = R[:, 0], R[:, 1], R[:, 2]
    Kinv = np.linalg.inv(np.array([[f, 0, cx], [0, f, cy], [0, 0, 1]]))
    sig = 1 / (1 + math.exp(-np.float32(3.0)))
    alpha, depth = out["alpha"].numpy(), out["depth"].numpy()
    c = (f * mc[0] / mc[2] + cx, f * mc[1] / mc[2] + cy)
    checked = 0
    for y in range(H):
        for x in range(W):
            d = Kinv @ np.array([x, y, 1.0])
            t = (tw @ mc) / (tw @ d)
            P = t * d
            u, v = (P - mc) @ tu / np.exp(ls[0]), (P - mc) @ tv / np.exp(ls[1])
            G = math.exp(-0.5 * (u * u + v * v))
            Glp = math.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2))
            a = min(A_MAX, sig * max(G, Glp))
            if a < 0.02 or G < 1.01 * Glp or a > 0.98 * A_MAX:
                continue
            assert abs(alpha[y, x] - a) < 1e-12
            assert abs(depth[y, x] - a * P[2]) < 1e-12
            checked += 1
    assert checked > 20


def test_edge_on_surfel_uses_the_low_pass():
    W, H, f, cx, cy = 40, 30, 32.0, 20.0, 15.0
    # normal along x: the disk contains the viewing ray through its centre
    q = np.array([math.cos(math.pi / 4), 0.0, math.sin(math.pi / 4), 0.0])
    out = _render([[0.0, 0.0, 2.0]], np.log([[0.05, 0.05]]), q[None], [2.0],
                  np.full((1, 1, 3), 0.3), 0, [(W, H, f, f, cx, cy, 0.2)], _ident())[0]
    sig = 1 / (1 + math.exp(-2.0))
    alpha = out["alpha"].numpy()
    # off the column x = c_x, whose rays lie in the disk's plane
    for (x, y) in [(21, 15), (19, 16), (21, 16), (22, 15)]:
        want = min(A_MAX, sig * math.exp(-((x - cx) ** 2 + (y - cy) ** 2)))
        assert abs(alpha[y, x] - want) < 1e-12, (x, y)


def test_over_operator_and_order():
    W, H, f = 40, 30, 30.0
    cams = [(W, H, f, f, 20.0, 15.0, 0.2)]
    zs = [2.5, 1.5]
    logit = [0.3, -0.4]
    cols = [0.9, 0.2]
    sh = np.array([[[(c - 0.5) * 2 * math.sqrt(math.pi)] * 3] for c in cols])
    for perm in ([0, 1], [1, 0]):
        out = _render(np.array([[0, 0, zs[k]] for k in perm]), np.log(np.full((2, 2), 0.1)),
                      np.tile([[1.0, 0, 0, 0]], (2, 1)), np.array([logit[k] for k in perm]),
                      sh[perm], 0, cams, _ident(), (0.05, 0.1, 0.15))[0]
        T, C = 1.0, 0.0
        for k in sorted(range(2), key=lambda k: zs[k]):
            a = min(A_MAX, 1 / (1 + math.exp(-logit[k])))
            C += cols[k] * a * T
            T *= 1 - a
        assert abs(out["rgb"].numpy()[0, 15, 20] - (C + 0.05 * T)) < 1e-13
        assert abs(out["alpha"].numpy()[15, 20] - (1 - T)) < 1e-13


def _tiny(seed, n=12, F=2):
    from paper_2411_17660_amd import scenes
    sc = scenes.tiny_scene(seed=seed, n=n, W=32, H=24, f=26.0, n_frames=F, sh_degree=1,
                           ls_mean=-2.4, ls_sigma=0.2, opacity_sigma=1.0)
    return sc


def test_zero_opacity_and_permutation():
    sc = _tiny(4)
    ls = sc.log_scales[:, :2]
    base = _render(sc.means, ls, sc.quats, sc.opacity, sc.sh, 1, sc.cams, sc.poses, sc.background)
    zero = _render(sc.means, ls, sc.quats, np.full(sc.n, -30.0), sc.sh, 1, sc.cams, sc.poses,
                   sc.background)
    for fr in zero:
        assert np.allclose(fr["rgb"].numpy(), np.array(sc.background)[:, None, None], atol=0)
        assert np.all(fr["alpha"].numpy() == 0)
    perm = np.random.default_rng(4).permutation(sc.n)
    pm = _render(sc.means[perm], ls[perm], sc.quats[perm], sc.opacity[perm], sc.sh[perm], 1,
                 sc.cams, sc.poses, sc.background)
    for a, b in zip(base, pm):
        for k in ("rgb", "depth", "alpha", "normal"):
            assert np.abs(a[k].numpy() - b[k].numpy()).max() < 1e-14
    assert sum(int((fr["alpha"].numpy() > 0).sum()) for fr in base) > 200


def test_autograd_matches_central_differences():
    sc = _tiny(5, n=6, F=1)
    rng = np.random.default_rng(5)
    G = [S.to64(rng.normal(size=s)) for s in ((3, 24, 32), (24, 32), (24, 32), (3, 24, 32))]
    poses = S.to64(sc.poses)

    def loss(means, ls, quats, opac, sh, twist):
        fr = S.render(means, ls, quats, opac, sh, 1, sc.cams, poses, sc.background, twist)[0]
        return ((fr["rgb"] * G[0]).sum() + (fr["depth"] * G[1]).sum()
                + (fr["alpha"] * G[2]).sum() + (fr["normal"] * G[3]).sum())
    args = (S.to64(sc.means, True), S.to64(sc.log_scales[:, :2], True),
            S.to64(sc.quats, True), S.to64(sc.opacity, True), S.to64(sc.sh, True),
            S.to64(np.zeros((1, 6)), True))
    assert torch.autograd.gradcheck(loss, args, eps=1e-7, atol=1e-6, rtol=1e-5)
