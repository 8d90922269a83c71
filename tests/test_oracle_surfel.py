"""Pins of the 2DGS surfel oracle (oracle/surfel.py) against facts other
than itself (no GPU).

- SH colour: the basis equals the 3D oracle's (itself pinned to scipy);
- a surfel facing the camera: the ray-disk intersection has the closed
  form u = ((x - c_x) z / f_x - mu_x) / s_u, the depth is z and the normal
  (0, 0, -1); alpha is sigma max(G, G_lp) in closed form;
- any pose and rotation: (u, v) and the depth equal a ray-plane
  intersection computed geometrically (ray K^-1 (x, y, 1), the disk's plane
  through its centre with its normal, coordinates along its axes);
- the pixel box is the bounding box of the disk of radius r_a sampled along
  its boundary and projected, united with the low-pass square; a disk whose
  nearest point passes the near plane is culled;
- an edge-on surfel: the object-space Gaussian vanishes off its line and the
  screen-space low-pass exp(-|x - c|^2) sets alpha;
- layered "over" of two surfels and their order; zero opacity; permutation;
- depth distortion: each surfel rendered alone gives its alpha and depth per
  pixel; blending them in centre-depth order by hand and summing
  w_i w_j (z_i - z_j)^2 over all pairs i < j reproduces the map (and the
  depth, alpha and normal maps), a surfel alone has none, and two surfels at
  one depth have none;
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


@pytest.mark.parametrize("seed", [4, 5, 6, 7])
def test_box_is_the_bounding_box_of_the_projected_disk(seed):
    """The pixel box is [ceil, floor] of the extremes of the disk of radius
    r_a = sqrt(2 ln(255 sigma)) mapped to the image (sampled densely along
    its boundary), united with the low-pass square around the centre; a
    tilted disk whose nearest point passes the near plane is culled."""
    rng = np.random.default_rng(seed)
    W, H, f, cx, cy, near = 200, 160, 90.0, 99.4, 80.7, 0.2
    n = 12
    mu = np.stack([rng.uniform(-0.8, 0.8, n), rng.uniform(-0.6, 0.6, n),
                   rng.uniform(1.0, 3.0, n)], 1)
    q = rng.normal(size=(n, 4))
    ls = np.log(rng.uniform(0.05, 0.3, (n, 2)))
    lo = rng.normal(0, 1.5, n)
    out = _render(mu, ls, q, lo, np.full((n, 1, 3), 0.3), 0, [(W, H, f, f, cx, cy, near)],
                  _ident())[0]
    th = np.linspace(0, 2 * np.pi, 40001)
    K = np.array([[f, 0, cx], [0, f, cy], [0, 0, 1.0]])
    checked = 0
    for g in range(n):
        o = 1 / (1 + math.exp(-lo[g]))
        if o <= S.A_MIN:
            assert out["box"][g, 0] < 0
            continue
        ra = math.sqrt(2 * math.log(o / S.A_MIN))
        rl = math.sqrt(math.log(o / S.A_MIN))
        R = _rot(q[g])
        P = mu[g][:, None] + np.exp(ls[g, 0]) * R[:, :1] * (ra * np.cos(th)) \
            + np.exp(ls[g, 1]) * R[:, 1:2] * (ra * np.sin(th))
        if P[2].min() <= near:
            assert out["box"][g, 0] < 0
            continue
        p = K @ P
        px, py = p[0] / p[2], p[1] / p[2]
        c = (f * mu[g, 0] / mu[g, 2] + cx, f * mu[g, 1] / mu[g, 2] + cy)
        x0 = min(px.min(), c[0] - rl)
        x1 = max(px.max(), c[0] + rl)
        y0 = min(py.min(), c[1] - rl)
        y1 = max(py.max(), c[1] + rl)
        want = (max(0, math.ceil(x0)), min(W - 1, math.floor(x1)),
                max(0, math.ceil(y0)), min(H - 1, math.floor(y1)))
        if not (want[0] <= want[1] and want[2] <= want[3]):
            assert out["box"][g, 0] < 0
            continue
        # a sampled extreme sits within ~1e-6 px of the true one
        near_int = [abs(v - round(v)) < 1e-4 for v in (x0, x1, y0, y1)]
        if any(near_int):
            continue
        assert tuple(out["box"][g]) == want, (g, out["box"][g], want)
        checked += 1
    assert checked >= 6


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


def test_distortion_is_the_pair_sum_of_separately_rendered_surfels():
    from paper_2411_17660_amd import scenes
    sc = scenes.tiny_scene(seed=21, n=7, W=32, H=24, f=22.0, n_frames=1, sh_degree=0,
                           ls_mean=-1.6, ls_sigma=0.2, opacity_sigma=0.3)
    ls = sc.log_scales[:, :2]
    lo = np.clip(sc.opacity, -1.0, 0.5)          # alpha <= 0.63: T stays above 1e-4
    full = _render(sc.means, ls, sc.quats, lo, sc.sh, 0, sc.cams, sc.poses)[0]
    H, W = 24, 32
    a_i, z_i, n_i = [], [], []
    for g in range(sc.n):
        o = np.full(sc.n, -40.0)
        o[g] = lo[g]
        one = _render(sc.means, ls, sc.quats, o, sc.sh, 0, sc.cams, sc.poses)[0]
        a = one["alpha"].numpy()
        assert np.all(one["dist"].numpy() == 0)
        a_i.append(a)
        z_i.append(np.where(a > 0, one["depth"].numpy() / np.where(a > 0, a, 1), 0))
        n_i.append(np.where(a > 0, one["normal"].numpy() / np.where(a > 0, a, 1), 0))
    mc = sc.means @ sc.poses[0, :, :3].T + sc.poses[0, :, 3]
    order = np.argsort(mc[:, 2].astype(np.float32), kind="stable")
    T = np.ones((H, W))
    w = []
    for g in order:
        w.append(a_i[g] * T)
        T = T * (1 - a_i[g])
    zs = [z_i[g] for g in order]
    dist = np.zeros((H, W))
    for j in range(len(w)):
        for i in range(j):
            dist += w[i] * w[j] * (zs[i] - zs[j]) ** 2
    assert dist.max() > 1e-3
    assert np.abs(full["dist"].numpy() - dist).max() < 1e-12
    assert np.abs(full["depth"].numpy() - sum(wi * zi for wi, zi in zip(w, zs))).max() < 1e-12
    assert np.abs(full["alpha"].numpy() - (1 - T)).max() < 1e-12
    nsum = sum(wi * n_i[g] for wi, g in zip(w, order))
    assert np.abs(full["normal"].numpy() - nsum).max() < 1e-12


def test_pair_count_by_brute_force():
    """pairs = sum over surfels of the pixels inside its box that have not
    stopped when it comes, counted here by walking each pixel's list."""
    from paper_2411_17660_amd import scenes
    sc = scenes.tiny_scene(seed=23, n=30, W=24, H=18, f=20.0, n_frames=1, sh_degree=0,
                           ls_mean=-1.8, ls_sigma=0.3, opacity_sigma=2.0)
    out = _render(sc.means, sc.log_scales[:, :2], sc.quats, sc.opacity, sc.sh, 0, sc.cams,
                  sc.poses)[0]
    box, order = out["box"], out["order"]
    one = []
    for g in order:                      # each surfel's alpha map, alone
        o = np.full(sc.n, -40.0)
        o[g] = sc.opacity[g]
        one.append(_render(sc.means, sc.log_scales[:, :2], sc.quats, o, sc.sh, 0, sc.cams,
                           sc.poses)[0]["alpha"].numpy())
    count = 0
    for y in range(18):
        for x in range(24):
            T = 1.0
            for k, g in enumerate(order):
                if not (box[g, 0] <= x <= box[g, 1] and box[g, 2] <= y <= box[g, 3]):
                    continue
                count += 1
                a = one[k][y, x]
                if a >= S.A_MIN:
                    if T * (1 - a) < S.T_MIN:
                        break
                    T *= 1 - a
    assert out["pairs"] == count and count > 100


def test_distortion_vanishes_for_coplanar_fronto_parallel_surfels():
    cams = [(40, 30, 30.0, 30.0, 20.0, 15.0, 0.2)]
    out = _render(np.array([[0.0, 0, 2.0], [0.01, 0.02, 2.0]]), np.log(np.full((2, 2), 0.1)),
                  np.tile([[1.0, 0, 0, 0]], (2, 1)), np.array([0.2, -0.1]),
                  np.zeros((2, 1, 3)), 0, cams, _ident())[0]
    d = out["dist"].numpy()
    assert np.abs(d).max() < 1e-13 and out["alpha"].numpy().max() > 0.5


def test_autograd_matches_central_differences():
    sc = _tiny(5, n=6, F=1)
    rng = np.random.default_rng(5)
    G = [S.to64(rng.normal(size=s)) for s in ((3, 24, 32), (24, 32), (24, 32), (3, 24, 32),
                                             (24, 32))]
    poses = S.to64(sc.poses)

    def loss(means, ls, quats, opac, sh, twist):
        fr = S.render(means, ls, quats, opac, sh, 1, sc.cams, poses, sc.background, twist)[0]
        return ((fr["rgb"] * G[0]).sum() + (fr["depth"] * G[1]).sum()
                + (fr["alpha"] * G[2]).sum() + (fr["normal"] * G[3]).sum()
                + (fr["dist"] * G[4]).sum())
    args = (S.to64(sc.means, True), S.to64(sc.log_scales[:, :2], True),
            S.to64(sc.quats, True), S.to64(sc.opacity, True), S.to64(sc.sh, True),
            S.to64(np.zeros((1, 6)), True))
    assert torch.autograd.gradcheck(loss, args, eps=1e-7, atol=1e-6, rtol=1e-5)


def _plane_depth(n, d, cam):
    """Depth map of the plane n . P = d seen through cam: the ray
    K^-1 (x, y, 1) meets it at D = d / (n . K^-1 (x, y, 1))."""
    W, H, fx, fy, cx, cy = cam[:6]
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    r = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)])
    return d / np.einsum("i,ihw->hw", n, r)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_depth_normals_of_a_plane_are_its_normal(seed):
    rng = np.random.default_rng(seed)
    cam = (36, 28, 30.0, 32.0, 17.3, 13.9, 0.1)
    n = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), -1.0])
    n /= np.linalg.norm(n)                  # faces the camera (n_z < 0)
    d = -2.0 * abs(n[2])                     # through (0, 0, 2)
    D = _plane_depth(n, d, cam)
    assert D.min() > 0
    N, valid = S.depth_normals(torch.from_numpy(D), cam)
    N = N.numpy()
    assert valid.numpy()[1:-1, 1:-1].all() and not valid.numpy()[0].any()
    err = np.abs(N[:, 1:-1, 1:-1] - n[:, None, None]).max()
    assert err < 1e-12, err
    assert np.all(N[:, 0] == 0) and np.all(N[:, :, -1] == 0)


def test_normal_consistency_closed_forms():
    cam = (20, 16, 18.0, 18.0, 9.5, 7.5, 0.1)
    D = np.full((16, 20), 3.0)
    Dt = torch.from_numpy(D)
    rng = np.random.default_rng(3)
    alpha = torch.from_numpy(rng.uniform(0.2, 1.0, (16, 20)))
    # normal map alpha * N with N = (0, 0, -1): every interior term vanishes
    nm = torch.zeros(3, 16, 20, dtype=torch.float64)
    nm[2] = -alpha
    loss, term = S.normal_consistency(Dt, alpha, nm, cam)
    assert abs(float(loss)) < 1e-15
    # a normal map rotated by 90 degrees: each term is alpha, the mean over
    # the (W-2)(H-2) interior pixels
    nm2 = torch.zeros(3, 16, 20, dtype=torch.float64)
    nm2[0] = alpha
    loss2, term2 = S.normal_consistency(Dt, alpha, nm2, cam)
    want = alpha.numpy()[1:-1, 1:-1].sum() / (18 * 14)
    assert abs(float(loss2) - want) < 1e-14
    assert np.all(term2.numpy()[0] == 0)


def test_normal_consistency_autograd_matches_central_differences():
    cam = (9, 7, 8.0, 9.0, 4.2, 3.1, 0.1)
    rng = np.random.default_rng(4)
    D = S.to64(2.0 + 0.2 * rng.normal(size=(7, 9)), True)
    a = S.to64(rng.uniform(0.1, 1.0, (7, 9)), True)
    nm = S.to64(rng.normal(size=(3, 7, 9)), True)
    f = lambda D, a, nm: S.normal_consistency(D, a, nm, cam)[0]       # noqa: E731
    assert torch.autograd.gradcheck(f, (D, a, nm), eps=1e-7, atol=1e-7, rtol=1e-6)


def test_window_equals_the_whole_image_cropped():
    from paper_2411_17660_amd import scenes
    sc = _tiny(6, n=20, F=2)
    ls = sc.log_scales[:, :2]
    full = _render(sc.means, ls, sc.quats, sc.opacity, sc.sh, 1, sc.cams, sc.poses, sc.background)
    win = S.render(*[S.to64(a) for a in (sc.means, ls, sc.quats, sc.opacity, sc.sh)], 1, sc.cams,
                   S.to64(sc.poses), sc.background, window=(5, 17, 3, 11))
    for a, b in zip(full, win):
        for k in ("rgb", "depth", "alpha", "normal", "dist"):
            assert np.array_equal(a[k].numpy()[..., 3:12, 5:18], b[k].numpy()), k
        assert np.array_equal(a["flags"][3:12, 5:18], b["flags"])
        assert np.array_equal(a["box"], b["box"])


@pytest.mark.parametrize("group,idx,val", [("means", (1,), np.nan), ("ls", (0,), np.inf),
                                           ("quats", (2,), -np.inf), ("opac", (), np.nan),
                                           ("sh", (3, 0), np.nan)])
def test_nonfinite_surfel_is_removed(group, idx, val):
    """A surfel with a NaN or infinite parameter is culled in every frame: the
    maps equal those of the scene without it, and its gradients are 0 while
    every other surfel's equal the reduced scene's."""
    sc = _tiny(6, n=14)
    arrs = dict(means=sc.means.astype(np.float64), ls=sc.log_scales[:, :2].astype(np.float64),
                quats=sc.quats.astype(np.float64), opac=sc.opacity.astype(np.float64),
                sh=sc.sh.astype(np.float64))
    g = 5
    base = _render(arrs["means"], arrs["ls"], arrs["quats"], arrs["opac"], arrs["sh"], 1,
                   sc.cams, sc.poses, sc.background)
    assert all(fr["box"][g, 0] >= 0 for fr in base)  # visible in both frames
    bad = {k: v.copy() for k, v in arrs.items()}
    bad[group][(g,) + idx] = val
    keep = np.arange(sc.n) != g
    red = {k: v[keep] for k, v in arrs.items()}

    def run(a):
        ts = {k: torch.tensor(v, requires_grad=True) for k, v in a.items()}
        out = S.render(ts["means"], ts["ls"], ts["quats"], ts["opac"], ts["sh"], 1, sc.cams,
                       S.to64(sc.poses), sc.background)
        rng = np.random.default_rng(1)
        L = 0.0
        for fr in out:
            for k in ("rgb", "depth", "alpha", "normal", "dist"):
                L = L + (fr[k] * torch.tensor(rng.normal(size=tuple(fr[k].shape)))).sum()
        L.backward()
        return out, {k: t.grad.numpy() for k, t in ts.items()}
    ob, gb = run(bad)
    orf, gr = run(red)
    for fa, fb in zip(ob, orf):
        assert fa["box"][g, 0] == -1
        for k in ("rgb", "depth", "alpha", "normal", "dist"):
            assert np.array_equal(fa[k].detach().numpy(), fb[k].detach().numpy()), k
    for k in gb:
        assert np.all(gb[k][g] == 0), k
        np.testing.assert_allclose(np.delete(gb[k], g, axis=0), gr[k], rtol=1e-12, atol=1e-14)
