"""Pins of the oracle's median-depth mode (no GPU).

Sec. 3.3 names MonoGS's median depth as the depth the renderer outputs: the
depth at which a pixel's transmittance first falls below 1/2.  Read as: the
z of the first blended entry k (front to back) with T_k (1 - a_k) < 1/2, or
0 where T never falls below 1/2; its gradient reaches that entry's z only.
- brute force over all Gaussians x all pixels (tests/brute.py),
- closed forms for layered Gaussians centred on one pixel (first, second or
  no crossing), and for the gradient of one pixel's median depth (dz/dmu is
  the third row of the camera rotation),
- invariants: the median is 0 or one of the pixel's blended depths; colours
  do not move it; RGB and alpha equal the blended mode's,
- central differences of the loss through every parameter group and the
  twist, gated on the decision hash (which includes the median entry).
"""
import copy
import math

import numpy as np
import pytest

import brute
import oracle
from paper_2411_17660_amd import scenes

import test_oracle_fd as fd

A_MAX = float(np.float32(0.99))
Y00 = 0.5 / math.sqrt(math.pi)


@pytest.mark.parametrize("seed,n,frames,tile", [(0, 60, 1, (16, 16)), (2, 150, 2, (32, 8)),
                                                (4, 90, 3, (8, 8))])
def test_median_matches_brute_force(seed, n, frames, tile):
    sc = scenes.tiny_scene(seed=seed, n=n, W=48, H=32, f=36.0, n_frames=frames, sh_degree=1,
                           ls_mean=-2.6, opacity_sigma=1.5)
    r = oracle.forward(sc, tile=tile, median=True)
    ref = brute.render_median(sc)
    hits = 0
    for (_, d, _), bd in zip(r.frames(), ref):
        assert np.abs(d - bd).max() < 1e-12
        hits += int((bd > 0).sum())
    assert hits > 50   # the scenes do cross 1/2 at many pixels


def _stack(opacity_logits, zs, W=40, H=30):
    n = len(zs)
    means = np.array([[0.0, 0.0, z] for z in zs], np.float32)
    sh = np.full((n, 1, 3), 0.3, np.float32)
    return scenes.Scene(means, np.full((n, 3), -3.0, np.float32),
                        np.tile(np.array([[1, 0, 0, 0]], np.float32), (n, 1)),
                        np.array(opacity_logits, np.float32), sh, 0,
                        [(W, H, 30.0, 30.0, 20.0, 15.0, 0.2)],
                        np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None].astype(np.float32))


def _sig(o):
    return min(A_MAX, 1.0 / (1.0 + math.exp(-float(np.float32(o)))))


@pytest.mark.parametrize("logits,zs", [
    ([0.5, -0.2], [2.0, 3.0]),          # a1 = 0.62: crosses at the first
    ([-0.9, -0.4], [2.0, 3.0]),         # 0.29, 0.40: T = 0.71, 0.43 -> second
    ([-1.5, -2.0], [2.0, 3.0]),         # 0.18, 0.12: T = 0.72 -> never
    ([-0.9, -0.4, 2.0], [3.5, 2.0, 2.5]),  # input order differs from depth order
])
def test_layered_closed_form(logits, zs):
    sc = _stack(logits, zs)
    _, d, _ = oracle.forward(sc, median=True).frames()[0]
    T, want = 1.0, 0.0
    for k in sorted(range(len(zs)), key=lambda k: zs[k]):
        T *= 1.0 - _sig(logits[k])
        if T < 0.5:
            want = float(np.float32(zs[k]))
            break
    assert abs(d[15, 20] - want) < 1e-14


def test_single_pixel_gradient_closed_form():
    """With only G_D = 1 at one pixel, dL/dmu of the median Gaussian is the
    third row of R (identity pose: (0, 0, 1)); every other gradient is 0."""
    sc = _stack([-0.9, -0.4, 2.0], [3.5, 2.0, 2.5])
    r = oracle.forward(sc, median=True)
    P = r.P
    Gd = np.zeros(P)
    Gd[15 * 40 + 20] = 1.0
    g = r.backward(np.zeros(3 * P), Gd, np.zeros(P))
    # depth order 2.0 (a 0.40), 2.5 (a 0.88): T = 0.60, 0.07 -> Gaussian 2 (z 2.5)
    want = np.zeros((3, 3))
    want[2] = (0.0, 0.0, 1.0)
    np.testing.assert_allclose(g["means"], want, atol=1e-14)
    for k in ("log_scales", "quats", "opacity", "sh"):
        assert np.abs(g[k]).max() < 1e-14, k


def test_invariants():
    sc = scenes.tiny_scene(seed=5, n=120, W=40, H=30, f=30.0, n_frames=2, sh_degree=2,
                           ls_mean=-2.5, opacity_sigma=1.5)
    rb = oracle.forward(sc)
    rm = oracle.forward(sc, median=True)
    for (c1, _, a1), (c2, d2, a2) in zip(rb.frames(), rm.frames()):
        assert np.array_equal(c1, c2) and np.array_equal(a1, a2)
    # the median is 0 or the depth of one of the frame's kept Gaussians
    zs = []
    for f in range(2):
        pr = brute.project(sc, f)
        zs.append(pr["z"][pr["keep"]])
    for f, (_, d, _) in enumerate(rm.frames()):
        for v in np.unique(d):
            assert v == 0.0 or np.abs(zs[f] - v).min() < 1e-12
    # colours do not move it
    sc2 = copy.copy(sc)
    sc2.sh = (sc.sh * np.float32(-1.7)).astype(np.float32)
    for (_, d1, _), (_, d2, _) in zip(rm.frames(), oracle.forward(sc2, median=True).frames()):
        assert np.array_equal(d1, d2)
    assert int((rm.depth_flat > 0).sum()) > 100


def _loss_median(sc, G):
    r = oracle.forward(sc, f64=True, median=True)
    return (float(r.rgb_flat @ G[0] + r.depth_flat @ G[1] + r.alpha_flat @ G[2]),
            r.decision_hash)


@pytest.mark.parametrize("seed", [31, 32])
def test_gradients_match_central_differences(seed):
    sc = fd._as64(scenes.tiny_scene(seed=seed, n=24, W=40, H=30, f=32.0, n_frames=2,
                                    sh_degree=2, ls_mean=-2.2, opacity_sigma=1.5))
    r = oracle.forward(sc, f64=True, median=True)
    rng = np.random.default_rng(seed)
    G = (rng.normal(size=3 * r.P), rng.normal(size=r.P), rng.normal(size=r.P))
    grads = r.backward(*G)
    base = r.decision_hash
    used = bad = 0
    for name in ("means", "log_scales", "quats", "opacity", "sh"):
        arr = getattr(sc, name)
        ga = grads[name].reshape(arr.shape)
        scale = np.sqrt(np.mean(ga ** 2)) + 1e-30
        for fi in rng.choice(arr.size, size=min(arr.size, 36), replace=False):
            idx = np.unravel_index(fi, arr.shape)
            x0 = arr[idx]
            h = 1e-5 * max(abs(x0), 0.1)
            arr[idx] = x0 + h
            lp, hp = _loss_median(sc, G)
            arr[idx] = x0 - h
            lm, hm = _loss_median(sc, G)
            arr[idx] = x0
            if hp != base or hm != base:
                continue
            used += 1
            num = (lp - lm) / (2 * h)
            if not fd._check(ga[idx], num, scale):
                bad += 1
                print("mismatch", name, idx, ga[idx], num)
    # twist, left perturbation of each frame's pose
    tw = grads["twist"]
    for f in range(2):
        for k in range(6):
            p0 = sc.poses[f].copy()
            eps = 1e-6
            sc.poses[f] = fd._exp_left(p0, k, eps)
            lp, hp = _loss_median(sc, G)
            sc.poses[f] = fd._exp_left(p0, k, -eps)
            lm, hm = _loss_median(sc, G)
            sc.poses[f] = p0
            if hp != base or hm != base:
                continue
            used += 1
            num = (lp - lm) / (2 * eps)
            if not fd._check(tw[f, k], num, np.abs(tw).max()):
                bad += 1
                print("twist mismatch", f, k, tw[f, k], num)
    assert used >= 120
    assert bad == 0
