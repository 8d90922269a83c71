"""Finite-difference pins of the oracle's analytic backward (no GPU).

Central differences in FP64 of L = <G_C,RGB> + <G_D,D> + <G_A,Alpha> for
every parameter group and each twist component (T <- Exp(eps e_k) T, left
perturbation, xi = (rho, phi)).  A coordinate is used only where the decision
hash (squares, tile lists, blended sets, stop positions, clamp states) is the
same at +eps and -eps as at the base point; the scenes keep every mean well
inside the Jacobian guard and in front of the near plane.
Sources: DROID-Splat Sec. 3.3 (gradients to the Gaussians and, through the
rendering objective, to keyframe poses) and supplementary S1.3.
"""
import copy
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2411_17660_amd import scenes


def _as64(sc):
    s = copy.copy(sc)
    for k in ("means", "log_scales", "quats", "opacity", "sh", "poses"):
        setattr(s, k, np.array(getattr(sc, k), dtype=np.float64))
    return s


def _loss(sc, G):
    r = oracle.forward(sc, f64=True)
    return (float(r.rgb_flat @ G[0] + r.depth_flat @ G[1] + r.alpha_flat @ G[2]),
            r.decision_hash)


def _check(an, fd, scale):
    return abs(an - fd) <= 1e-5 * max(abs(an), 1e-2 * scale)


@pytest.mark.parametrize("seed,deg,frames,bg", [(11, 3, 2, (0.1, 0.2, 0.3)),
                                                (12, 1, 1, (0.0, 0.0, 0.0)),
                                                (13, 2, 3, (0.5, 0.4, 0.3))])
def test_parameter_gradients_match_central_differences(seed, deg, frames, bg):
    sc = _as64(scenes.tiny_scene(seed=seed, n=24, W=40, H=30, f=32.0, n_frames=frames,
                                 sh_degree=deg, ls_mean=-2.3, opacity_sigma=1.0, background=bg))
    r = oracle.forward(sc, f64=True)
    rng = np.random.default_rng(seed)
    G = (rng.normal(size=3 * r.P), rng.normal(size=r.P), rng.normal(size=r.P))
    grads = r.backward(*G)
    base_hash = r.decision_hash
    used = bad = 0
    for name in ("means", "log_scales", "quats", "opacity", "sh"):
        arr = getattr(sc, name)
        ga = grads[name].reshape(arr.shape)
        scale = np.sqrt(np.mean(ga ** 2)) + 1e-30
        flat_idx = rng.choice(arr.size, size=min(arr.size, 40), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, arr.shape)
            x0 = arr[idx]
            h = 1e-5 * max(abs(x0), 0.1)
            arr[idx] = x0 + h
            lp, hp = _loss(sc, G)
            arr[idx] = x0 - h
            lm, hm = _loss(sc, G)
            arr[idx] = x0
            if hp != base_hash or hm != base_hash:
                continue
            fd = (lp - lm) / (2 * h)
            used += 1
            if not _check(ga[idx], fd, scale):
                bad += 1
                print("mismatch", name, idx, ga[idx], fd)
    assert used >= 150
    assert bad == 0


def _exp_left(pose, k, eps):
    """Exp(eps e_k) T for xi = (rho, phi); rotation parts via scipy."""
    R, t = pose[:, :3], pose[:, 3]
    if k < 3:
        dt = np.zeros(3)
        dt[k] = eps
        return np.concatenate([R, (t + dt)[:, None]], 1)
    phi = np.zeros(3)
    phi[k - 3] = eps
    Rp = Rotation.from_rotvec(phi).as_matrix()
    return np.concatenate([Rp @ R, (Rp @ t)[:, None]], 1)


@pytest.mark.parametrize("seed,deg", [(21, 3), (22, 0), (23, 2)])
def test_twist_gradient_matches_central_differences(seed, deg):
    sc = _as64(scenes.tiny_scene(seed=seed, n=30, W=40, H=30, f=32.0, n_frames=2, sh_degree=deg,
                                 ls_mean=-2.3))
    r = oracle.forward(sc, f64=True)
    rng = np.random.default_rng(seed)
    G = (rng.normal(size=3 * r.P), rng.normal(size=r.P), rng.normal(size=r.P))
    tw = r.backward(*G)["twist"]
    base = r.decision_hash
    used = 0
    for f in range(2):
        P0 = sc.poses[f].copy()
        for k in range(6):
            eps = 1e-7
            sc.poses[f] = _exp_left(P0, k, eps)
            lp, hp = _loss(sc, G)
            sc.poses[f] = _exp_left(P0, k, -eps)
            lm, hm = _loss(sc, G)
            sc.poses[f] = P0
            if hp != base or hm != base:
                continue
            used += 1
            fd = (lp - lm) / (2 * eps)
            assert abs(tw[f, k] - fd) <= 2e-6 * max(abs(tw[f, k]), 1e-2 * np.abs(tw[f]).max()), \
                (f, k, tw[f, k], fd)
    assert used >= 10


def test_colour_clamp_and_direction_paths():
    """A scene where some raw colours are negative (clamped) and SH3 terms are
    large, so the view-direction path (and its camera-centre part in the
    twist) carries much of the gradient."""
    sc = _as64(scenes.tiny_scene(seed=31, n=20, n_frames=2, sh_degree=3, ls_mean=-2.2))
    rng = np.random.default_rng(0)
    sc.sh[:, 1:, :] = rng.normal(0, 1.0, size=sc.sh[:, 1:, :].shape)
    sc.sh[:, 0, :] = rng.normal(-0.2, 1.0, size=sc.sh[:, 0, :].shape)
    r = oracle.forward(sc, f64=True)
    assert (r.records()["raw0"] < 0).any()
    G = (rng.normal(size=3 * r.P), np.zeros(r.P), np.zeros(r.P))
    g = r.backward(*G)
    base = r.decision_hash
    checked = 0
    for gi in range(sc.n):
        for a in range(3):
            x0 = sc.means[gi, a]
            h = 1e-6
            sc.means[gi, a] = x0 + h
            lp, hp = _loss(sc, G)
            sc.means[gi, a] = x0 - h
            lm, hm = _loss(sc, G)
            sc.means[gi, a] = x0
            if hp != base or hm != base:
                continue
            fd = (lp - lm) / (2 * h)
            checked += 1
            assert abs(g["means"][gi, a] - fd) <= 2e-6 * max(abs(fd), 1e-3), (gi, a)
    assert checked > 30
    P0 = sc.poses[0].copy()
    for k in range(3):
        sc.poses[0] = _exp_left(P0, k, 1e-7)
        lp, _ = _loss(sc, G)
        sc.poses[0] = _exp_left(P0, k, -1e-7)
        lm, _ = _loss(sc, G)
        sc.poses[0] = P0
        fd = (lp - lm) / 2e-7
        assert abs(g["twist"][0, k] - fd) <= 2e-6 * max(abs(fd), 1e-3)


# The EWA projection's Jacobian guard (the 3DGS lineage's frustum guard, which
# the paper inherits through its renderer): J is evaluated at t_x/t_z clamped
# to +-1.3 W/(2 f_x) (likewise y).  These scenes put every Gaussian beyond the
# image on one or both axes, large enough that its square still reaches it.
GUARD = 1.3


def guard_scene(seed, deg, n=36):
    return scenes.tiny_scene(seed=seed, n=n, W=40, H=30, f=32.0, n_frames=2, sh_degree=deg,
                             ls_mean=-1.0, ls_sigma=0.3, zrange=(1.5, 3.0), outside=(1.35, 1.8))


def clamped_records(sc, rec):
    """(clamped in x, clamped in y) per record, from the projected means:
    t_x/t_z = (u - c_x)/f_x."""
    cx = np.repeat([c[4] for c in sc.cams], sc.n)
    cy = np.repeat([c[5] for c in sc.cams], sc.n)
    fx = np.repeat([c[2] for c in sc.cams], sc.n)
    fy = np.repeat([c[3] for c in sc.cams], sc.n)
    W = np.repeat([c[0] for c in sc.cams], sc.n)
    H = np.repeat([c[1] for c in sc.cams], sc.n)
    clx = np.abs(rec["u"] - cx) / fx > GUARD * W / (2 * fx)
    cly = np.abs(rec["v"] - cy) / fy > GUARD * H / (2 * fy)
    return clx, cly


@pytest.mark.parametrize("seed,deg", [(41, 2), (42, 3)])
def test_gradients_through_the_jacobian_guard(seed, deg):
    """Central differences on Gaussians outside the guard: every parameter
    group (all coordinates of the Gaussians that have a clamped kept record)
    and all six twist components of both frames."""
    sc = _as64(guard_scene(seed, deg))
    r = oracle.forward(sc, f64=True)
    rec = r.records()
    keep = rec["keep"].astype(bool)
    clx, cly = clamped_records(sc, rec)
    assert (keep & clx).sum() >= 10 and (keep & cly).sum() >= 10
    assert (keep & clx & cly).sum() >= 5
    clamped_g = np.unique(np.nonzero(keep & (clx | cly))[0] % sc.n)
    rng = np.random.default_rng(seed)
    G = (rng.normal(size=3 * r.P), rng.normal(size=r.P), rng.normal(size=r.P))
    grads = r.backward(*G)
    base = r.decision_hash
    used = bad = 0
    for name in ("means", "log_scales", "quats", "opacity", "sh"):
        arr = getattr(sc, name)
        ga = grads[name].reshape(arr.shape)
        scale = np.sqrt(np.mean(ga ** 2)) + 1e-30
        for g in clamped_g:
            coords = list(np.ndindex(arr.shape[1:])) if arr.ndim > 1 else [()]
            if name == "sh":
                coords = coords[:6]
            for c in coords:
                idx = (g,) + tuple(c)
                x0 = arr[idx]
                h = 1e-5 * max(abs(x0), 0.1)
                arr[idx] = x0 + h
                lp, hp = _loss(sc, G)
                arr[idx] = x0 - h
                lm, hm = _loss(sc, G)
                arr[idx] = x0
                if hp != base or hm != base:
                    continue
                fd = (lp - lm) / (2 * h)
                used += 1
                if not _check(ga[idx], fd, scale):
                    bad += 1
                    print("mismatch", name, idx, ga[idx], fd)
    assert used >= 300
    assert bad == 0
    tw = grads["twist"]
    tused = 0
    for f in range(2):
        P0 = sc.poses[f].copy()
        for k in range(6):
            eps = 1e-7
            sc.poses[f] = _exp_left(P0, k, eps)
            lp, hp = _loss(sc, G)
            sc.poses[f] = _exp_left(P0, k, -eps)
            lm, hm = _loss(sc, G)
            sc.poses[f] = P0
            if hp != base or hm != base:
                continue
            tused += 1
            fd = (lp - lm) / (2 * eps)
            assert abs(tw[f, k] - fd) <= 2e-6 * max(abs(tw[f, k]), 1e-2 * np.abs(tw[f]).max()), \
                (f, k, tw[f, k], fd)
    assert tused >= 10
