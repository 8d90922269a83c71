"""Pins of the oracle's L1 loss (no GPU).

The L1 terms of DROID-Splat's rendering objective (eqn rnd_loss, Sec. 3.3;
weights in supplementary S1.2), read as per-frame means with the depth term
over pixels that have a target depth:
    L = sum_f [ mean_{c,p} |RGB - RGB*| + w_d mean_{p: D* > 0} |D - D*| ].
The value is pinned against a per-pixel loop over each frame, the gradient
against central differences of that loop, and planted mistakes in the
oracle's source must fail one of the two.
"""
import inspect
import types

import numpy as np
import pytest

import oracle
from oracle import loss as oloss

SIZES = [(7, 5), (3, 11), (1, 1), (13, 2)]


def _images(seed, sizes, invalid=0.3, ties=True):
    rng = np.random.default_rng(seed)
    P = sum(w * h for w, h in sizes)
    rgb = rng.uniform(0, 1, 3 * P)
    t_rgb = rng.uniform(0, 1, 3 * P)
    depth = rng.uniform(0.5, 4, P)
    t_depth = rng.uniform(0.5, 4, P)
    t_depth[rng.uniform(size=P) < invalid] = 0.0
    if ties:  # a few exact ties, where sign(0) = 0 applies
        k = rng.choice(3 * P, 3, replace=False)
        t_rgb[k] = rgb[k]
        k = rng.choice(P, 2, replace=False)
        t_depth[k] = depth[k]
    return rgb, depth, t_rgb, t_depth


def _loop_loss(rgb, depth, t_rgb, t_depth, wd, sizes):
    """The objective written out pixel by pixel."""
    total = 0.0
    off = 0
    for (w, h) in sizes:
        s = 0.0
        for c in range(3):
            for y in range(h):
                for x in range(w):
                    i = 3 * off + c * w * h + y * w + x
                    s += abs(rgb[i] - t_rgb[i])
        total += s / (3 * w * h)
        sd, cnt = 0.0, 0
        for y in range(h):
            for x in range(w):
                i = off + y * w + x
                if t_depth[i] > 0:
                    sd += abs(depth[i] - t_depth[i])
                    cnt += 1
        if cnt:
            total += wd * sd / cnt
        off += w * h
    return total


@pytest.mark.parametrize("seed,wd", [(0, 1.0), (1, 0.1), (2, 0.0)])
def test_loss_value_matches_per_pixel_loop(seed, wd, fn=None):
    fn = fn or oracle.loss_l1
    rgb, depth, t_rgb, t_depth = _images(seed, SIZES)
    loss, _, _, g_a = fn(rgb, depth, t_rgb, t_depth, wd, SIZES)
    ref = _loop_loss(rgb, depth, t_rgb, t_depth, wd, SIZES)
    assert abs(loss - ref) <= 1e-13 * max(1.0, abs(ref))
    assert np.all(g_a == 0)


@pytest.mark.parametrize("seed,wd", [(3, 1.0), (4, 0.37)])
def test_loss_gradient_matches_central_differences(seed, wd, fn=None):
    """Every colour and depth value.  L is piecewise linear, so a central
    difference with a step below the distance to the nearest kink is the
    exact slope, and at an exact tie it is 0 = sign(0)."""
    fn = fn or oracle.loss_l1
    rgb, depth, t_rgb, t_depth = _images(seed, SIZES)
    _, g_rgb, g_depth, _ = fn(rgb, depth, t_rgb, t_depth, wd, SIZES)
    for arr, t_arr, g in ((rgb, t_rgb, g_rgb), (depth, t_depth, g_depth)):
        for i in range(arr.size):
            d = abs(arr[i] - t_arr[i])
            h = 1e-3 if d == 0 else min(1e-3, d / 4)
            x0 = arr[i]
            arr[i] = x0 + h
            lp = _loop_loss(rgb, depth, t_rgb, t_depth, wd, SIZES)
            arr[i] = x0 - h
            lm = _loop_loss(rgb, depth, t_rgb, t_depth, wd, SIZES)
            arr[i] = x0
            fd = (lp - lm) / (2 * h)
            assert abs(g[i] - fd) <= 1e-9 * max(abs(fd), 1e-3), (i, g[i], fd)


def test_frame_without_target_depth_has_no_depth_term():
    sizes = [(4, 3), (5, 2)]
    rgb, depth, t_rgb, t_depth = _images(5, sizes, invalid=0.0, ties=False)
    t_depth[:12] = 0.0  # frame 0 has no valid target depth
    loss, _, g_d, _ = oracle.loss_l1(rgb, depth, t_rgb, t_depth, 1.0, sizes)
    assert np.all(g_d[:12] == 0) and np.all(g_d[12:] != 0)
    assert abs(loss - _loop_loss(rgb, depth, t_rgb, t_depth, 1.0, sizes)) < 1e-13


MUTANTS = [
    ("mean_over_P", "np.abs(diff).sum() / (3.0 * P)", "np.abs(diff).sum() / P"),
    ("grad_over_P", "np.sign(diff) / (3.0 * P)", "np.sign(diff) / P"),
    ("depth_count_all", "cnt = m.sum()", "cnt = P"),
    ("depth_sign", "depth_weight * np.sign(dd) / cnt", "depth_weight * np.sign(-dd) / cnt"),
    ("depth_unmasked", "np.where(m, depth_weight * np.sign(dd) / cnt, 0.0)",
     "depth_weight * np.sign(dd) / cnt"),
    ("no_depth_weight_grad", "depth_weight * np.sign(dd) / cnt", "np.sign(dd) / cnt"),
]


def _mutant(orig, bad):
    src = inspect.getsource(oloss)
    assert src.count(orig) == 1
    mod = types.ModuleType("loss_mutant")
    exec(compile(src.replace(orig, bad), "loss_mutant", "exec"), mod.__dict__)
    return mod.loss_l1


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_loss_mistake_is_caught(name, orig, bad):
    fn = _mutant(orig, bad)
    caught = False
    for check in (lambda: test_loss_value_matches_per_pixel_loop(1, 0.1, fn),
                  lambda: test_loss_gradient_matches_central_differences(4, 0.37, fn)):
        try:
            check()
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name} passed the loss pins"
