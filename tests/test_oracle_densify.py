"""Pins of the oracle's densification support against facts other than
itself (no GPU).

- The screen-space gradient that the ADC statistic sums is pinned by
  central differences through the principal point: moving c_x (c_y) by h
  moves every projected mean u (v) of the frame by h and nothing else, so
  dL/dc_x is the frame's sum of dL/du (one Gaussian: its own dL/du).
- MCMC noise: the covariance against scipy's rotations, the gate's values
  at the threshold, at full opacity and far below.
- MCMC relocation: one copy changes nothing; N copies composited at the
  centre give back the source opacity; the integral of the composited
  opacity along a line through the centre equals the source's (scipy
  quadrature); planted mistakes in the scale rule fail that check.
Sources: DROID-Splat Sec. 3.3 and supplementary S1.2 (ADC or MCMC
densification, lr_noise), and the MCMC densification method it cites.
"""
import copy
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial.transform import Rotation

import oracle
from oracle import densify as D
from paper_2411_17660_amd import scenes


def _shift_cam(sc, f, dcx, dcy):
    s = copy.copy(sc)
    cams = list(sc.cams)
    W, H, fx, fy, cx, cy, near = cams[f]
    cams[f] = (W, H, fx, fy, cx + dcx, cy + dcy, near)
    s.cams = cams
    return s


def _loss(sc, G):
    r = oracle.forward(sc, f64=True)
    return float(r.rgb_flat @ G[0] + r.depth_flat @ G[1] + r.alpha_flat @ G[2]), r.decision_hash


@pytest.mark.parametrize("seed,n", [(3, 1), (4, 1), (5, 12)])
def test_screen_gradient_is_derivative_in_principal_point(seed, n):
    sc = scenes.tiny_scene(seed=seed, n=n, W=40, H=30, f=32.0, n_frames=2, sh_degree=1,
                           ls_mean=-1.8, ls_sigma=0.2, spread=0.3, opacity_sigma=0.5)
    r = oracle.forward(sc, f64=True)
    rng = np.random.default_rng(seed)
    G = (rng.normal(size=3 * r.P), rng.normal(size=r.P), rng.normal(size=r.P))
    r.backward(*G)
    sg = r.screen_grads().reshape(2, n, 10)
    keep = r.records()["keep"].reshape(2, n).astype(bool)
    h = 2.0 ** -12   # exact in FP32 at these principal points
    checked = 0
    for f in range(2):
        for axis in (0, 1):
            d = (h, 0.0) if axis == 0 else (0.0, h)
            lp, hp = _loss(_shift_cam(sc, f, *d), G)
            lm, hm = _loss(_shift_cam(sc, f, -d[0], -d[1]), G)
            if hp != r.decision_hash or hm != r.decision_hash:
                continue
            num = (lp - lm) / (2 * h)
            an = sg[f, keep[f], axis].sum()
            assert abs(an - num) <= 1e-4 * max(abs(an), 1e-3), (f, axis, an, num)
            checked += 1
    assert checked >= 3


def test_stats_are_sums_over_kept_records():
    sc = scenes.tiny_scene(seed=6, n=80, W=48, H=32, f=36.0, n_frames=3, sh_degree=2,
                           ls_mean=-2.6)
    r = oracle.forward(sc)
    G = scenes.upstream(1, sc)
    r.backward(*[g.astype(np.float64) for g in G])
    acc, cnt = D.densify_stats(r)
    sg = r.screen_grads().reshape(3, sc.n, 10)
    keep = r.records()["keep"].reshape(3, sc.n).astype(bool)
    g = 7
    want = sum(math.hypot(sg[f, g, 0], sg[f, g, 1]) for f in range(3) if keep[f, g])
    assert abs(acc[g] - want) < 1e-15 and cnt[g] == keep[:, g].sum()
    assert np.all(cnt <= 3) and np.all(acc >= 0) and np.all(acc[cnt == 0] == 0)


def test_noise_covariance_and_gate():
    rng = np.random.default_rng(7)
    n = 64
    q = rng.normal(size=(n, 4))
    ls = rng.normal(-3, 0.5, (n, 3))
    logit = rng.normal(0, 3, n)
    eps = rng.normal(size=(n, 3))
    mu = rng.normal(size=(n, 3))
    out = D.mcmc_noise(mu, ls, q, logit, eps, 0.37)
    Rs = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    for i in range(n):
        cov = Rs[i] @ np.diag(np.exp(2 * ls[i])) @ Rs[i].T
        o = 1 / (1 + math.exp(-logit[i]))
        gate = 1 / (1 + math.exp(100 * (o - 0.995)))
        np.testing.assert_allclose(out[i], mu[i] + 0.37 * gate * cov @ eps[i], rtol=1e-12,
                                   atol=1e-15)
    assert abs(D.gate(0.995) - 0.5) < 1e-15
    assert abs(D.gate(1.0) - 1 / (1 + math.exp(0.5))) < 1e-15 and D.gate(0.5) > 1 - 1e-15


def _composite_centre(o_new, N):
    return 1 - (1 - o_new) ** N


@pytest.mark.parametrize("o,N", [(0.3, 2), (0.9, 3), (0.05, 7), (0.999, 2), (0.6, 16)])
def test_relocation_rule(o, N):
    o_new, f = D.relocated_opacity_scale(o, N)
    assert abs(_composite_centre(o_new, N) - o) < 1e-13
    s = 1.7
    lhs = integrate.quad(lambda x: 1 - (1 - o_new * math.exp(-x * x / (2 * (f * s) ** 2))) ** N,
                         -np.inf, np.inf, epsabs=1e-13, epsrel=1e-12)[0]
    rhs = o * s * math.sqrt(2 * math.pi)
    assert abs(lhs - rhs) < 1e-9 * rhs
    assert D.relocated_opacity_scale(o, 1) == pytest.approx((o, 1.0), rel=1e-14)


def test_relocate_copies_and_leaves_others():
    rng = np.random.default_rng(8)
    n, K = 20, 4
    p = dict(means=rng.normal(size=(n, 3)), log_scales=rng.normal(-3, 0.3, (n, 3)),
             quats=rng.normal(size=(n, 4)), opacity=rng.normal(0, 2, n),
             sh=rng.normal(size=(n, K, 3)))
    src = -np.ones(n, np.int64)
    src[[2, 5, 11]] = [7, 7, 3]
    out = D.mcmc_relocate(p["means"], p["log_scales"], p["quats"], p["opacity"], p["sh"], src)
    m, ls, q, lo, sh = out
    untouched = [g for g in range(n) if g not in (2, 5, 11, 7, 3)]
    for g in untouched:
        assert np.array_equal(m[g], p["means"][g]) and lo[g] == p["opacity"][g]
    for g, i, N in ((2, 7, 3), (5, 7, 3), (11, 3, 2), (7, 7, 3), (3, 3, 2)):
        assert np.array_equal(m[g], p["means"][i]) and np.array_equal(sh[g], p["sh"][i])
        assert np.array_equal(q[g], p["quats"][i])
        o = 1 / (1 + math.exp(-p["opacity"][i]))
        o_new, f = D.relocated_opacity_scale(o, N)
        assert abs(1 / (1 + math.exp(-lo[g])) - o_new) < 1e-14
        np.testing.assert_allclose(ls[g], p["log_scales"][i] + math.log(f), rtol=0, atol=1e-14)


@pytest.mark.parametrize("mut", ["power", "no_binomial_sign"])
def test_planted_mistakes_in_the_scale_rule_fail(mut, monkeypatch):
    def bad(o, N):
        o_new = 1.0 - (1.0 - o) ** (1.0 / N)
        den = 0.0
        for j in range(1, N + 1):
            for k in range(j):
                sgn = 1.0 if mut == "no_binomial_sign" else (-1.0) ** k
                root = (k + 1) if mut == "power" else math.sqrt(k + 1)
                den += math.comb(j - 1, k) * sgn * o_new ** (k + 1) / root
        return o_new, o / den
    monkeypatch.setattr(D, "relocated_opacity_scale", bad)
    with pytest.raises(AssertionError):
        test_relocation_rule(0.6, 4)
