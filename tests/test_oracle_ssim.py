"""Pins of the oracle's rendering loss with SSIM against facts other than
itself (no GPU).

- the window sum is scipy's Gaussian filter with zero padding (library),
- the SSIM map equals a per-pixel brute force with two-pass weighted
  variances (different arithmetic from the oracle's E[x^2] - mu^2),
- closed forms: SSIM(x, x) = 1; constant images; y = a x + b in the
  interior, where the structure term is (2 a var + C2)/((1 + a^2) var + C2),
- symmetry SSIM(x, y) = SSIM(y, x),
- the analytic gradient against central differences of the loss,
- lambda2 = 0 reduces the loss to the two L1 means,
- planted mistakes in the derivative each fail one of the checks.
Sources: DROID-Splat Sec. 3.3 (eqn rnd_loss), supplementary S1.2 (lambda2
= 0.2), and Wang et al.'s SSIM index that the paper cites.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ssim as S

R = S.WINDOW // 2


def _img(rng, h, w, lo=0.0, hi=1.0):
    return rng.uniform(lo, hi, (h, w))


def _scipy_window_sum(img):
    return ndimage.gaussian_filter(np.asarray(img, np.float64), sigma=S.SIGMA, mode="constant",
                                   cval=0.0, truncate=(R + 0.25) / S.SIGMA)


def test_window_is_scipy_gaussian_filter():
    rng = np.random.default_rng(0)
    for (h, w) in [(7, 9), (23, 31), (40, 17)]:
        x = _img(rng, h, w)
        assert np.abs(S.window_sum(x) - _scipy_window_sum(x)).max() < 1e-14
    g = S.window_1d()
    assert g.size == 11 and abs(g.sum() - 1.0) < 1e-15 and np.allclose(g, g[::-1], 0, 0)


def _brute_ssim(x, y):
    """Per pixel: weighted means and two-pass weighted (co)variances over the
    zero-padded 11 x 11 window, then Wang et al.'s formula."""
    h, w = x.shape
    g = S.window_1d()
    w2 = np.outer(g, g)
    xp = np.zeros((h + 2 * R, w + 2 * R))
    yp = np.zeros_like(xp)
    xp[R:R + h, R:R + w] = x
    yp[R:R + h, R:R + w] = y
    out = np.zeros((h, w))
    for i in range(h):
        for j in range(w):
            a = xp[i:i + S.WINDOW, j:j + S.WINDOW]
            b = yp[i:i + S.WINDOW, j:j + S.WINDOW]
            mx, my = (w2 * a).sum(), (w2 * b).sum()
            vx = (w2 * (a - mx) ** 2).sum()
            vy = (w2 * (b - my) ** 2).sum()
            cv = (w2 * (a - mx) * (b - my)).sum()
            out[i, j] = ((2 * mx * my + S.C1) * (2 * cv + S.C2)
                         / ((mx * mx + my * my + S.C1) * (vx + vy + S.C2)))
    return out


def test_map_matches_brute_force():
    rng = np.random.default_rng(1)
    for (h, w) in [(9, 13), (16, 12)]:
        x, y = _img(rng, h, w), _img(rng, h, w)
        m = S.ssim_map(x, y)[0]
        assert np.abs(m - _brute_ssim(x, y)).max() < 1e-12


def test_identity_and_symmetry():
    rng = np.random.default_rng(2)
    x, y = _img(rng, 20, 24), _img(rng, 20, 24)
    s, g = S.ssim_grad(x, x)
    assert np.abs(s - 1.0).max() < 1e-13
    # the map is maximal at y = x, so its sum is stationary there
    assert np.abs(g).max() < 1e-9
    assert np.abs(S.ssim_map(x, y)[0] - S.ssim_map(y, x)[0]).max() < 1e-13


def test_constant_images_interior():
    a, b = 0.3, 0.7
    x = np.full((30, 30), a)
    y = np.full((30, 30), b)
    m = S.ssim_map(x, y)[0][R:-R, R:-R]
    # w * x^2 - mu^2 cancels in FP64: an error of a few 1e-16 over C2 = 9e-4
    assert np.abs(m - (2 * a * b + S.C1) / (a * a + b * b + S.C1)).max() < 1e-11


@pytest.mark.parametrize("a,b", [(0.5, 0.2), (1.7, -0.3), (-0.8, 0.9)])
def test_affine_pair_interior(a, b):
    """y = a x + b: var_y = a^2 var_x, cov = a var_x at every interior pixel."""
    rng = np.random.default_rng(3)
    x = _img(rng, 36, 40)
    y = a * x + b
    mx = _scipy_window_sum(x)
    vx = _scipy_window_sum(x * x) - mx * mx
    my = a * mx + b
    ref = ((2 * mx * my + S.C1) / (mx * mx + my * my + S.C1)
           * (2 * a * vx + S.C2) / ((1 + a * a) * vx + S.C2))
    m = S.ssim_map(x, y)[0]
    assert np.abs(m - ref)[R:-R, R:-R].max() < 1e-11


def _frames(rng, sizes):
    P = sum(w * h for w, h in sizes)
    rgb = rng.uniform(0, 1, 3 * P)
    t_rgb = rng.uniform(0, 1, 3 * P)
    depth = rng.uniform(0.5, 4, P)
    t_depth = np.where(rng.uniform(0, 1, P) < 0.2, 0.0, rng.uniform(0.5, 4, P))
    return rgb, depth, t_rgb, t_depth


def fd_error(seed=4, every=1):
    """Largest |analytic - central difference| / max |analytic| over every
    `every`-th colour and depth value of two small frames."""
    rng = np.random.default_rng(seed)
    sizes = [(9, 7), (6, 11)]
    rgb, depth, t_rgb, t_depth = _frames(rng, sizes)
    l1, l2 = 0.8, 0.2

    def loss(r, d):
        return S.render_loss(r, d, t_rgb, t_depth, l1, l2, sizes)[0]

    _, g_rgb, g_dep, _, _ = S.render_loss(rgb, depth, t_rgb, t_depth, l1, l2, sizes)
    h = 1e-6
    err = 0.0
    for i in range(0, rgb.size, every):
        e = np.zeros_like(rgb)
        e[i] = h
        num = (loss(rgb + e, depth) - loss(rgb - e, depth)) / (2 * h)
        err = max(err, abs(g_rgb[i] - num))
    for i in range(0, depth.size, every):
        e = np.zeros_like(depth)
        e[i] = h
        num = (loss(rgb, depth + e) - loss(rgb, depth - e)) / (2 * h)
        err = max(err, abs(g_dep[i] - num))
    return err / np.abs(g_rgb).max()


@pytest.mark.slow
def test_gradient_matches_central_differences():
    assert fd_error() < 1e-6


def test_lambda2_zero_is_l1():
    rng = np.random.default_rng(5)
    sizes = [(10, 8), (7, 5)]
    rgb, depth, t_rgb, t_depth = _frames(rng, sizes)
    loss = S.render_loss(rgb, depth, t_rgb, t_depth, 0.9, 0.0, sizes)[0]
    ref, off = 0.0, 0
    for (w, h) in sizes:
        P = w * h
        ref += 0.9 * np.mean(np.abs(rgb[3 * off:3 * (off + P)] - t_rgb[3 * off:3 * (off + P)]))
        m = t_depth[off:off + P] > 0
        ref += 0.1 * np.mean(np.abs(depth[off:off + P] - t_depth[off:off + P])[m])
        off += P
    assert abs(loss - ref) < 1e-13


def test_loss_value_matches_brute_force():
    rng = np.random.default_rng(6)
    sizes = [(12, 9)]
    rgb, depth, t_rgb, t_depth = _frames(rng, sizes)
    loss, _, _, _, ssim = S.render_loss(rgb, depth, t_rgb, t_depth, 0.9, 0.2, sizes)
    img, tgt = rgb.reshape(3, 9, 12), t_rgb.reshape(3, 9, 12)
    ref = np.mean([_brute_ssim(img[c], tgt[c]).mean() for c in range(3)])
    assert abs(ssim[0] - ref) < 1e-13
    m = t_depth > 0
    want = (0.9 * (0.8 * np.abs(rgb - t_rgb).mean() + 0.2 * (1 - ref))
            + 0.1 * np.abs(depth - t_depth)[m].mean())
    assert abs(loss - want) < 1e-13


# ------------------------------------------------------------------ planted mistakes
def _mutant(kind):
    """ssim_map with one plausible mistake in its derivative."""
    orig = S.ssim_map

    def m(x, y):
        Sm, A, B, C = orig(x, y)
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        mx, my = S.window_sum(x), S.window_sum(y)
        if kind == "drop_var_mu":      # forgets var_x's dependence on mu_x
            A = A + 2.0 * mx * B
        elif kind == "cov_factor":     # dS/dcov without its factor 2
            C = 0.5 * C
        elif kind == "swap_mu":        # mu_y where mu_x belongs
            A = A + 2.0 * mx * B - 2.0 * my * B
        return Sm, A, B, C
    return m


@pytest.mark.parametrize("kind", ["drop_var_mu", "cov_factor", "swap_mu"])
def test_planted_mistakes_fail(kind, monkeypatch):
    monkeypatch.setattr(S, "ssim_map", _mutant(kind))
    assert fd_error(every=7) > 1e-3
