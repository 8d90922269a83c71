"""Rendering loss with SSIM, plain FP64 numpy (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use
this module; it shares no code with the HIP path.

The mapper's objective (DROID-Splat Sec. 3.3, eqn rnd_loss; weights in
supplementary S1.2: lambda2 = 0.2, lambda1 = 0.9 or 0.8) is, per frame,
    L_f = l1 [ (1 - l2) |I' - I*| + l2 (1 - SSIM(I', I*)) ] + (1 - l1) |Z' - Z*|
and the step sums L_f over the frames of the batch.  Readings where the
paper is silent:
  - |.| is the mean absolute error: over the 3 H W colour values, and over
    the pixels with a valid target depth (Z* > 0) for the depth term (no
    valid pixel: the term is 0);
  - SSIM is Wang et al.'s structural similarity with an 11 x 11 Gaussian
    window of standard deviation 1.5 (weights normalised to sum 1),
    C1 = (0.01 L)^2, C2 = (0.03 L)^2 with dynamic range L = 1, the window
    sums taken with zero padding so the map has the image's size (the
    3DGS lineage the paper follows), and SSIM(I', I*) the mean of the map
    over the 3 channels and all pixels;
  - the derivative of |d| at d = 0 is 0; nothing depends on alpha.

The SSIM map at pixel p of one channel, with mu = w * x (w the window,
* the zero-padded window sum), var_x = w * x^2 - mu_x^2 and
cov = w * (x y) - mu_x mu_y, is
    S = (2 mu_x mu_y + C1)(2 cov + C2) / ((mu_x^2 + mu_y^2 + C1)(var_x + var_y + C2)).
Its derivative is the chain rule through the three window sums that hold
x: with A = dS/dmu_x (var_x and cov held at their definitions), B =
dS/d(w * x^2) and C = dS/d(w * x y) at every pixel p, and the window
symmetric, d(sum_p S_p)/dx_q = (w * A)_q + 2 x_q (w * B)_q + y_q (w * C)_q.
"""
import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window_1d(size=WINDOW, sigma=SIGMA):
    """Normalised 1-D Gaussian weights g_k, k = -(size // 2) .. size // 2."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def window_sum(img):
    """Zero-padded window sum (w * img)[i, j] = sum_{a,b} w[a,b] img[i+a, j+b]
    over the 11 x 11 window w = g g^T, written out over the window's
    offsets; the output has img's shape."""
    img = np.asarray(img, np.float64)
    r = WINDOW // 2
    g = window_1d()
    w2 = np.outer(g, g)
    H, W = img.shape
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    out = np.zeros((H, W))
    for a in range(WINDOW):
        for b in range(WINDOW):
            out += w2[a, b] * pad[a:a + H, b:b + W]
    return out


def ssim_map(x, y):
    """SSIM map of two single-channel images and the partial derivatives
    (A, B, C) of each entry with respect to mu_x, w * x^2 and w * x y."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = window_sum(x), window_sum(y)
    exx, eyy, exy = window_sum(x * x), window_sum(y * y), window_sum(x * y)
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    l_num = 2.0 * mx * my + C1
    l_den = mx * mx + my * my + C1
    c_num = 2.0 * cxy + C2
    c_den = vx + vy + C2
    S = (l_num * c_num) / (l_den * c_den)
    # partials of S in the variables (mu_x, var_x, cov) ...
    dS_dmu = c_num / c_den * (2.0 * my * l_den - 2.0 * mx * l_num) / (l_den * l_den)
    dS_dvar = -S / c_den
    dS_dcov = 2.0 * l_num / (l_den * c_den)
    # ... moved to (mu_x, w*x^2, w*xy): var_x = w*x^2 - mu_x^2, cov = w*xy - mu_x mu_y
    A = dS_dmu - 2.0 * mx * dS_dvar - my * dS_dcov
    return S, A, dS_dvar, dS_dcov


def ssim_grad(x, y):
    """SSIM map of channel x against y and d(sum of the map)/dx."""
    S, A, B, C = ssim_map(x, y)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return S, window_sum(A) + 2.0 * x * window_sum(B) + y * window_sum(C)


def render_loss(rgb, depth, t_rgb, t_depth, lambda1, lambda2, sizes):
    """rgb/t_rgb packed [3,H,W] per frame, depth/t_depth [H,W] per frame,
    sizes = [(W, H)].  Returns (loss, g_rgb, g_depth, g_alpha, ssim) in FP64,
    ssim the per-frame SSIM(I', I*)."""
    rgb = np.asarray(rgb, np.float64)
    depth = np.asarray(depth, np.float64)
    t_rgb = np.asarray(t_rgb, np.float64)
    t_depth = np.asarray(t_depth, np.float64)
    g_rgb = np.zeros_like(rgb)
    g_depth = np.zeros_like(depth)
    l1, l2 = float(lambda1), float(lambda2)
    loss = 0.0
    ssims = []
    off = 0
    for (w, h) in sizes:
        P = w * h
        img = rgb[3 * off:3 * (off + P)].reshape(3, h, w)
        tgt = t_rgb[3 * off:3 * (off + P)].reshape(3, h, w)
        g = np.zeros((3, h, w))
        s_sum = 0.0
        for c in range(3):
            S, dS = ssim_grad(img[c], tgt[c])
            s_sum += S.sum()
            g[c] = dS
        ssim = s_sum / (3.0 * P)
        ssims.append(ssim)
        diff = img - tgt
        loss += l1 * ((1.0 - l2) * np.abs(diff).sum() / (3.0 * P) + l2 * (1.0 - ssim))
        g = l1 * (1.0 - l2) * np.sign(diff) / (3.0 * P) - l1 * l2 * g / (3.0 * P)
        g_rgb[3 * off:3 * (off + P)] = g.ravel()
        sl = slice(off, off + P)
        m = t_depth[sl] > 0
        cnt = m.sum()
        if cnt:
            dd = depth[sl] - t_depth[sl]
            loss += (1.0 - l1) * np.abs(dd[m]).sum() / cnt
            g_depth[sl] = np.where(m, (1.0 - l1) * np.sign(dd) / cnt, 0.0)
        off += P
    return loss, g_rgb, g_depth, np.zeros_like(depth), np.array(ssims)
