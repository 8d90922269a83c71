"""L1 terms of the rendering loss, plain FP64 numpy (test infrastructure).

DROID-Splat's rendering objective (eqn rnd_loss, Sec. 3.3; weights in
supplementary S1.2) is lambda1 [(1 - lambda2) |I' - I*| + lambda2 (1 - SSIM)]
+ (1 - lambda1) |Z' - Z*|.  The hot path implements its L1 terms, read as
per-frame means, with the depth term restricted to pixels with a valid
target depth (Z* > 0):
    L = sum_f [ mean_{c,p} |RGB - RGB*| + w_d * mean_{p: Z*>0} |D - Z*| ],
with sign(0) = 0 in the gradient and no gradient to alpha.
"""
import numpy as np


def loss_l1(rgb, depth, t_rgb, t_depth, depth_weight, sizes):
    """rgb/t_rgb packed [3,H,W] per frame, depth/t_depth [H,W] per frame;
    sizes = [(W, H)].  Returns (loss, g_rgb, g_depth, g_alpha) in FP64."""
    rgb = np.asarray(rgb, np.float64)
    depth = np.asarray(depth, np.float64)
    t_rgb = np.asarray(t_rgb, np.float64)
    t_depth = np.asarray(t_depth, np.float64)
    g_rgb = np.zeros_like(rgb)
    g_depth = np.zeros_like(depth)
    loss = 0.0
    off = 0
    for (w, h) in sizes:
        P = w * h
        sl3 = slice(3 * off, 3 * (off + P))
        sl = slice(off, off + P)
        diff = rgb[sl3] - t_rgb[sl3]
        loss += np.abs(diff).sum() / (3.0 * P)
        g_rgb[sl3] = np.sign(diff) / (3.0 * P)
        m = t_depth[sl] > 0
        cnt = m.sum()
        if cnt:
            dd = depth[sl] - t_depth[sl]
            loss += depth_weight * np.abs(dd[m]).sum() / cnt
            g_depth[sl] = np.where(m, depth_weight * np.sign(dd) / cnt, 0.0)
        off += P
    return loss, g_rgb, g_depth, np.zeros_like(depth)
