"""Brute-force renderer for tiny inputs: every Gaussian against every pixel.

An independent restatement of what the rasterizer computes (DROID-Splat
Sec. 3.3, eqn:rendering, alpha_i = sigma_i * G), with no tiles and no
sorting structure: each pixel's list is every kept Gaussian whose 3-sigma
pixel square contains it, ordered by (fp32 depth, index).  Library routines
stand in for the hand-written steps of the oracle: scipy's Rotation for the
quaternion, numpy.linalg.inv / eigvalsh for the conic and the extent, and
scipy's complex spherical harmonics (converted to the real basis) for colour.
Used to pin the oracle on inputs of at most a few hundred Gaussians.
"""
import math

import numpy as np
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

A_MIN = float(np.float32(1.0 / 255.0))
A_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))


def real_sh(degree, dirs):
    """Real SH basis, order (l, m = -l..l), from scipy's complex harmonics
    (which carry the Condon-Shortley phase): m>0 -> sqrt2 Re Y_l^m,
    m<0 -> sqrt2 Im Y_l^|m|, m=0 -> Y_l^0.  dirs: [n,3] unit vectors."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                out.append(math.sqrt(2.0) * Y.real)
            elif m < 0:
                out.append(math.sqrt(2.0) * Y.imag)
            else:
                out.append(Y.real)
    return np.stack(out, 1)


def project(scene, f):
    """Per-Gaussian screen-space quantities for frame f (FP64)."""
    c = scene.cams[f]
    W, H = int(c[0]), int(c[1])
    fx, fy, cx, cy, near = [float(np.float32(v)) for v in c[2:7]]  # the FP32 the ABI takes
    P = scene.poses[f].astype(np.float64)
    Rw, tw = P[:, :3], P[:, 3]
    mu = scene.means.astype(np.float64)
    q = scene.quats.astype(np.float64)
    Rg = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    s2 = np.exp(2.0 * scene.log_scales.astype(np.float64))
    Sigma = np.einsum("nij,nj,nkj->nik", Rg, s2, Rg)
    t = mu @ Rw.T + tw
    tz = t[:, 2]
    with np.errstate(all="ignore"):
        u = fx * t[:, 0] / tz + cx
        v = fy * t[:, 1] / tz + cy
        limx, limy = 1.3 * W / (2 * fx), 1.3 * H / (2 * fy)
        txc = tz * np.clip(t[:, 0] / tz, -limx, limx)
        tyc = tz * np.clip(t[:, 1] / tz, -limy, limy)
        J = np.zeros((len(mu), 2, 3))
        J[:, 0, 0] = fx / tz
        J[:, 0, 2] = -fx * txc / tz ** 2
        J[:, 1, 1] = fy / tz
        J[:, 1, 2] = -fy * tyc / tz ** 2
        Sc = Rw @ Sigma @ Rw.T
        S2 = J @ Sc @ np.transpose(J, (0, 2, 1)) + 0.3 * np.eye(2)
    keep = tz > near
    det = np.linalg.det(S2)
    keep &= det > 0
    conic = np.zeros_like(S2)
    lmax = np.zeros(len(mu))
    conic[keep] = np.linalg.inv(S2[keep])
    lmax[keep] = np.linalg.eigvalsh(S2[keep])[:, -1]
    r = 3.0 * np.sqrt(lmax)
    with np.errstate(all="ignore"):
        xa, xb = np.ceil(u - r), np.floor(u + r)
        ya, yb = np.ceil(v - r), np.floor(v + r)
    keep &= (xa <= W - 1) & (xb >= 0) & (xa <= xb) & (ya <= H - 1) & (yb >= 0) & (ya <= yb)
    x_lo = np.where(keep, np.maximum(xa, 0), 0).astype(np.int64)
    x_hi = np.where(keep, np.minimum(xb, W - 1), -1).astype(np.int64)
    y_lo = np.where(keep, np.maximum(ya, 0), 0).astype(np.int64)
    y_hi = np.where(keep, np.minimum(yb, H - 1), -1).astype(np.int64)
    Cc = -Rw.T @ tw
    d = mu - Cc
    dirs = d / np.linalg.norm(d, axis=1, keepdims=True)
    Y = real_sh(scene.sh_degree, dirs)
    raw = np.einsum("nk,nkc->nc", Y, scene.sh.astype(np.float64)) + 0.5
    col = np.maximum(raw, 0.0)
    opac = 1.0 / (1.0 + np.exp(-scene.opacity.astype(np.float64)))
    depth_bits = tz.astype(np.float32).view(np.uint32)
    return dict(keep=keep, u=u, v=v, z=tz, conic=conic, lmax=lmax, radius=r, x_lo=x_lo,
                x_hi=x_hi, y_lo=y_lo, y_hi=y_hi, color=col, raw=raw, opacity=opac,
                depth_bits=depth_bits, cov=S2)


def visible(scene, f, p=None):
    """Per Gaussian: does alpha reach 1/255 at some pixel of its square?"""
    p = p if p is not None else project(scene, f)
    out = np.zeros(len(p["keep"]), bool)
    for g in np.nonzero(p["keep"])[0]:
        xs = np.arange(p["x_lo"][g], p["x_hi"][g] + 1)
        ys = np.arange(p["y_lo"][g], p["y_hi"][g] + 1)
        dx = p["u"][g] - xs[None, :]
        dy = p["v"][g] - ys[:, None]
        Q = p["conic"][g]
        q = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
        a = np.minimum(A_MAX, p["opacity"][g] * np.exp(-0.5 * q))
        out[g] = bool((a >= A_MIN).any())
    return out


def render(scene):
    """Per frame (rgb [3,H,W], depth [H,W], alpha [H,W]) by brute force."""
    out = []
    bg = np.asarray(scene.background, np.float32).astype(np.float64)
    for f in range(len(scene.cams)):
        W, H = int(scene.cams[f][0]), int(scene.cams[f][1])
        p = project(scene, f)
        idx = np.nonzero(p["keep"])[0]
        order = idx[np.lexsort((idx, p["depth_bits"][idx]))]
        rgb = np.zeros((3, H, W))
        dep = np.zeros((H, W))
        alp = np.zeros((H, W))
        for j in range(H):
            for i in range(W):
                inside = order[(p["x_lo"][order] <= i) & (i <= p["x_hi"][order]) &
                               (p["y_lo"][order] <= j) & (j <= p["y_hi"][order])]
                T = 1.0
                acc = np.zeros(3)
                accz = 0.0
                for g in inside:
                    dx, dy = p["u"][g] - i, p["v"][g] - j
                    Q = p["conic"][g]
                    q = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
                    a = min(A_MAX, p["opacity"][g] * math.exp(-0.5 * q))
                    if a < A_MIN:
                        continue
                    Tn = T * (1 - a)
                    if Tn < T_MIN:
                        break
                    acc += p["color"][g] * a * T
                    accz += p["z"][g] * a * T
                    T = Tn
                rgb[:, j, i] = acc + T * bg
                dep[j, i] = accz
                alp[j, i] = 1 - T
        out.append((rgb, dep, alp))
    return out


def render_median(scene):
    """Per frame the median depth [H,W] by brute force: walking each pixel's
    entries front to back, the depth of the first blended entry after which
    the transmittance is below 1/2 (0 if it never is)."""
    out = []
    for f in range(len(scene.cams)):
        W, H = int(scene.cams[f][0]), int(scene.cams[f][1])
        p = project(scene, f)
        idx = np.nonzero(p["keep"])[0]
        order = idx[np.lexsort((idx, p["depth_bits"][idx]))]
        med = np.zeros((H, W))
        for j in range(H):
            for i in range(W):
                inside = order[(p["x_lo"][order] <= i) & (i <= p["x_hi"][order]) &
                               (p["y_lo"][order] <= j) & (j <= p["y_hi"][order])]
                T = 1.0
                for g in inside:
                    dx, dy = p["u"][g] - i, p["v"][g] - j
                    Q = p["conic"][g]
                    q = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
                    a = min(A_MAX, p["opacity"][g] * math.exp(-0.5 * q))
                    if a < A_MIN:
                        continue
                    if T * (1 - a) < T_MIN:
                        break
                    T = T * (1 - a)
                    if T < 0.5:
                        med[j, i] = p["z"][g]
                        break
        out.append(med)
    return out
