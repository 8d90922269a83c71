"""2D Gaussian surfel (2DGS) renderer, plain PyTorch FP64 on the CPU (test
infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use
this module; it shares no code with the HIP path.  Gradients are PyTorch's
autograd of this forward.

DROID-Splat compares its 3D Gaussians with 2D surfel Gaussians (Sec. 3.3,
tab:renderer; the 2DGS method it cites): flat disks that are intersected with
each pixel's ray instead of being projected as 2D Gaussians.  Per surfel:
mean mu, two log-scales (s_u, s_v), rotation q (w, x, y, z) whose first two
axes t_u, t_v span the disk and whose third is its normal, opacity logit and
SH colour (as for the 3D Gaussians).  Per frame, with the world->camera pose
[R_f | t_f] and K = [[fx, 0, cx], [0, fy, cy], [0, 0, 1]]:
    M = K [s_u R_f t_u | s_v R_f t_v | R_f mu + t_f]        (3 x 3, rows M0..M2)
maps disk coordinates (u, v, 1) to homogeneous pixels.  The ray through
pixel (x, y) meets the disk at (u, v) = (p0 / p2, p1 / p2), p = h_u x h_v,
h_u = x M2 - M0, h_v = y M2 - M1, at depth z = M2 . (u, v, 1).  Readings
where the paper is silent:
  - G = exp(-(u^2 + v^2) / 2); the screen-space low-pass of 2DGS,
    G_lp = exp(-|(x, y) - c|^2) (standard deviation sqrt(2)/2 px around the
    projected centre c), and G' = max(G, G_lp); a pixel where G_lp wins
    sees the surfel at its centre's depth;
  - alpha = min(0.99, sigma G'), skip alpha < 1/255, stop before T < 1e-4,
    front to back in order of (fp32(centre depth) bits, index), as for the
    3D Gaussians;
  - a surfel contributes only inside its pixel box: the bounding box of the
    image of the disk |(u, v)| <= r_a (r_a = sqrt(2 ln(255 sigma)), outside
    which G < 1/(255 sigma)), from the dual conic M diag(r_a^2, r_a^2, -1)
    M^T, united with the square of half width sqrt(ln(255 sigma)) around c
    (where G_lp can reach it), as [ceil(lo), floor(hi)] clipped to the
    image; culled if sigma <= 1/255, if the centre or the disk's nearest
    point (depth z_c - r_a |(M2_0, M2_1)|) is not in front of the near
    plane, or if the box is empty;
  - outputs: RGB (+ T_final * background), depth sum_i w_i z_i, alpha
    1 - T_final and normal sum_i w_i n_i with n_i = R_f t_w turned to face
    the camera (n . (R_f mu + t_f) < 0), in camera coordinates;
  - the depth distortion of 2DGS (the L_dist term that the supplementary's
    Rendering settings, 2D Gaussian Splatting paragraph, adds to the
    objective for surfels), per pixel the sum over pairs i < j of
    blended entries of w_i w_j (z_i - z_j)^2, with z the depth above
    (squared distance in camera depth units).  Written here as the pair sum
    expanded over the entries in front: entry j adds
    w_j sum_{i<j} w_i (z_j - z_i)^2 = w_j (A z_j^2 - 2 z_j D_1 + D_2) with
    A, D_1, D_2 the sums of w_i, w_i z_i, w_i z_i^2 over i < j;
  - the normal consistency of 2DGS (its L_normal, the other term that
    paragraph adds) is an image-space function of the depth, alpha and
    normal maps: normal_consistency below.
"""
import math

import numpy as np
import torch

A_MIN = float(np.float32(1.0 / 255.0))
A_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))
BAND = 1e-4
EPS32 = 2.0 ** -24

FLAG_ALPHA, FLAG_T, FLAG_CLAMP, FLAG_LOWPASS = 1, 2, 4, 16
# The ray-disk intersection loses accuracy with its conditioning
# kappa = |h_u| |h_v| / |h_u x h_v| (1 / sin of the angle between the two
# planes through the ray): G computed in FP32 from the stored surfel errs by
# up to ~5 kappa (1 + q) ulps relative (measured on FP32 evaluations of
# tilted surfels), and a tilted surfel's rotation gradient sums per-pixel
# terms that cancel to ~1 % of their size.  FLAG_COND marks the pixels where
# the disk term is blended with kappa (1 + q) above KAPPA_GRAD (so ~1e-5 of a
# term, ~1e-3 after such cancellation); they carry no decision, so image
# comparisons keep them and gradient comparisons do not.
FLAG_COND = 32
KAPPA_GRAD = 32.0


def _rot(q):
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)],
        -2)


def _skew(v):
    z = torch.zeros_like(v[0])
    return torch.stack([torch.stack([z, -v[2], v[1]]), torch.stack([v[2], z, -v[0]]),
                        torch.stack([-v[1], v[0], z])])


def _sh_colour(sh, deg, dirs):
    """max(0, sum_k sh_k Y_k(dir) + 1/2) with the real SH basis of the 3D
    Gaussians (textbook magnitudes, sign (-1)^|m|)."""
    pi = math.pi
    x, y, z = dirs.unbind(-1)
    Y = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    if deg >= 1:
        k = math.sqrt(3.0 / (4.0 * pi))
        Y += [-k * y, k * z, -k * x]
    if deg >= 2:
        a, b, c = 0.5 * math.sqrt(15.0 / pi), 0.25 * math.sqrt(5.0 / pi), 0.25 * math.sqrt(15.0 / pi)
        Y += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z,
              c * (x * x - y * y)]
    if deg >= 3:
        a = 0.25 * math.sqrt(35.0 / (2 * pi))
        b = 0.5 * math.sqrt(105.0 / pi)
        c = 0.25 * math.sqrt(21.0 / (2 * pi))
        d = 0.25 * math.sqrt(7.0 / pi)
        e = 0.25 * math.sqrt(105.0 / pi)
        Y += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
              d * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
              e * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    Yt = torch.stack(Y, -1)                       # [n, K]
    raw = torch.einsum("nk,nkc->nc", Yt, sh) + 0.5
    return torch.clamp(raw, min=0.0)


def render(means, log_scales, quats, opacity_logits, sh, sh_degree, cams, poses,
           background=(0.0, 0.0, 0.0), twist=None, window=None, jitter=None):
    """FP64 torch tensors in (means [n,3], log_scales [n,2], quats [n,4],
    opacity_logits [n], sh [n,K,3], poses [F,3,4]; twist [F,6] = (rho, phi)
    left perturbation, first order at 0).  Returns a list per frame of dicts
    rgb [3,H,W], depth, alpha, dist [H,W], normal [3,H,W], flags [H,W]
    (uint8, numpy), box (numpy int [n,4] x_lo, x_hi, y_lo, y_hi, -1 if
    culled), order and pairs (the (pixel, surfel) pairs whose box holds the
    pixel before it stops).  window = (x0, x1, y0, y1), inclusive, renders
    only those pixels of every frame (the images are then of the window's
    size; each pixel's value is the same as in the whole image).

    jitter (a torch.Generator, for tests): scales each surfel's M2,
    k_u = c_x M2 - M0 and k_v = c_y M2 - M1 (per component) by
    (1 + 2^-24 xi), xi ~ N(0, 1) drawn from it, and evaluates each pixel's
    intersection (h_u, h_v from the offset to the centre, their cross
    product, u, v, q, G, G_lp and the depth) as a kernel does in FP32, each operation
    followed by such a factor; the factors are constants of the autograd
    graph.  The change this makes to the gradients is the size of change
    the FP32 rounding of the stored surfel and of the intersection causes,
    ill-conditioning and cancellation included; None renders exactly."""
    out = []
    bg = torch.tensor([float(b) for b in background], dtype=torch.float64)
    # a surfel with a non-finite parameter is culled in every frame; its
    # values are replaced by harmless ones behind a mask, so that its
    # gradients are exactly 0 instead of 0 * NaN
    K3 = (sh_degree + 1) ** 2
    finite = (torch.isfinite(means).all(1) & torch.isfinite(log_scales).all(1)
              & torch.isfinite(quats).all(1) & torch.isfinite(opacity_logits)
              & torch.isfinite(sh[:, :K3].reshape(sh.shape[0], -1)).all(1))
    if not bool(finite.all()):
        fm = finite[:, None]
        means = torch.where(fm, means, torch.zeros_like(means))
        log_scales = torch.where(fm, log_scales, torch.zeros_like(log_scales))
        quats = torch.where(fm, quats, torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=quats.dtype))
        opacity_logits = torch.where(finite, opacity_logits, torch.zeros_like(opacity_logits))
        sh = torch.where(finite[:, None, None], sh, torch.zeros_like(sh))
    finite_np = finite.numpy()
    Rg = _rot(quats)                                # [n,3,3]
    su, sv = torch.exp(log_scales[:, 0]), torch.exp(log_scales[:, 1])
    opac = torch.sigmoid(opacity_logits)
    for f, cam in enumerate(cams):
        W, H, fx, fy, cx, cy, near = [float(v) for v in cam[:7]]
        W, H = int(W), int(H)
        Rf, tf = poses[f, :, :3], poses[f, :, 3]
        if twist is not None:
            Kx = _skew(twist[f, 3:])
            Rf = Rf + Kx @ Rf
            tf = tf + Kx @ tf + twist[f, :3]
        K = torch.tensor([[fx, 0.0, cx], [0.0, fy, cy], [0.0, 0.0, 1.0]], dtype=torch.float64)
        tu = torch.einsum("ij,njk->nik", Rf, Rg)[:, :, 0]
        tv = torch.einsum("ij,njk->nik", Rf, Rg)[:, :, 1]
        tw = torch.einsum("ij,njk->nik", Rf, Rg)[:, :, 2]
        mc = means @ Rf.T + tf
        M = torch.stack([(su[:, None] * tu) @ K.T, (sv[:, None] * tv) @ K.T, mc @ K.T], -1)
        # M[n] columns: a, b, c  -> rows M0, M1, M2
        ctr = torch.stack([M[:, 0, 2] / M[:, 2, 2], M[:, 1, 2] / M[:, 2, 2]], -1)
        nrm = torch.where(((tw * mc).sum(-1) < 0)[:, None], tw, -tw)
        # colour: direction from the camera centre to the mean
        Cw = -(Rf.T @ tf)
        d = means - Cw
        dirs = d / torch.linalg.norm(d, dim=-1, keepdim=True)
        col = _sh_colour(sh, sh_degree, dirs)
        n = means.shape[0]
        box = -np.ones((n, 4), np.int64)
        with torch.no_grad():
            Mn, opn = M.detach().numpy(), opac.detach().numpy()
            mcn, ctrn = mc.detach().numpy(), ctr.detach().numpy()
            for g in range(n):
                o = float(opn[g])
                zc = float(mcn[g, 2])
                if not finite_np[g] or not (o > A_MIN) or not (zc > near):
                    continue
                r2 = 2.0 * math.log(o / A_MIN)          # r_a^2
                ra = math.sqrt(r2)
                rl = math.sqrt(math.log(o / A_MIN))
                m = Mn[g].tolist()
                # the disk's nearest point to the camera plane
                if not (m[2][2] - ra * math.sqrt(m[2][0] * m[2][0] + m[2][1] * m[2][1]) > near):
                    continue
                # bounding box of the image of the circle |(u, v)| = r_a: its dual
                # conic is C* = M diag(r_a^2, r_a^2, -1) M^T, and the vertical
                # tangents x = x0 solve C*_00 - 2 x0 C*_02 + x0^2 C*_22 = 0
                def dual(i, j):
                    return r2 * (m[i][0] * m[j][0] + m[i][1] * m[j][1]) - m[i][2] * m[j][2]
                c22 = dual(2, 2)
                ext = []
                for i in (0, 1):
                    ci2, cii = dual(i, 2), dual(i, i)
                    sq = math.sqrt(max(ci2 * ci2 - cii * c22, 0.0))
                    ext.append(((ci2 + sq) / c22, (ci2 - sq) / c22))
                c0 = ctrn[g]
                lo = [min(ext[i][0], ext[i][1], c0[i] - rl) for i in (0, 1)]
                hi = [max(ext[i][0], ext[i][1], c0[i] + rl) for i in (0, 1)]
                x_lo, x_hi = max(0, math.ceil(lo[0])), min(W - 1, math.floor(hi[0]))
                y_lo, y_hi = max(0, math.ceil(lo[1])), min(H - 1, math.floor(hi[1]))
                if x_lo <= x_hi and y_lo <= y_hi:
                    box[g] = (x_lo, x_hi, y_lo, y_hi)
            keep = np.nonzero(box[:, 0] >= 0)[0]
            zbits = mc[:, 2].detach().numpy().astype(np.float32).view(np.uint32)
            order = keep[np.lexsort((keep, zbits[keep]))]
        wx0, wx1, wy0, wy1 = (0, W - 1, 0, H - 1) if window is None else window
        ys, xs = torch.meshgrid(torch.arange(wy0, wy1 + 1, dtype=torch.float64),
                                torch.arange(wx0, wx1 + 1, dtype=torch.float64), indexing="ij")
        Hw, Ww = xs.shape
        T = torch.ones(Hw, Ww, dtype=torch.float64)
        C = torch.zeros(3, Hw, Ww, dtype=torch.float64)
        D = torch.zeros(Hw, Ww, dtype=torch.float64)
        N = torch.zeros(3, Hw, Ww, dtype=torch.float64)
        Dist = torch.zeros(Hw, Ww, dtype=torch.float64)
        SA = torch.zeros(Hw, Ww, dtype=torch.float64)   # sum of w over entries in front
        SZ = torch.zeros(Hw, Ww, dtype=torch.float64)   # ... of w z
        SZZ = torch.zeros(Hw, Ww, dtype=torch.float64)  # ... of w z^2
        done = torch.zeros(Hw, Ww, dtype=torch.bool)
        flags = np.zeros((Hw, Ww), np.uint8)
        nb = torch.zeros(Hw, Ww, dtype=torch.float64)
        pairs = 0
        for g in order:
            x_lo, x_hi, y_lo, y_hi = box[g]
            if x_hi < wx0 or x_lo > wx1 or y_hi < wy0 or y_lo > wy1:
                continue
            inside = (xs >= x_lo) & (xs <= x_hi) & (ys >= y_lo) & (ys <= y_hi) & ~done
            pairs += int(inside.sum())
            if not bool(inside.any()):
                continue
            M0, M1, M2 = M[g, 0], M[g, 1], M[g, 2]
            if jitter is not None:
                # the surfel's stored values M2, k_u = c_x M2 - M0 and
                # k_v = c_y M2 - M1, each off by one rounding, shared by all
                # its pixels
                ku, kv = ctr[g, 0] * M2 - M0, ctr[g, 1] * M2 - M1
                e = [1.0 + EPS32 * torch.randn(3, generator=jitter, dtype=torch.float64)
                     for _ in range(3)]
                M2, ku, kv = M2 * e[0], ku * e[1], kv * e[2]
                M0, M1 = ctr[g, 0] * M2 - ku, ctr[g, 1] * M2 - kv
            if jitter is None:
                hu = xs[..., None] * M2 - M0
                hv = ys[..., None] * M2 - M1
                p = torch.linalg.cross(hu, hv, dim=-1)
                ok = p[..., 2].abs() > 1e-300
                p2 = torch.where(ok, p[..., 2], torch.ones_like(p[..., 2]))
                u, v = p[..., 0] / p2, p[..., 1] / p2
                q = torch.where(ok, u * u + v * v, torch.full_like(u, float("inf")))
                G = torch.exp(-0.5 * q)
                dd = (xs - ctr[g, 0]) ** 2 + (ys - ctr[g, 1]) ** 2
                Glp = torch.exp(-dd)
            else:
                # the same steps as a kernel takes them in FP32 from the
                # pixel's offset to the centre, each operation followed by
                # one rounding (a random relative error of one ulp)
                def rd(t):
                    return t * (1.0 + EPS32 * torch.randn(t.shape, generator=jitter,
                                                          dtype=torch.float64))
                ex, ey = rd(xs - ctr[g, 0]), rd(ys - ctr[g, 1])
                hu = torch.stack([rd(rd(ex * M2[0]) + ku[0]), rd(rd(ex * M2[1]) + ku[1]),
                                  rd(ex * M2[2])], -1)
                hv = torch.stack([rd(rd(ey * M2[0]) + kv[0]), rd(rd(ey * M2[1]) + kv[1]),
                                  rd(ey * M2[2])], -1)
                p = torch.stack([
                    rd(rd(hu[..., 1] * hv[..., 2]) - rd(hu[..., 2] * hv[..., 1])),
                    rd(rd(hu[..., 2] * hv[..., 0]) - rd(hu[..., 0] * hv[..., 2])),
                    rd(rd(hu[..., 0] * hv[..., 1]) - rd(hu[..., 1] * hv[..., 0]))], -1)
                ok = p[..., 2].abs() > 1e-300
                ip = rd(1.0 / torch.where(ok, p[..., 2], torch.ones_like(p[..., 2])))
                u, v = rd(p[..., 0] * ip), rd(p[..., 1] * ip)
                q = torch.where(ok, rd(rd(u * u) + rd(v * v)), torch.full_like(u, float("inf")))
                G = rd(torch.exp(-0.5 * q))
                dd = rd(rd(ex * ex) + rd(ey * ey))
                Glp = rd(torch.exp(-dd))
            # conditioning of the intersection: 1 / sin of the angle of h_u, h_v
            kappa = (torch.linalg.norm(hu, dim=-1) * torch.linalg.norm(hv, dim=-1)
                     / torch.linalg.norm(p, dim=-1).clamp(min=1e-300)).detach()
            use_obj = G >= Glp
            Gh = torch.where(use_obj, G, Glp)
            zobj = M2[0] * u + M2[1] * v + M2[2]
            if jitter is not None:
                zobj = rd(rd(rd(M2[0] * u) + rd(M2[1] * v)) + M2[2])
            zint = torch.where(use_obj, zobj, mc[g, 2].expand_as(u))
            araw = opac[g] * Gh
            a = torch.clamp(araw, max=A_MAX)
            with torch.no_grad():
                an, Tn_ = a.detach().numpy(), (T * (1 - a)).detach().numpy()
                ins = inside.numpy()
                Gn, Gl = G.detach().numpy(), Glp.detach().numpy()
                # alpha's FP32 error is that of the term that sets it: the
                # disk term's exponent errs by ~(1 + q) kappa ulps, the
                # low-pass's by ~(1 + |x - c|^2); near their switch either may
                # set it.  An exponent off by e moves ln(alpha) by e, so the
                # decision alpha >= A_MIN is in doubt where |ln(alpha / A_MIN)|
                # is below the band (for small bands the same as a relative
                # band on alpha; a pixel that alpha cannot reach is not)
                band_obj = np.maximum(BAND, 64 * EPS32 * (1 + np.minimum(q.detach().numpy(), 1e30))
                                      * np.minimum(kappa.numpy(), 1e30))
                band_lp = np.maximum(BAND, 64 * EPS32 * (1 + dd.detach().numpy()))
                # which term is larger is in doubt where their exponents q/2
                # and |x - c|^2 differ by less than 1e-3 or than the terms'
                # own FP32 error (an ill-conditioned disk term can overtake
                # the low-pass)
                qn = np.minimum(q.detach().numpy(), 1e300)
                switch = (np.abs(0.5 * qn - dd.detach().numpy())
                          < np.maximum(1e-3, band_obj + band_lp))
                band_a = np.where(switch, np.maximum(np.maximum(band_obj, band_lp), 1e-3),
                                  np.where(use_obj.numpy(), band_obj, band_lp))
                lna = np.abs(np.log(np.maximum(an, 1e-300) / A_MIN))
                flags[ins & (lna < band_a)] |= FLAG_ALPHA
                live = ins & (an >= A_MIN)
                band_t = np.maximum(BAND, 4 * EPS32 * (nb.numpy() + 1))
                flags[live & (np.abs(Tn_ - T_MIN) < band_t * T_MIN)] |= FLAG_T
                flags[live & (np.abs(araw.detach().numpy() - A_MAX) < BAND * A_MAX)] |= FLAG_CLAMP
                flags[live & switch] |= FLAG_LOWPASS
                flags[live & use_obj.numpy() &
                      ((1 + qn) * np.minimum(kappa.numpy(), 1e300) > KAPPA_GRAD)] |= FLAG_COND
            blend = inside & (a >= A_MIN)
            Tn = T * (1 - a)
            stop = blend & (Tn < T_MIN)
            done = done | stop
            blend = blend & ~stop
            w = torch.where(blend, a * T, torch.zeros_like(T))
            C = C + col[g][:, None, None] * w
            D = D + zint * w
            N = N + nrm[g][:, None, None] * w
            Dist = Dist + w * (SA * zint * zint - 2.0 * zint * SZ + SZZ)
            SA = SA + w
            SZ = SZ + w * zint
            SZZ = SZZ + w * zint * zint
            T = torch.where(blend, Tn, T)
            nb = nb + blend.to(torch.float64)
        rgb = C + T * bg[:, None, None]
        out.append(dict(rgb=rgb, depth=D, alpha=1 - T, normal=N, dist=Dist, flags=flags,
                        box=box, order=order, pairs=pairs))
    return out


def to64(a, grad=False):
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64)))
    return t.requires_grad_(grad)


def depth_normals(depth, cam):
    """Normals of the surface the depth map describes (2DGS's normal from
    depth): each pixel back-projects to P = D(x, y) K^-1 (x, y, 1); with the
    central differences dP_x = P(x+1, y) - P(x-1, y) and dP_y = P(x, y+1) -
    P(x, y-1), N = (dP_y x dP_x) / |dP_y x dP_x|, which faces the camera for
    a surface in front of it.  Defined on interior pixels (1 <= x <= W-2,
    1 <= y <= H-2) where the cross product is non-zero; 0 elsewhere.
    Returns (N [3,H,W], valid [H,W] bool)."""
    W, H, fx, fy, cx, cy = [float(v) for v in cam[:6]]
    W, H = int(W), int(H)
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64),
                            torch.arange(W, dtype=torch.float64), indexing="ij")
    P = torch.stack([depth * (xs - cx) / fx, depth * (ys - cy) / fy, depth])   # [3,H,W]
    dPx = torch.zeros_like(P)
    dPy = torch.zeros_like(P)
    dPx[:, 1:-1, 1:-1] = P[:, 1:-1, 2:] - P[:, 1:-1, :-2]
    dPy[:, 1:-1, 1:-1] = P[:, 2:, 1:-1] - P[:, :-2, 1:-1]
    v = torch.linalg.cross(dPy, dPx, dim=0)
    nv = torch.linalg.norm(v, dim=0)
    valid = torch.zeros(H, W, dtype=torch.bool)
    valid[1:-1, 1:-1] = True
    valid = valid & (nv.detach() > 0)
    N = torch.where(valid, v / torch.where(valid, nv, torch.ones_like(nv)), torch.zeros_like(v))
    return N, valid


def normal_consistency(depth, alpha, normal, cam):
    """The normal-consistency term of the surfel objective (2DGS's L_normal,
    added for surfels in the supplementary's Rendering settings), per frame:
    the mean over the interior pixels of sum_i w_i (1 - n_i . N), N the
    normal from the depth map (depth_normals).  As sum_i w_i = alpha and
    sum_i w_i n_i is the normal map, a pixel's term is alpha - normal . N.
    Pixels where N is not defined add 0; the mean divides by the interior
    pixel count (W-2)(H-2).  Returns (loss, per-pixel map [H,W])."""
    N, valid = depth_normals(depth, cam)
    term = torch.where(valid, alpha - (normal * N).sum(0), torch.zeros_like(alpha))
    W, H = int(cam[0]), int(cam[1])
    return term.sum() / float((W - 2) * (H - 2)), term
