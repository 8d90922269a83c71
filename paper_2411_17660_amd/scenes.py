"""Seeded synthetic scenes shaped like the mapper's workloads.

This module is the only code shared by the oracle tests and the HIP path.  It
draws inputs and holds none of the renderer's arithmetic (no projection of
Gaussians, no compositing): pinhole back-projection of a synthetic depth map
is used only to place means on surfaces, the way the paper initialises its
Gaussians from the tracker's dense depth (Sec. 3.3; supplementary S1.2).

All draws use numpy's PCG64 (``default_rng(seed)``) in FP64 and are cast once
to FP32, so every consumer sees identical FP32 values.

Workloads (sizes from the paper's resolutions, Gaussian counts and batch of
keyframes per mapping iteration; supplementary S1, Tab. tab:supp_full_render):
  c1  2,000 Gaussians, one 128x96 camera, SH degree 0
  c2  100k Gaussians, one 640x480 camera, piecewise-planar depth-map scene, SH3
  c3  500k Gaussians, 8 keyframes at 1200x680 on a smooth trajectory, SH3
  c4  1M Gaussians, 16 keyframes of mixed resolution, Student-t log-scales
  c5  3M Gaussians, 12 keyframes at 1920x1080
"""
from dataclasses import dataclass, field
import math

import numpy as np

NEAR = 0.2


@dataclass
class Scene:
    means: np.ndarray        # [N,3] f32
    log_scales: np.ndarray   # [N,3] f32
    quats: np.ndarray        # [N,4] f32, (w, x, y, z)
    opacity: np.ndarray      # [N]   f32, logits
    sh: np.ndarray           # [N,(d+1)^2,3] f32
    sh_degree: int
    cams: list               # [(W, H, fx, fy, cx, cy, near)] per frame
    poses: np.ndarray        # [F,3,4] f32, world -> camera
    background: tuple = (0.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.means.shape[0])

    @property
    def n_frames(self):
        return len(self.cams)

    @property
    def n_pixels(self):
        return int(sum(c[0] * c[1] for c in self.cams))

    def frame_pixels(self):
        return [int(c[0] * c[1]) for c in self.cams]

    def subset_frames(self, idx):
        """Same Gaussians, a subset of the frames."""
        idx = list(idx)
        return Scene(self.means, self.log_scales, self.quats, self.opacity, self.sh,
                     self.sh_degree, [self.cams[i] for i in idx],
                     np.ascontiguousarray(self.poses[idx]), self.background, dict(self.extra))

    def with_means(self, means):
        return Scene(np.ascontiguousarray(means, np.float32), self.log_scales, self.quats,
                     self.opacity, self.sh, self.sh_degree, self.cams, self.poses,
                     self.background, dict(self.extra))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _unit_quats(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _axis_angle(axis, ang):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)


def _perturb_dir(rng, d, max_deg):
    """Random walk step of a unit vector: turn by <= max_deg about a random
    axis perpendicular to it."""
    a = rng.normal(size=3)
    a -= a.dot(d) * d
    a /= np.linalg.norm(a)
    ang = math.radians(max_deg) * rng.uniform(0.0, 1.0)
    out = _axis_angle(a, ang) @ d
    return out / np.linalg.norm(out)


def trajectory(rng, n_frames, step_m=0.1, step_deg=5.0, heading_walk=10.0, axis_walk=20.0):
    """Camera-to-world rotations and centres along a smooth random trajectory:
    each step moves step_m along a heading that turns by <= heading_walk deg and
    rotates by step_deg about an axis that turns by <= axis_walk deg."""
    R = np.eye(3)
    Cc = np.zeros(3)
    heading = np.array([0.0, 0.0, 1.0])
    heading = _perturb_dir(rng, heading, 60.0)
    axis = _perturb_dir(rng, np.array([0.0, 1.0, 0.0]), 30.0)
    Rs, Cs = [R.copy()], [Cc.copy()]
    for _ in range(n_frames - 1):
        heading = _perturb_dir(rng, heading, heading_walk)
        axis = _perturb_dir(rng, axis, axis_walk)
        Cc = Cc + step_m * heading
        R = R @ _axis_angle(axis, math.radians(step_deg))
        Rs.append(R.copy())
        Cs.append(Cc.copy())
    return Rs, Cs


def w2c_poses(Rs, Cs):
    """World->camera [R^T | -R^T C] from camera->world (R, C)."""
    out = []
    for R, Cc in zip(Rs, Cs):
        Rw = R.T
        out.append(np.concatenate([Rw, (-Rw @ Cc)[:, None]], axis=1))
    return np.stack(out)


def planar_depth_samples(rng, W, H, n, cells=32, zmin=0.5, zmax=4.0, max_grad=2e-3):
    """n pixel positions (u, v) with depths from a piecewise-planar depth map
    of `cells` Voronoi cells with image-uniform seeds; cell k is the plane
    z = z_k + g_k . (u - su_k, v - sv_k), |g_k| <= max_grad m/px, clamped."""
    seeds = np.stack([rng.uniform(0, W, cells), rng.uniform(0, H, cells)], 1)
    z0 = rng.uniform(zmin, zmax, cells)
    ang = rng.uniform(0, 2 * math.pi, cells)
    mag = rng.uniform(0, max_grad, cells)
    grad = np.stack([mag * np.cos(ang), mag * np.sin(ang)], 1)
    u = rng.uniform(0, W, n)
    v = rng.uniform(0, H, n)
    z = np.empty(n)
    chunk = 1 << 18
    for s in range(0, n, chunk):
        uu, vv = u[s:s + chunk], v[s:s + chunk]
        d2 = (uu[:, None] - seeds[None, :, 0]) ** 2 + (vv[:, None] - seeds[None, :, 1]) ** 2
        k = np.argmin(d2, axis=1)
        zz = z0[k] + grad[k, 0] * (uu - seeds[k, 0]) + grad[k, 1] * (vv - seeds[k, 1])
        z[s:s + chunk] = np.clip(zz, zmin, zmax)
    return u, v, z


def backproject(u, v, z, fx, fy, cx, cy, R_c2w, C):
    """World points of pixels (u, v) at view depth z (placement of means only)."""
    pc = np.stack([(u - cx) * z / fx, (v - cy) * z / fy, z], 1)
    return pc @ np.asarray(R_c2w).T + np.asarray(C)[None, :]


def _appearance(rng, n, sh_degree, opacity_sigma=1.5):
    K = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.1, size=(n, K, 3))
    sh[:, 0, :] = rng.normal(0.5, 0.2, size=(n, 3))
    opac = rng.normal(0.0, opacity_sigma, size=n)
    return sh, opac


def _clip_anisotropy(ls, max_ratio=20.0):
    """Per Gaussian, pull the log-scales towards their mean so that
    max - min <= ln(max_ratio)."""
    lim = math.log(max_ratio)
    spread = ls.max(1) - ls.min(1)
    over = spread > lim
    if np.any(over):
        m = ls[over].mean(1, keepdims=True)
        ls[over] = m + (ls[over] - m) * (lim / spread[over])[:, None]
    return ls


def scene_c1(seed=0, n=2000):
    """2,000 Gaussians, 128x96 camera f=100, identity pose, SH0, black bg."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(1, 5, n)], 1)
    ls = rng.normal(-3.0, 0.5, size=(n, 3))
    q = _unit_quats(rng, n)
    opac = rng.normal(0.0, 1.0, size=n)
    sh = rng.normal(0.5, 0.2, size=(n, 1, 3))
    cams = [(128, 96, 100.0, 100.0, 64.0, 48.0, NEAR)]
    poses = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None]
    sc = Scene(_f32(means), _f32(ls), _f32(q), _f32(opac), _f32(sh), 0, cams, _f32(poses))
    sc.extra["rng_state"] = rng
    return sc


def upstream(rng_or_seed, scene):
    """N(0,1) upstream gradients (rgb [3P], depth [P], alpha [P]) packed like
    the outputs, drawn after the scene."""
    rng = rng_or_seed if isinstance(rng_or_seed, np.random.Generator) else \
        np.random.default_rng(rng_or_seed)
    P = scene.n_pixels
    g_rgb = rng.normal(size=3 * P)
    g_d = rng.normal(size=P)
    g_a = rng.normal(size=P)
    return _f32(g_rgb), _f32(g_d), _f32(g_a)


def scene_c2(seed=0, n=100_000, W=640, H=480, f=525.0):
    """One 640x480 keyframe, means on a noisy piecewise-planar depth map, SH3."""
    rng = np.random.default_rng(seed)
    cx, cy = W / 2.0, H / 2.0
    u, v, z = planar_depth_samples(rng, W, H, n)
    means = backproject(u, v, z, f, f, cx, cy, np.eye(3), np.zeros(3))
    means += rng.normal(0.0, 0.01, size=means.shape)
    ls = rng.normal(-4.0, 0.7, size=(n, 3))
    q = _unit_quats(rng, n)
    sh, opac = _appearance(rng, n, 3)
    cams = [(W, H, f, f, cx, cy, NEAR)]
    poses = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None]
    sc = Scene(_f32(means), _f32(ls), _f32(q), _f32(opac), _f32(sh), 3, cams, _f32(poses))
    sc.extra["rng_state"] = rng
    return sc


def _multi_frame(rng, n, cams, ls_sampler, Rs, Cs):
    F = len(cams)
    per = [n // F + (1 if i < n % F else 0) for i in range(F)]
    pts = []
    for i, (W, H, fx, fy, cx, cy, _) in enumerate(cams):
        u, v, z = planar_depth_samples(rng, W, H, per[i])
        pts.append(backproject(u, v, z, fx, fy, cx, cy, Rs[i], Cs[i]))
    means = np.concatenate(pts, 0)
    means += rng.normal(0.0, 0.01, size=means.shape)
    ls = _clip_anisotropy(ls_sampler(rng, n))
    q = _unit_quats(rng, n)
    sh, opac = _appearance(rng, n, 3)
    return means, ls, q, sh, opac


def scene_c3(seed=0, n=500_000, n_frames=8, W=1200, H=680, f=600.0, perturb=0.005):
    """8 keyframes at 1200x680 (f=600) on a smooth trajectory (0.1 m / 5 deg
    steps); 500k Gaussians, SH3, anisotropy <= 20:1.  `means` are the ground
    truth perturbed by N(0, perturb^2); extra['gt_means'] holds the truth."""
    rng = np.random.default_rng(seed)
    cams = [(W, H, f, f, W / 2.0, H / 2.0, NEAR)] * n_frames
    Rs, Cs = trajectory(rng, n_frames)
    means, ls, q, sh, opac = _multi_frame(
        rng, n, cams, lambda r, m: r.normal(-4.0, 0.7, size=(m, 3)), Rs, Cs)
    gt = _f32(means)
    meas = _f32(means + rng.normal(0.0, perturb, size=means.shape)) if perturb > 0 else gt
    sc = Scene(meas, _f32(ls), _f32(q), _f32(opac), _f32(sh), 3, cams, _f32(w2c_poses(Rs, Cs)))
    sc.extra["gt_means"] = gt
    sc.extra["rng_state"] = rng
    return sc


C4_SIZES = [(320, 240), (640, 480), (1200, 680), (1296, 968)]


def scene_c4(seed=0, n=1_000_000, n_frames=16):
    """16 keyframes, resolutions drawn from C4_SIZES, intrinsics f=(H+W)/2,
    c=(W/2,H/2) (the paper's calibration-free heuristic, supplementary S4);
    log-scales -4 + 0.6 t_3 truncated to [-12, 2]."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(C4_SIZES), n_frames)
    cams = []
    for i in idx:
        W, H = C4_SIZES[i]
        fv = (H + W) / 2.0
        cams.append((W, H, fv, fv, W / 2.0, H / 2.0, NEAR))
    Rs, Cs = trajectory(rng, n_frames)

    def ls_t(r, m):
        return np.clip(-4.0 + 0.6 * r.standard_t(3, size=(m, 3)), -12.0, 2.0)

    means, ls, q, sh, opac = _multi_frame(rng, n, cams, ls_t, Rs, Cs)
    gt = _f32(means)
    meas = _f32(means + rng.normal(0.0, 0.005, size=means.shape))
    sc = Scene(meas, _f32(ls), _f32(q), _f32(opac), _f32(sh), 3, cams, _f32(w2c_poses(Rs, Cs)))
    sc.extra["gt_means"] = gt
    sc.extra["rng_state"] = rng
    return sc


def scene_c5(seed=0, n=3_000_000, n_frames=12, W=1920, H=1080, f=1000.0):
    """12 keyframes at 1920x1080 (f=1000), 3M Gaussians, generator as c3."""
    return scene_c3(seed=seed, n=n, n_frames=n_frames, W=W, H=H, f=f)


def tiny_scene(seed=0, n=40, W=40, H=30, f=30.0, n_frames=1, sh_degree=3,
               ls_mean=-2.5, ls_sigma=0.4, zrange=(1.5, 4.0), spread=0.9, opacity_sigma=1.0,
               background=(0.1, 0.2, 0.3), outside=None):
    """Small scene for brute force, closed forms and finite differences: means
    in front of every camera of a short trajectory.

    Lateral positions are drawn in units of the half field of view (x/z in
    [-spread, spread] * W/(2f), likewise y).  With outside=(lo, hi), each
    Gaussian instead lies beyond the image on one or both axes (chosen at
    random): there |x/z| (|y/z|) is drawn from [lo, hi] of the half field of
    view with a random sign, and the other axis from [-spread, spread]."""
    rng = np.random.default_rng(seed)
    Rs, Cs = trajectory(rng, n_frames, step_m=0.05, step_deg=3.0)
    cams = [(W, H, f, f, W / 2.0 - 0.3, H / 2.0 + 0.2, NEAR)] * n_frames
    z = rng.uniform(zrange[0], zrange[1], n)
    ux = rng.uniform(-spread, spread, n)
    uy = rng.uniform(-spread, spread, n)
    if outside is not None:
        mode = rng.integers(0, 3, n)  # 0: x outside, 1: y outside, 2: both
        mag = rng.uniform(outside[0], outside[1], (n, 2))
        sgn = np.where(rng.uniform(size=(n, 2)) < 0.5, -1.0, 1.0)
        ux = np.where(mode != 1, sgn[:, 0] * mag[:, 0], ux)
        uy = np.where(mode != 0, sgn[:, 1] * mag[:, 1], uy)
    x = ux * z * (W / (2 * f))
    y = uy * z * (H / (2 * f))
    means = np.stack([x, y, z], 1) @ Rs[0].T + Cs[0][None, :]
    ls = rng.normal(ls_mean, ls_sigma, size=(n, 3))
    q = _unit_quats(rng, n)
    K = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.3, size=(n, K, 3))
    sh[:, 0, :] = rng.normal(0.5, 0.3, size=(n, 3))
    opac = rng.normal(0.5, opacity_sigma, size=n)
    sc = Scene(_f32(means), _f32(ls), _f32(q), _f32(opac), _f32(sh), sh_degree, cams,
               _f32(w2c_poses(Rs, Cs)), tuple(background))
    sc.extra["rng_state"] = rng
    return sc


def layout_scene(sizes, seed=0, n=8):
    """A few Gaussians in front of identity cameras of the given (W, H)
    sizes: a forward over it fixes the frame layout that the loss calls
    take from the last forward."""
    rng = np.random.default_rng(seed)
    cams = [(w, h, 0.8 * max(w, h), 0.8 * max(w, h), w / 2.0, h / 2.0, NEAR) for (w, h) in sizes]
    means = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n),
                      rng.uniform(2.0, 3.0, n)], 1)
    poses = np.repeat(np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None], len(sizes), 0)
    sh = rng.normal(0.5, 0.2, size=(n, 1, 3))
    return Scene(_f32(means), _f32(rng.normal(-2.5, 0.3, (n, 3))), _f32(_unit_quats(rng, n)),
                 _f32(rng.normal(0.0, 1.0, n)), _f32(sh), 0, cams, _f32(poses))


def loss_images(seed, sizes, depth_invalid=0.2):
    """Rendered and target images for the rendering-loss tests, packed like
    the renderer's outputs: (rgb [3P], depth [P], target_rgb, target_depth).

    Each target channel is a smooth field (a few low-frequency waves) with
    constant rectangles pasted in and light noise.  The rendered image equals
    the target exactly on one rectangle (flat and identical: the SSIM map's
    derivatives cancel most there), is the target plus small noise on the
    left half and independent values elsewhere.  A fraction of the target
    depths is 0 (no measurement)."""
    rng = np.random.default_rng(seed)
    rgb, dep, t_rgb, t_dep = [], [], [], []
    for (w, h) in sizes:
        yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
        tgt = np.empty((3, h, w))
        for c in range(3):
            f = np.full((h, w), rng.uniform(0.3, 0.7))
            for _ in range(3):
                kx, ky = rng.uniform(-0.15, 0.15, 2)
                f += rng.uniform(0.05, 0.2) * np.sin(kx * xx + ky * yy + rng.uniform(0, 6.3))
            for _ in range(2):
                x0, y0 = rng.integers(0, w), rng.integers(0, h)
                f[y0:y0 + rng.integers(1, 40), x0:x0 + rng.integers(1, 40)] = rng.uniform(0, 1)
            tgt[c] = f + rng.normal(0, 0.01, (h, w))
        img = rng.uniform(0, 1, (3, h, w))
        left = xx < w / 2
        img[:, left] = tgt[:, left] + rng.normal(0, 0.02, (3, int(left.sum())))
        x0, y0 = rng.integers(0, w), rng.integers(0, h)
        ex, ey = x0 + rng.integers(1, 48), y0 + rng.integers(1, 48)
        tgt[:, y0:ey, x0:ex] = rng.uniform(0, 1, (3, 1, 1))
        img[:, y0:ey, x0:ex] = tgt[:, y0:ey, x0:ex]
        tz = rng.uniform(0.5, 4.0, (h, w))
        z = tz + rng.normal(0, 0.05, (h, w))
        tz[rng.uniform(0, 1, (h, w)) < depth_invalid] = 0.0
        rgb.append(img.ravel())
        t_rgb.append(tgt.ravel())
        dep.append(z.ravel())
        t_dep.append(tz.ravel())
    return (_f32(np.concatenate(rgb)), _f32(np.concatenate(dep)), _f32(np.concatenate(t_rgb)),
            _f32(np.concatenate(t_dep)))


SCENES = {"c1": scene_c1, "c2": scene_c2, "c3": scene_c3, "c4": scene_c4, "c5": scene_c5}
