"""PyTorch-facing API of the HIP tile rasterizer.

`Rasterizer` owns one library context (workspace, saved forward state) and
renders a batch of keyframes into packed device tensors.  `rasterize` is the
differentiable entry point behind a torch.autograd.Function: its backward
calls the library's hand-written backward.  The pose gradient is the
left-perturbation twist xi = (rho, phi) at xi = 0 (DROID-Splat Sec. 3.3, pose
refinement through the rendering objective); a caller that optimises poses
keeps a zero twist tensor per frame and folds each step into the pose.
PyTorch provides device memory and the stream only.
"""
import ctypes as C

import numpy as np
import torch

from . import native


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), \
        "tensors must be contiguous float32 on the GPU"
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Rasterizer:
    """One library context on one device."""

    def __init__(self, device=0):
        self.lib = native.load()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.gsr_create(C.byref(h), int(device))
        if rc != native.GSR_OK:
            raise native.GsrError(rc, f"gsr_create(device={device}) failed")
        self.h = h
        self.n = 0
        self.F = 0
        self.sizes = []
        # advanced by every call that replaces the saved forward state, so that
        # a backward can tell whether the state it reads is still its own
        self.generation = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.gsr_destroy(h)
            self.h = None

    def _check(self, rc):
        if rc != native.GSR_OK:
            raise native.GsrError(rc, self.lib.gsr_last_error(self.h).decode())

    def forward(self, means, log_scales, quats, opacity, sh, poses, cams, sh_degree,
                background=(0.0, 0.0, 0.0), tile=(16, 16), key_capacity=0, xcd_remap=True,
                out=None, timing=False, count_pairs=False, median=False, lds_batch=0):
        """Renders F frames; returns packed (rgb [sum 3HW], depth [sum HW],
        alpha [sum HW]) float32 device tensors."""
        F = len(cams)
        P = int(sum(int(c[0]) * int(c[1]) for c in cams))
        dev = means.device
        if out is None:
            rgb = torch.empty(3 * P, device=dev, dtype=torch.float32)
            depth = torch.empty(P, device=dev, dtype=torch.float32)
            alpha = torch.empty(P, device=dev, dtype=torch.float32)
        else:
            rgb, depth, alpha = out
        self.settings = native.make_settings(sh_degree, background, tile, key_capacity,
                                             xcd_remap, lds_batch=lds_batch, timing=timing,
                                             count_pairs=count_pairs, median=median)
        self.cams = native.make_cameras(cams)
        n = int(means.shape[0])
        self.generation += 1
        self._check(self.lib.gsr_forward(self.h, C.byref(self.settings), n, _ptr(means),
                                         _ptr(log_scales), _ptr(quats), _ptr(opacity), _ptr(sh),
                                         F, self.cams, _ptr(poses), _ptr(rgb), _ptr(depth),
                                         _ptr(alpha), _stream()))
        self.n, self.F, self.sh_degree = n, F, sh_degree
        self.sizes = [(int(c[0]), int(c[1])) for c in cams]
        # gsr_loss_l1 reads these buffers by pointer: keep them alive
        self._fwd_out = (rgb, depth, alpha)
        return rgb, depth, alpha

    def forward_surfel(self, means, log_scales, quats, opacity, sh, poses, cams, sh_degree,
                       background=(0.0, 0.0, 0.0), tile=(16, 16), key_capacity=0, out=None,
                       timing=False, count_pairs=False):
        """Renders F frames of 2D surfels (log_scales [n,2]); returns packed
        (rgb, depth, alpha, normal [sum 3HW], dist [sum HW])."""
        P = int(sum(int(c[0]) * int(c[1]) for c in cams))
        dev = means.device
        if out is None:
            out = (torch.empty(3 * P, device=dev), torch.empty(P, device=dev),
                   torch.empty(P, device=dev), torch.empty(3 * P, device=dev),
                   torch.empty(P, device=dev))
        rgb, depth, alpha, normal, dist = out
        self.settings = native.make_settings(sh_degree, background, tile, key_capacity,
                                             timing=timing, count_pairs=count_pairs)
        self.cams = native.make_cameras(cams)
        n = int(means.shape[0])
        self.generation += 1
        self._check(self.lib.gsr_forward_surfel(
            self.h, C.byref(self.settings), n, _ptr(means), _ptr(log_scales), _ptr(quats),
            _ptr(opacity), _ptr(sh), len(cams), self.cams, _ptr(poses), _ptr(rgb), _ptr(depth),
            _ptr(alpha), _ptr(normal), _ptr(dist), _stream()))
        self.n, self.F, self.sh_degree = n, len(cams), sh_degree
        self.sizes = [(int(c[0]), int(c[1])) for c in cams]
        self._fwd_out = out
        return rgb, depth, alpha, normal, dist

    def normal_consistency(self, cams, depth, alpha, normal, weight, g_depth, g_alpha,
                           g_normal, loss=None):
        """weight * (normal-consistency term) of packed depth / alpha / normal
        images; adds its gradient to g_depth, g_alpha, g_normal and returns
        the loss (device float tensor [1])."""
        if loss is None:
            loss = torch.empty(1, device=depth.device)
        cm = native.make_cameras(cams)
        self._check(self.lib.gsr_normal_consistency(
            self.h, len(cams), cm, _ptr(depth), _ptr(alpha), _ptr(normal), float(weight),
            _ptr(loss), _ptr(g_depth), _ptr(g_alpha), _ptr(g_normal), _stream()))
        return loss

    def backward_surfel(self, g_rgb, g_depth, g_alpha, g_normal, g_dist, out=None):
        """Gradients of the last forward_surfel for upstream gradients of its
        five outputs; returns means [n,3], log_scales [n,2], quats [n,4],
        opacity [n], sh [n,K,3], twist [F,6]."""
        n, F = self.n, self.F
        dev = g_rgb.device
        K = (self.sh_degree + 1) ** 2
        if out is None:
            out = dict(means=torch.empty(n, 3, device=dev), log_scales=torch.empty(n, 2, device=dev),
                       quats=torch.empty(n, 4, device=dev), opacity=torch.empty(n, device=dev),
                       sh=torch.empty(n, K, 3, device=dev), twist=torch.empty(F, 6, device=dev))
        self._check(self.lib.gsr_backward_surfel(
            self.h, _ptr(g_rgb), _ptr(g_depth), _ptr(g_alpha), _ptr(g_normal), _ptr(g_dist),
            _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
            _ptr(out["opacity"]), _ptr(out["sh"]), _ptr(out["twist"]), _stream()))
        return out

    def backward(self, g_rgb, g_depth, g_alpha, out=None):
        n, F = self.n, self.F
        dev = g_rgb.device
        K = (self.sh_degree + 1) ** 2
        if out is None:
            out = dict(means=torch.empty(n, 3, device=dev), log_scales=torch.empty(n, 3, device=dev),
                       quats=torch.empty(n, 4, device=dev), opacity=torch.empty(n, device=dev),
                       sh=torch.empty(n, K, 3, device=dev), twist=torch.empty(F, 6, device=dev))
        self._check(self.lib.gsr_backward(self.h, _ptr(g_rgb), _ptr(g_depth), _ptr(g_alpha),
                                          _ptr(out["means"]), _ptr(out["log_scales"]),
                                          _ptr(out["quats"]), _ptr(out["opacity"]),
                                          _ptr(out["sh"]), _ptr(out["twist"]), _stream()))
        return out

    def loss_l1(self, target_rgb, target_depth, depth_weight, out=None):
        dev = target_rgb.device
        if out is None:
            P = target_depth.numel()
            out = dict(loss=torch.empty(1, device=dev), g_rgb=torch.empty(3 * P, device=dev),
                       g_depth=torch.empty(P, device=dev), g_alpha=torch.empty(P, device=dev))
        self._check(self.lib.gsr_loss_l1(self.h, _ptr(target_rgb), _ptr(target_depth),
                                         float(depth_weight), _ptr(out["loss"]),
                                         _ptr(out["g_rgb"]), _ptr(out["g_depth"]),
                                         _ptr(out["g_alpha"]), _stream()))
        return out

    def loss_l1_noalloc(self, target_rgb, target_depth, depth_weight, out):
        """loss_l1 into preallocated `out` (dict loss, g_rgb, g_depth,
        g_alpha) through the entry point that allocates no device memory."""
        self._check(self.lib.gsr_loss_l1_noalloc(self.h, _ptr(target_rgb), _ptr(target_depth),
                                                 float(depth_weight), _ptr(out["loss"]),
                                                 _ptr(out["g_rgb"]), _ptr(out["g_depth"]),
                                                 _ptr(out["g_alpha"]), _stream()))
        return out

    def loss_render(self, rgb, depth, target_rgb, target_depth, lambda1=0.9, lambda2=0.2,
                    out=None):
        """Full rendering loss (L1 + SSIM colour term, L1 depth term) of
        images packed like the last forward's outputs; returns dict(loss,
        ssim [F], g_rgb, g_depth, g_alpha)."""
        dev = target_rgb.device
        if out is None:
            P = target_depth.numel()
            out = dict(loss=torch.empty(1, device=dev), ssim=torch.empty(self.F, device=dev),
                       g_rgb=torch.empty(3 * P, device=dev), g_depth=torch.empty(P, device=dev),
                       g_alpha=torch.empty(P, device=dev))
        self._check(self.lib.gsr_loss_render(
            self.h, _ptr(rgb), _ptr(depth), _ptr(target_rgb), _ptr(target_depth),
            float(lambda1), float(lambda2), _ptr(out["loss"]), _ptr(out.get("ssim")),
            _ptr(out["g_rgb"]), _ptr(out["g_depth"]), _ptr(out["g_alpha"]), _stream()))
        return out

    def step_render(self, means, log_scales, quats, opacity, sh, poses, cams, sh_degree,
                    target_rgb, target_depth, bufs, lambda1=0.9, lambda2=0.2,
                    background=(0.0, 0.0, 0.0), tile=(16, 16), key_capacity=0, xcd_remap=True,
                    timing=False, median=False, lds_batch=0):
        """Forward + full rendering loss + backward in one call into
        preallocated `bufs` (as for step_l1, plus an optional `ssim` [F])."""
        self.settings = native.make_settings(sh_degree, background, tile, key_capacity,
                                             xcd_remap, lds_batch=lds_batch, timing=timing,
                                             median=median)
        self.cams = native.make_cameras(cams)
        n = int(means.shape[0])
        b = bufs
        self.generation += 1
        self._check(self.lib.gsr_step_render(
            self.h, C.byref(self.settings), n, _ptr(means), _ptr(log_scales), _ptr(quats),
            _ptr(opacity), _ptr(sh), len(cams), self.cams, _ptr(poses), _ptr(target_rgb),
            _ptr(target_depth), float(lambda1), float(lambda2), _ptr(b["rgb"]),
            _ptr(b["depth"]), _ptr(b["alpha"]), _ptr(b["loss"]), _ptr(b.get("ssim")),
            _ptr(b["means"]), _ptr(b["log_scales"]), _ptr(b["quats"]), _ptr(b["opacity"]),
            _ptr(b["sh"]), _ptr(b["twist"]), _stream()))
        self.n, self.F, self.sh_degree = n, len(cams), sh_degree
        self.sizes = [(int(c[0]), int(c[1])) for c in cams]
        self._fwd_out = (b["rgb"], b["depth"], b["alpha"])

    def densify_stats(self, grad_accum, count):
        """Adds the last backward's |dL/d(u, v)| per kept (Gaussian, frame)
        to grad_accum [n] and the number of such frames to count [n]."""
        self._check(self.lib.gsr_densify_stats(self.h, _ptr(grad_accum), _ptr(count), _stream()))

    def mcmc_noise(self, means, log_scales, quats, opacity, eps, scale):
        """means += scale * gate(opacity) * Sigma eps, in place."""
        self._check(self.lib.gsr_mcmc_noise(self.h, int(means.shape[0]), _ptr(means),
                                            _ptr(log_scales), _ptr(quats), _ptr(opacity),
                                            _ptr(eps), float(scale), _stream()))

    def mcmc_relocate(self, means, log_scales, quats, opacity, sh, src, sh_degree):
        """Moves dead Gaussians (src[g] = source index, else -1; int32) onto
        their sources with the relocation rule, in place."""
        assert src.is_cuda and src.dtype == torch.int32 and src.is_contiguous()
        self._check(self.lib.gsr_mcmc_relocate(
            self.h, int(means.shape[0]), int(sh_degree), _ptr(means), _ptr(log_scales),
            _ptr(quats), _ptr(opacity), _ptr(sh), C.c_void_p(src.data_ptr()), _stream()))

    def step_l1(self, means, log_scales, quats, opacity, sh, poses, cams, sh_degree,
                target_rgb, target_depth, depth_weight, bufs, background=(0.0, 0.0, 0.0),
                tile=(16, 16), key_capacity=0, xcd_remap=True, timing=False, median=False,
                lds_batch=0):
        """Forward + L1 loss + backward in one call into preallocated `bufs`
        (dict with rgb, depth, alpha, loss and the gradient tensors)."""
        self.settings = native.make_settings(sh_degree, background, tile, key_capacity,
                                             xcd_remap, lds_batch=lds_batch, timing=timing,
                                             median=median)
        self.cams = native.make_cameras(cams)
        n = int(means.shape[0])
        b = bufs
        self.generation += 1
        self._check(self.lib.gsr_step_l1(
            self.h, C.byref(self.settings), n, _ptr(means), _ptr(log_scales), _ptr(quats),
            _ptr(opacity), _ptr(sh), len(cams), self.cams, _ptr(poses), _ptr(target_rgb),
            _ptr(target_depth), float(depth_weight), _ptr(b["rgb"]), _ptr(b["depth"]),
            _ptr(b["alpha"]), _ptr(b["loss"]), _ptr(b["means"]), _ptr(b["log_scales"]),
            _ptr(b["quats"]), _ptr(b["opacity"]), _ptr(b["sh"]), _ptr(b["twist"]), _stream()))
        self.n, self.F, self.sh_degree = n, len(cams), sh_degree
        self.sizes = [(int(c[0]), int(c[1])) for c in cams]
        self._fwd_out = (b["rgb"], b["depth"], b["alpha"])

    def autotune(self, means, log_scales, quats, opacity, sh, poses, cams, sh_degree,
                 target_rgb, target_depth, depth_weight, background=(0.0, 0.0, 0.0), reps=3,
                 force=False):
        """Measure every tile shape with every LDS batch on these inputs;
        returns (tile, lds_batch, key_capacity, {(tile, batch): median ms})."""
        base = native.make_settings(sh_degree, background)
        chosen = native.Settings()
        nt, nbt = len(native.TILE_SHAPES), len(native.LDS_BATCHES)
        ms = (C.c_float * (nt * nbt))()
        cams_c = native.make_cameras(cams)
        self.generation += 1
        self._check(self.lib.gsr_autotune(
            self.h, C.byref(base), int(means.shape[0]), _ptr(means), _ptr(log_scales),
            _ptr(quats), _ptr(opacity), _ptr(sh), len(cams), cams_c, _ptr(poses),
            _ptr(target_rgb), _ptr(target_depth), float(depth_weight), int(reps), int(force),
            C.byref(chosen), ms, _stream()))
        times = {(t, b): ms[i * nbt + j] for i, t in enumerate(native.TILE_SHAPES)
                 for j, b in enumerate(native.LDS_BATCHES)}
        return (chosen.tile_w, chosen.tile_h), chosen.lds_batch, chosen.key_capacity, times

    def adam_step(self, params, grads, state, lr_means=1.6e-4, lr_sh=5e-3, lr_pose=1e-3,
                  beta1=0.9, beta2=0.999, eps=1e-15):
        """Fused Adam on means, SH and pose twists with the pose fold.
        params: dict(means, sh, poses); grads: dict(means, sh, twist);
        state: dict(m_means, v_means, m_sh, v_sh, m_twist, v_twist, step)."""
        n = int(params["means"].shape[0])
        deg = int(round((params["sh"].shape[1]) ** 0.5)) - 1
        F = int(params["poses"].shape[0])
        p, g, s = params, grads, state
        self._check(self.lib.gsr_adam_step(
            self.h, n, deg, _ptr(p["means"]), _ptr(g["means"]), _ptr(s["m_means"]),
            _ptr(s["v_means"]), _ptr(p["sh"]), _ptr(g["sh"]), _ptr(s["m_sh"]), _ptr(s["v_sh"]),
            F, _ptr(p["poses"]), _ptr(g["twist"]), _ptr(s["m_twist"]), _ptr(s["v_twist"]),
            float(lr_means), float(lr_sh), float(lr_pose), float(beta1), float(beta2),
            float(eps), C.c_void_p(s["step"].data_ptr()), _stream()))

    def timings(self):
        """{stage: (total ms, launches)} of the timed calls since the last read."""
        ms = (C.c_double * len(native.STAGES))()
        calls = (C.c_int64 * len(native.STAGES))()
        self._check(self.lib.gsr_debug_timings(self.h, ms, calls))
        return {name: (ms[i], calls[i]) for i, name in enumerate(native.STAGES)}

    def debug_copy(self, src, dst):
        """dst <- src by the library's plain 16-byte copy kernel (bandwidth
        reference); both contiguous device tensors of the same byte size."""
        nbytes = src.numel() * src.element_size()
        assert src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()
        assert dst.numel() * dst.element_size() == nbytes
        self._check(self.lib.gsr_debug_copy(self.h, C.c_void_p(src.data_ptr()),
                                            C.c_void_p(dst.data_ptr()), nbytes, _stream()))

    def check_overflow(self):
        self._check(self.lib.gsr_check_overflow(self.h, _stream()))

    def stats(self):
        s = native.Stats()
        self._check(self.lib.gsr_debug_stats(self.h, C.byref(s), _stream()))
        return {k: getattr(s, k) for k, _ in native.Stats._fields_}

    def debug_lists(self):
        """Integer artefacts of the last forward as numpy arrays."""
        st = self.stats()
        M, K, T, P = st["n_records"], st["n_keys"], st["n_tiles"], st["n_pixels"]
        K = min(K, st["key_capacity"])
        out = dict(ntiles=np.zeros(M, np.uint32), depth_key=np.zeros(M, np.uint32),
                   square=np.zeros(2 * M, np.uint32), tile_keys=np.zeros(max(K, 1), np.uint32),
                   tile_vals=np.zeros(max(K, 1), np.uint32), ranges=np.zeros(2 * T, np.uint32),
                   n_last=np.zeros(P, np.int32), t_final=np.zeros(P, np.float32))

        def p(a):
            return C.c_void_p(a.ctypes.data)
        self._check(self.lib.gsr_debug_lists(self.h, p(out["ntiles"]), p(out["depth_key"]),
                                             p(out["square"]), p(out["tile_keys"]),
                                             p(out["tile_vals"]), p(out["ranges"]),
                                             p(out["n_last"]), p(out["t_final"]), _stream()))
        out["tile_keys"] = out["tile_keys"][:K]
        out["tile_vals"] = out["tile_vals"][:K]
        out["K"] = K
        return out

    def debug_grad2d(self):
        """Per-record screen-space gradients of the last backward, [n*F, 10]:
        d/du, d/dv, d/dSigma'_xx, d/dSigma'_xy, d/dSigma'_yy, d/dopacity,
        d/dcolour (3), d/dz."""
        M = self.stats()["n_records"]
        out = np.zeros((max(M, 1), 10), np.float64)
        self._check(self.lib.gsr_debug_grad2d(self.h, C.c_void_p(out.ctypes.data), _stream()))
        return out[:M]


class _RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity, sh, twist, poses, cams, sh_degree,
                background, tile, rast, median):
        inputs = [t.contiguous() for t in (means, log_scales, quats, opacity, sh, poses)]
        rgb, depth, alpha = rast.forward(*inputs, cams, sh_degree, background, tile,
                                         median=median)
        # the library's backward reads the inputs again: hold them until then
        ctx.inputs = inputs
        ctx.rast = rast
        ctx.generation = rast.generation
        return rgb, depth, alpha

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha):
        rast = ctx.rast
        if rast.generation != ctx.generation:
            raise RuntimeError(
                "rasterize(): the Rasterizer rendered again before this backward; run "
                "each forward's backward before the next forward on the same Rasterizer, "
                "or give each render its own Rasterizer")
        dev = next(t.device for t in (g_rgb, g_depth, g_alpha) if t is not None)
        P = sum(w * h for w, h in rast.sizes)

        def z(t, size):
            return t.contiguous() if t is not None else torch.zeros(size, device=dev)
        g = rast.backward(z(g_rgb, 3 * P), z(g_depth, P), z(g_alpha, P))
        ctx.inputs = None
        return (g["means"], g["log_scales"], g["quats"], g["opacity"], g["sh"], g["twist"],
                None, None, None, None, None, None, None)


_default = {}


def default_rasterizer(device=0):
    """One shared Rasterizer (library context and workspace) per device."""
    r = _default.get(device)
    if r is None:
        r = _default[device] = Rasterizer(device)
    return r


def rasterize(means, log_scales, quats, opacity, sh, poses, cams, sh_degree, twist=None,
              background=(0.0, 0.0, 0.0), tile=(16, 16), rasterizer=None, median=False,
              check_twist=True):
    """Differentiable render of F keyframes.  Returns packed (rgb, depth,
    alpha); depth is alpha-blended, or the median depth with median=True.

    Gradients reach every Gaussian tensor and `twist` ([F,6], the
    left-perturbation xi = (rho, phi) of each pose, T_f <- Exp(xi_f) T_f).
    The library differentiates at xi = 0, so `twist` must hold zeros: after
    an optimiser step on it, fold it into the poses (Rasterizer.adam_step
    does the fold) and zero it.  check_twist verifies this with one
    device-to-host read per call.  Renders share `rasterizer` (default: one
    per device); the backward of a render must run before the next render on
    the same rasterizer, else it raises."""
    dev = means.device.index if means.device.index is not None else 0
    rast = rasterizer if rasterizer is not None else default_rasterizer(dev)
    if twist is None:
        twist = torch.zeros(len(cams), 6, device=means.device)
    elif check_twist and int(torch.count_nonzero(twist.detach())) != 0:
        raise ValueError("rasterize(): twist must be zero (the pose gradient is taken at "
                         "xi = 0); fold a twist into the poses before rendering")
    return _RasterizeFn.apply(means, log_scales, quats, opacity, sh, twist, poses, cams,
                              sh_degree, tuple(background), tuple(tile), rast, bool(median))
