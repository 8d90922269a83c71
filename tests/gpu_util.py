"""Helpers shared by the GPU tests: move a scene to the device, run the HIP
path through the C-ABI binding, and compare with the oracle."""
import os

import numpy as np

IMG_TOL = 1e-4     # absolute, per channel, FP32 images vs the FP64 oracle
GRAD_REL = 1e-3    # relative, with a floor of 1e-2 * rms per tensor


def oracle_threads():
    return max(1, min(16, os.cpu_count() or 1))


def to_dev(scene):
    import torch
    d = {}
    for k in ("means", "log_scales", "quats", "opacity", "sh", "poses"):
        d[k] = torch.from_numpy(np.ascontiguousarray(getattr(scene, k), np.float32)).cuda()
    return d


def gpu_forward(rast, scene, tile=(16, 16), **kw):
    import torch
    d = to_dev(scene)
    rgb, dep, alp = rast.forward(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                                 d["poses"], scene.cams, scene.sh_degree, scene.background,
                                 tile=tile, **kw)
    torch.cuda.synchronize()
    # the library reads the inputs again in the backward: keep them alive
    rast._inputs = d
    return d, rgb, dep, alp


def gpu_backward(rast, G):
    import torch
    g = [torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda() for x in G]
    out = rast.backward(*g)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def masked_upstream(G, flags, sizes):
    """Zero the upstream gradients on the pixels the oracle flags as
    threshold-sensitive; both sides then agree on every decision of every
    pixel that carries gradient."""
    keep = (flags == 0).astype(np.float32)
    g_rgb = np.asarray(G[0], np.float32).copy()
    off = 0
    for (w, h) in sizes:
        P = w * h
        for c in range(3):
            g_rgb[3 * off + c * P:3 * off + (c + 1) * P] *= keep[off:off + P]
        off += P
    return g_rgb, (np.asarray(G[1], np.float32) * keep), (np.asarray(G[2], np.float32) * keep)


def expand_rgb_mask(px_mask, sizes):
    """Per-pixel mask -> mask over the packed [3,H,W]-per-frame rgb layout."""
    out, off = [], 0
    for (w, h) in sizes:
        P = w * h
        out.append(np.tile(px_mask[off:off + P], 3))
        off += P
    return np.concatenate(out)


def grad_bound(ref, rel=GRAD_REL):
    """Per-element bound rel * max(|g*|, 1e-2 |g*_block|, 1e-2 rms(g*)).

    ref has the Gaussian (or frame) index first; its block is that row, the
    parameter group of one Gaussian (3 means, 3 log-scales, 4 quaternion
    components, 1 opacity, 3 (d+1)^2 SH coefficients).  A component that
    cancels to below 1 % of its own group (the quaternion gradient after its
    tangent projection, one colour channel against the other two) is held to
    rel * 1e-2 of the group's norm: FP32 arithmetic errs in proportion to the
    group, not to the component."""
    ref = np.asarray(ref, np.float64)
    n = ref.shape[0] if ref.ndim else 1
    rows = ref.reshape(n, -1) if n else ref.reshape(0, 1)
    blk = np.repeat(np.sqrt((rows ** 2).sum(1)), rows.shape[1])
    flat = rows.ravel()
    rms = np.sqrt(np.mean(flat ** 2)) if flat.size else 0.0
    return rel * np.maximum(np.maximum(np.abs(flat), 1e-2 * blk), 1e-2 * rms)


def assert_grad_close(name, got, ref, rel=GRAD_REL):
    bound = grad_bound(ref, rel)
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    err = np.abs(got - ref)
    q = err / (bound + 1e-30)
    if q.size:
        print(f"[grad] {name}: max err/bound {q.max():.3g}, p99.9 {np.quantile(q, 0.999):.3g}",
              flush=True)
    bad = err > bound + 1e-30
    if bad.any():
        worst = np.argsort(-q)[:6]
        for i in worst:
            print(f"[grad]   {name}[{int(i)}] got {got[i]:.9g} ref {ref[i]:.9g} "
                  f"rel {err[i] / max(abs(ref[i]), 1e-300):.3g} |ref|/rms "
                  f"{abs(ref[i]) / max(rms, 1e-300):.3g}", flush=True)
        i = int(np.argmax(q))
        raise AssertionError(f"{name}: {int(bad.sum())} of {ref.size} elements exceed the "
                             f"bound; worst idx {i}: got {got[i]!r} ref {ref[i]!r} "
                             f"bound {bound[i]!r}")
