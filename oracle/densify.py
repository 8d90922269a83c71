"""Densification support, plain FP64 numpy (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use
this module; it shares no code with the HIP path.

DROID-Splat grows its map either by the adaptive density control of 3DGS,
which splits and clones Gaussians by their size and positional gradient, or
by MCMC densification with a capped number of Gaussians and position noise
(Sec. 3.3; lr_noise = 1e4 and the cap in supplementary S1.2; the variants
compared in tab:renderer).  The per-step pieces that touch every Gaussian:

densify_stats  (ADC): for every kept (Gaussian, frame) record of the last
    backward, the norm of the gradient of the loss with respect to the
    record's projected mean, |dL/d(u, v)|_2 in pixel units, summed per
    Gaussian, and the number of such records.  The split/clone/prune
    decisions on these statistics are host logic.

mcmc_noise  (MCMC): means += s * gate(o) * Sigma eps, with Sigma = R diag(s^2)
    R^T the Gaussian's covariance, o its opacity, gate(o) =
    1 / (1 + exp(k (o - t))) with k = 100 and t = 1 - 0.005 (Gaussians near
    full opacity are not moved), eps ~ N(0, I) drawn by the caller and s =
    lr_noise * the current position learning rate.

mcmc_relocate  (MCMC): dead Gaussians (the caller's choice, opacity below
    0.005 in the method) take the place of live sources the caller samples
    in proportion to opacity; src[g] is the source of dead g, -1 for the
    others.  A source i chosen c times is split into N = c + 1 equal copies
    (itself and the c dead slots) at its position, with
        o' = 1 - (1 - o)^(1/N),
        s' = s * o / sum_{j=1}^{N} sum_{k=0}^{j-1} C(j-1, k) (-1)^k o'^(k+1) / sqrt(k+1),
    so that N copies composited at the centre give back opacity o, and along
    a line through the centre the integral of the composited opacity
    equals that of the original.  Means, rotations and SH are copied.
    (Kheradmand et al., the MCMC method the paper cites.)
"""
import math

import numpy as np

GATE_K = 100.0
GATE_T = 1.0 - 0.005


def densify_stats(ref):
    """(grad_accum [n], count [n]) of the last backward of an oracle
    RefForward."""
    n, F = ref.n, ref.F
    sg = ref.screen_grads()
    keep = ref.records()["keep"].astype(bool).reshape(F, n)
    norm = np.hypot(sg[:, 0], sg[:, 1]).reshape(F, n)
    return np.where(keep, norm, 0.0).sum(0), keep.sum(0).astype(np.float64)


def rotation(q):
    """Unit-quaternion (w, x, y, z) rotation matrices [n,3,3]."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)


def sigmoid(v):
    return 1.0 / (1.0 + np.exp(-np.asarray(v, np.float64)))


def gate(o):
    return 1.0 / (1.0 + np.exp(GATE_K * (np.asarray(o, np.float64) - GATE_T)))


def mcmc_noise(means, log_scales, quats, opacity_logits, eps, scale):
    """New means (FP64)."""
    R = rotation(quats)
    s2 = np.exp(2.0 * np.asarray(log_scales, np.float64))
    cov = np.einsum("nij,nj,nkj->nik", R, s2, R)
    step = np.einsum("nij,nj->ni", cov, np.asarray(eps, np.float64))
    g = gate(sigmoid(opacity_logits))
    return np.asarray(means, np.float64) + float(scale) * g[:, None] * step


def relocated_opacity_scale(o, N):
    """(o', scale factor s'/s) of one source split into N copies."""
    o_new = 1.0 - (1.0 - o) ** (1.0 / N)
    denom = 0.0
    for j in range(1, N + 1):
        for k in range(j):
            denom += math.comb(j - 1, k) * (-1.0) ** k * o_new ** (k + 1) / math.sqrt(k + 1)
    return o_new, o / denom


def mcmc_relocate(means, log_scales, quats, opacity_logits, sh, src):
    """New (means, log_scales, quats, opacity_logits, sh) in FP64."""
    src = np.asarray(src, np.int64)
    out = [np.array(a, np.float64) for a in (means, log_scales, quats, opacity_logits, sh)]
    n = src.size
    counts = np.ones(n, np.int64)
    for i in src[src >= 0]:
        counts[i] += 1
    for i in np.nonzero(counts > 1)[0]:
        o = float(sigmoid(out[3][i]))
        o_new, f = relocated_opacity_scale(o, int(counts[i]))
        out[3][i] = math.log(o_new / (1.0 - o_new))
        out[1][i] = out[1][i] + math.log(f)
    for g in np.nonzero(src >= 0)[0]:
        i = src[g]
        for a in out:
            a[g] = a[i]
    return tuple(out)
