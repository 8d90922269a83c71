"""Parity of the densification kernels (HIP, through the C-ABI) against the
FP64 oracle (oracle/densify.py).

- ADC statistics: the per-Gaussian sum of |dL/d(u, v)| over kept frames is a
  function of the backward's screen-space gradient, so its bar is the
  gradient bar of the backward (1e-3 relative with its floors, or 3 times
  the oracle's own response to a 1e-6 jitter of the upstream); the counts
  are exact.
- MCMC noise and relocation run in FP64 and round once: 1e-6 relative per
  element (plus 1e-7 of the tensor's largest element); copied values are
  bitwise copies.
"""
import numpy as np
import pytest

import oracle
from oracle import densify as D
from paper_2411_17660_amd import scenes
from gpu_util import gpu_forward, gpu_backward, masked_upstream, perturbed, oracle_threads, \
    assert_grad_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    from paper_2411_17660_amd.raster import Rasterizer
    return Rasterizer(0)


def _t(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def _close(name, got, ref, rel=1e-6, abs_frac=1e-7):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    bound = rel * np.abs(ref) + abs_frac * (np.abs(ref).max() if ref.size else 0.0)
    q = float((np.abs(got - ref) / (bound + 1e-300)).max()) if ref.size else 0.0
    print(f"[densify] {name}: max err/bound {q:.3g}", flush=True)
    assert q <= 1.0, name


@pytest.mark.parametrize("label,make", [
    ("small", lambda: scenes.tiny_scene(seed=3, n=2000, W=130, H=70, f=100.0, n_frames=3,
                                        sh_degree=2, ls_mean=-3.0, opacity_sigma=1.5)),
    ("c2", lambda: scenes.scene_c2(seed=0, n=100_000))])
def test_densify_stats(rast, label, make):
    import torch
    sc = make()
    sizes = [(int(c[0]), int(c[1])) for c in sc.cams]
    print(f"[densify] stats {label}: oracle", flush=True)
    ref = oracle.forward(sc, threads=oracle_threads())
    flags = ref.pixel_info()[0]
    G = masked_upstream(scenes.upstream(5, sc), flags, sizes)
    gpu_forward(rast, sc)
    gpu_backward(rast, G)
    acc = torch.zeros(sc.n, device="cuda")
    cnt = torch.zeros(sc.n, device="cuda")
    rast.densify_stats(acc, cnt)
    rast.densify_stats(acc, cnt)       # accumulates
    torch.cuda.synchronize()
    ref.backward(*[g.astype(np.float64) for g in G])
    acc_ref, cnt_ref = D.densify_stats(ref)
    ref.backward(*[g.astype(np.float64) for g in perturbed(G)])
    acc_pert, _ = D.densify_stats(ref)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), 2 * cnt_ref.astype(np.int64))
    assert_grad_close(f"{label} grad_accum", acc.cpu().numpy() / 2, acc_ref,
                      noise=np.abs(acc_pert - acc_ref))


def test_densify_stats_needs_a_backward(rast):
    import torch
    from paper_2411_17660_amd.native import GsrError
    sc = scenes.tiny_scene(seed=4, n=50)
    gpu_forward(rast, sc)
    with pytest.raises(GsrError):
        rast.densify_stats(torch.zeros(sc.n, device="cuda"), torch.zeros(sc.n, device="cuda"))


def test_mcmc_noise(rast):
    import torch
    rng = np.random.default_rng(11)
    n = 200_003
    mu = rng.uniform(-2, 2, (n, 3)).astype(np.float32)
    ls = rng.normal(-3.5, 0.8, (n, 3)).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    lo = rng.normal(0, 3, n).astype(np.float32)
    lo[:1000] = 6.0                     # nearly opaque: gate ~ 0.4 .. 0
    eps = rng.normal(size=(n, 3)).astype(np.float32)
    scale = np.float32(1e4 * 1.6e-4)
    dm = _t(mu)
    rast.mcmc_noise(dm, _t(ls), _t(q), _t(lo), _t(eps), float(scale))
    torch.cuda.synchronize()
    ref = D.mcmc_noise(mu, ls, q, lo, eps, float(scale))
    got = dm.cpu().numpy()
    # FP64 evaluation rounded once: within FP32 rounding of the new means,
    # which is far below the displacement itself
    step = np.abs(ref - mu)
    assert np.median(step) > 1e3 * 2 ** -23 * np.median(np.abs(ref))
    err = np.abs(got - ref)
    print(f"[densify] noise: max err / ulp-bound {float((err / (2 ** -23 * np.abs(ref))).max()):.3g}",
          flush=True)
    assert np.all(err <= 2 ** -23 * np.abs(ref))


def _params(rng, n, K):
    return dict(means=rng.uniform(-2, 2, (n, 3)).astype(np.float32),
                log_scales=rng.normal(-3.5, 0.8, (n, 3)).astype(np.float32),
                quats=rng.normal(size=(n, 4)).astype(np.float32),
                opacity=rng.normal(0, 2.5, n).astype(np.float32),
                sh=rng.normal(size=(n, K, 3)).astype(np.float32))


def _gpu_relocate(rast, p, src, deg):
    import torch
    d = {k: _t(v) for k, v in p.items()}
    rast.mcmc_relocate(d["means"], d["log_scales"], d["quats"], d["opacity"], d["sh"],
                       _t(src, np.int32), deg)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in d.items()}


@pytest.mark.parametrize("n,deg,seed", [(50_000, 3, 12), (4_097, 0, 13)])
def test_mcmc_relocate(rast, n, deg, seed):
    rng = np.random.default_rng(seed)
    K = (deg + 1) ** 2
    p = _params(rng, n, K)
    o = 1 / (1 + np.exp(-p["opacity"].astype(np.float64)))
    dead = o < 0.05
    live = np.nonzero(~dead)[0]
    src = -np.ones(n, np.int64)
    src[dead] = rng.choice(live, size=int(dead.sum()), p=o[live] / o[live].sum())
    src[np.nonzero(dead)[0][:30]] = live[0]          # one source split 31 ways
    got = _gpu_relocate(rast, p, src, deg)
    ref = D.mcmc_relocate(p["means"], p["log_scales"], p["quats"], p["opacity"], p["sh"], src)
    print(f"[densify] relocate n={n}: {int(dead.sum())} dead", flush=True)
    for k, r in zip(("means", "log_scales", "quats", "opacity", "sh"), ref):
        r32 = np.asarray(r)
        if k in ("means", "quats", "sh"):
            assert np.array_equal(got[k], r32.astype(np.float32)), k   # copies
        else:
            _close(f"relocate {k}", got[k], r32, rel=1e-6, abs_frac=1e-7)


def test_mcmc_relocate_without_dead_is_identity(rast):
    rng = np.random.default_rng(14)
    p = _params(rng, 1000, 16)
    got = _gpu_relocate(rast, p, -np.ones(1000, np.int64), 3)
    for k in p:
        assert np.array_equal(got[k], p[k]), k
