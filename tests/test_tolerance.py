"""The gradient bound used by the GPU parity tests (CPU only)."""
import numpy as np

from gpu_util import GRAD_REL, grad_bound


def test_bound_is_relative_to_element_block_and_tensor():
    ref = np.array([[10.0, 0.0, 0.0, 1e-3],      # small component of a large block
                    [1e-4, 2e-4, 0.0, 0.0],      # small block: the tensor floor applies
                    [1.0, -1.0, 0.5, 0.25]])
    b = grad_bound(ref).reshape(ref.shape)
    rms = np.sqrt(np.mean(ref ** 2))
    # element term
    assert np.isclose(b[0, 0], GRAD_REL * 10.0)
    assert np.isclose(b[2, 0], GRAD_REL * max(1.0, 1e-2 * np.sqrt(1 + 1 + 0.25 + 0.0625), 1e-2 * rms))
    # block term: 1 % of the row norm
    assert np.isclose(b[0, 3], GRAD_REL * 1e-2 * np.sqrt(100 + 1e-6))
    # tensor term: 1 % of the rms
    assert np.isclose(b[1, 2], GRAD_REL * 1e-2 * rms)


def test_bound_handles_vectors_and_empty():
    v = np.array([3.0, -4.0, 0.0])
    b = grad_bound(v)
    assert b.shape == (3,)
    assert np.isclose(b[2], GRAD_REL * 1e-2 * np.sqrt(np.mean(v ** 2)))
    assert grad_bound(np.zeros((0, 3))).size == 0


def test_noise_floor_is_far_below_the_relative_bound_on_a_plain_scene():
    """The oracle's response to 1e-6 per-pixel perturbations stays orders of
    magnitude below the 1e-3 bound for ordinary elements, so the noise term
    only widens the bound where the chain rule amplifies rounding."""
    import oracle
    from gpu_util import noise_floor, perturbed
    from paper_2411_17660_amd import scenes
    sc = scenes.tiny_scene(seed=3, n=300, W=64, H=48, f=50.0)
    ref = oracle.forward(sc)
    G = [x.astype(np.float64) for x in scenes.upstream(3, sc)]
    p1, p2 = perturbed(G), perturbed(G)
    assert all(np.array_equal(a, b) for a, b in zip(p1, p2))
    assert max(np.max(np.abs(a / np.where(g == 0, 1, g) - 1)) for a, g in zip(p1, G)) < 1e-5
    g = ref.backward(*G)
    nz = noise_floor(ref, G, g)
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        ratio = nz[k].ravel() / grad_bound(g[k])
        assert np.median(ratio) < 1e-2, k
