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
