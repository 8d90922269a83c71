"""Adam and the SE(3) pose fold, plain FP64 numpy (test infrastructure).

The mapping loop optimises the Gaussians and the keyframe poses for a fixed
number of iterations (DROID-Splat supplementary S1.2; pose refinement
through the rendering objective, Sec. 3.3 and S1.3).  Adam (Kingma & Ba):
m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, p <- p - lr mhat / (sqrt(vhat)
+ eps), mhat = m / (1 - b1^t), vhat = v / (1 - b2^t).  A pose is updated by
its twist xi = (rho, phi) as T <- Exp(xi) T, Exp(xi) = [R(phi), V(phi) rho]
with R from the rotation vector and V = I + (1-cos t)/t^2 K + (t - sin t)/t^3
K^2, K = [phi]x, t = |phi|.
"""
import numpy as np
from scipy.spatial.transform import Rotation


def adam_update(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-15):
    """In-place Adam on FP64 arrays; t is the 1-based step number."""
    m[...] = b1 * m + (1 - b1) * g
    v[...] = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p[...] = p - lr * mh / (np.sqrt(vh) + eps)


def se3_exp(xi):
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-8:
        V = np.eye(3) + 0.5 * K
    else:
        V = np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * (K @ K)
    R = Rotation.from_rotvec(phi).as_matrix()
    return R, V @ rho


def fold_pose(pose, xi):
    """[R|t] world->camera -> Exp(xi) [R|t]."""
    Re, te = se3_exp(xi)
    R, t = pose[:, :3], pose[:, 3]
    return np.concatenate([Re @ R, (Re @ t + te)[:, None]], 1)
