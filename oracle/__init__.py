"""FP64 CPU oracle of the differentiable tile rasterizer (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg import
this package.  It shares no code with the HIP path.
"""
from .ref import RefForward, forward, sh_basis, sh_basis_grad, quat_to_rotmat, load  # noqa: F401
from .loss import loss_l1  # noqa: F401
from .ssim import render_loss, ssim_map  # noqa: F401
from .adam import adam_update, fold_pose, se3_exp  # noqa: F401
