"""FP64 CPU oracle of the differentiable tile rasterizer (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg import
this package.  It shares no code with the HIP path.
"""
from .ref import RefForward, forward, sh_basis, sh_basis_grad, quat_to_rotmat, load  # noqa: F401
from .loss import loss_l1  # noqa: F401
