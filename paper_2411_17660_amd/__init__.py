"""MI355X-native differentiable tile rasterizer for 3D Gaussian Splatting.

The hot path of DROID-Splat's renderer (Sec. 3.3): Gaussians, pinhole
cameras and world->camera poses in; RGB, alpha-blended depth and accumulated
alpha out, with gradients for every Gaussian parameter and each pose twist.
All compute runs in hand-written HIP kernels for gfx950 behind the C-ABI
library libgsr.so (include/gsr.h); this package only marshals arguments.
"""
__all__ = ["scenes"]
