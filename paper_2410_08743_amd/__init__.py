"""Pose-differentiable 3D Gaussian splatting rasterizer for MI355X (gfx950).

Hot path of "Look Gauss, No Pose" (arXiv 2410.08743, Sec. III-A/III-B): a
tile rasterizer, forward and backward, with analytic gradients of the loss
with respect to each camera's se(3) twist, implemented as hand-written HIP
kernels behind the C ABI declared in include/gsp.h.  The Python layer only
marshals arguments; importing a submodule that needs the native library
raises when libgsp.so is missing.
"""
__version__ = "0.1.0"
