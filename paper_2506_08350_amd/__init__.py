"""MI355X-native hot path of complex-valued holographic radiance fields.

Complex 3D Gaussians -> projection and culling -> tile binning with a stable
radix sort -> front-to-back complex compositing -> band-limited angular
spectrum propagation to K planes -> |u|^2, with the analytic backward.  All
steps run in the HIP library ``libchrf.so`` (C ABI in ``include/chrf.h``);
``api`` wraps it for PyTorch tensors and autograd.
"""
from . import _lib  # noqa: F401
from . import api  # noqa: F401

__all__ = ["_lib", "api"]
