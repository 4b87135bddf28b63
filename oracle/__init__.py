"""CPU oracle for the complex-hologram hot path (test infrastructure only).

A plain, slow, FP64 NumPy implementation of what the GPU path computes:
projection of complex 3D Gaussians (Sec. 3, Eqs. 2-4 and 8), front-to-back
complex compositing (Eqs. 10 and 13 with L = 1; Algorithm 2; Supplementary D
forward equations), band-limited angular-spectrum propagation (Eqs. 7, 14, 16),
the focal-stack MSE (Eq. 17) and the analytic gradient of all of it
(Supplementary D backward pass); ``layers.py`` adds the multi-layer hologram
with hard plane assignment, forward recording and inverse propagation
(Sec. 4.1, Eqs. 12-16) and its gradient with the straight-through estimator;
``losses.py`` the paper's training loss (masked three-term reconstruction
loss plus the SSIM term) and its gradient; ``phase_only.py`` the loss and
phase gradient of the phase-only hologram conversion; ``training.py`` the
Adan update and the densification of the optimisation loop.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never calls it; the product path must not route through it.

Precision: FP64 everywhere except the integer decisions that the GPU takes in
FP32 (the depth sort key and the pixel/tile rectangle of each Gaussian); for
those the oracle follows the same fixed single-precision recipe, written out
independently in ``binning.py``.
"""
from .projection import quat_to_rotmat, project, ProjectedGaussians
from .binning import fp32_footprint, bin_pairs
from .raster import render_field, render_field_backward, RasterResult
from .asm import transfer_function, band_mask, propagate, propagate_adjoint
from .pipeline import Thresholds, SMOOTH, DEFAULT, forward, backward, mse_loss
from . import layers, losses, phase_only, training

__all__ = [
    "quat_to_rotmat", "project", "ProjectedGaussians", "fp32_footprint", "bin_pairs",
    "render_field", "render_field_backward", "RasterResult", "transfer_function",
    "band_mask", "propagate", "propagate_adjoint", "Thresholds", "SMOOTH", "DEFAULT",
    "forward", "backward", "mse_loss", "layers", "losses", "phase_only", "training",
]
