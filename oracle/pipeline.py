"""FP64 end-to-end forward and backward of the hot path.

forward:  per view b, project (projection.py) -> footprint (binning.py) ->
          composite U[b, l] (raster.py) -> for every wavelength l and distance
          z_k: u[b, l, k] = ASM(U[b, l]; lambda_l, z_k) (asm.py),
          I = |u|^2 (Eq. 16), optional loss = mean((I - I_gt)^2) (Eq. 17 with
          the mean over every element; reading: the paper's 1/L sum of squared
          norms differs only by a constant factor).
backward: dL/dI -> G_u = 2 u dL/dI (+ dL/du) -> G_U = sum_k ASM^H(G_u[k])
          -> raster backward -> projection backward, summed over views.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .asm import propagate, propagate_adjoint
from .binning import fp32_footprint
from .projection import project, project_backward
from .raster import render_field, render_field_backward


@dataclass(frozen=True)
class Thresholds:
    """Compositing thresholds.  The paper names epsilon_T and the support test
    but prints no values; the defaults are the 3D Gaussian splatting ones it
    builds on (k = 3, alpha_min = 1/255, alpha_max = 0.99, T_min = 1e-4)."""
    k_sigma: float = 3.0
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4


DEFAULT = Thresholds()
# Differentiable everywhere that matters: used by the finite-difference pins.
# alpha_max is the largest single-precision value below 1 (the backward
# recovers T by dividing by 1 - alpha, so the GPU plans require alpha_max < 1);
# no opacity of these scenes reaches it, so nothing clamps.
SMOOTH = Thresholds(k_sigma=8.0, alpha_min=0.0, alpha_max=1.0 - 2.0 ** -24, t_min=0.0)


def mse_loss(I, target):
    return float(np.mean((np.asarray(I, np.float64) - np.asarray(target, np.float64)) ** 2))


def forward(scene, cameras, optics, thr=DEFAULT, targets=None, tile=(16, 16), keep_field=True):
    views = []
    B = len(cameras)
    L = scene.n_lambda
    K = len(optics.distances)
    H, W = cameras[0].height, cameras[0].width
    u = np.zeros((B, L, K, H, W), np.complex128)
    for b, cam in enumerate(cameras):
        proj = project(scene.means, scene.log_scales, scene.quats, scene.amp, scene.phase, cam)
        fp = fp32_footprint(scene.means, scene.log_scales, scene.quats, cam, tile[0], tile[1], thr.k_sigma,
                            scene.opacity, thr.alpha_min)
        res = render_field(proj, scene.opacity, fp, W, H, thr)
        for li, lam in enumerate(optics.wavelengths):
            for ki, z in enumerate(optics.distances):
                u[b, li, ki] = propagate(res.U[li], lam, z, optics.pitch, optics.pad, optics.band_limit)
        views.append({"proj": proj, "fp": fp, "res": res, "cam": cam})
    I = np.abs(u) ** 2
    out = {"views": views, "u": u, "I": I, "U": np.stack([v["res"].U for v in views]),
           "scene": scene, "optics": optics, "thr": thr}
    if targets is not None:
        out["loss"] = mse_loss(I, targets)
        out["targets"] = np.asarray(targets, np.float64)
    return out


def backward(state, dL_dI=None, dL_du=None):
    """Gradients of the loss w.r.t. the scene parameters (FP64 dict)."""
    scene, optics, thr = state["scene"], state["optics"], state["thr"]
    u, I = state["u"], state["I"]
    if dL_dI is None:
        dL_dI = 2.0 * (I - state["targets"]) / I.size
    G_u = 2.0 * u * dL_dI
    if dL_du is not None:
        G_u = G_u + dL_du
    grads = {k: np.zeros(a.shape, np.float64) for k, a in
             zip(("means", "log_scales", "quats", "opacity", "amp", "phase"), scene.arrays())}
    for b, view in enumerate(state["views"]):
        G_U = np.zeros_like(view["res"].U)
        for li, lam in enumerate(optics.wavelengths):
            for ki, z in enumerate(optics.distances):
                G_U[li] += propagate_adjoint(G_u[b, li, ki], lam, z, optics.pitch, optics.pad, optics.band_limit)
        d_mu, d_conic, d_op, d_v = render_field_backward(view["proj"], scene.opacity, view["fp"], view["res"], G_U, thr)
        g = project_backward(view["proj"], scene.quats, scene.amp, scene.phase, view["cam"], d_mu, d_conic, d_op, d_v)
        vis = view["fp"]["visible"]
        for k in grads:
            m = vis.reshape((-1,) + (1,) * (g[k].ndim - 1))
            grads[k] += np.where(m, np.nan_to_num(g[k]), 0.0)
        view["G_U"] = G_U
        view["d_mu"] = d_mu   # dL/d mu_2D of this view (pixels), the densification statistic
    return grads
