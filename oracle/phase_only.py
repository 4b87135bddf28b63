"""FP64 phase-only hologram conversion (test infrastructure only).

The displayable hologram of a phase-only modulator is P_phi = exp(j phi)
(the paper's phase-only conversion: propagate the complex hologram P and
P_phi to the same depth layers and match them):

    U_l = ASM(P; -Z_l),   V_l = ASM(exp(j phi); -Z_l),
    L   = mean |U_l - V_l|^2 + w (1 - SSIM_c(U_l, V_l)),   w = 0.005.

Readings: the squared norm is a mean over all elements (views, wavelengths,
layers, pixels), as for the other losses; the paper states that the real
and imaginary components are compared, so SSIM_c of two complex fields is
the mean of SSIM over their real parts and over their imaginary parts (each
SSIM as in ``losses.py``), averaged over views, wavelengths and layers.

Gradient.  With G_l = dL/dRe V_l + j dL/dIm V_l,
G_P = sum_l ASM^H(G_l; -Z_l) is the gradient w.r.t. P_phi and, since
dP_phi/dphi = j P_phi, dL/dphi = Im(G_P exp(-j phi)).
"""
from __future__ import annotations

import numpy as np

from .asm import propagate, propagate_adjoint
from .losses import SSIM_WEIGHT, ssim, ssim_grad


def layer_fields(P, wavelengths, distances, pitch, pad=2, mode=2):
    """ASM(P; -Z_l) for P [B, wavelengths, H, W] -> [B, wavelengths, layers, H, W]."""
    P = np.asarray(P, np.complex128)
    B, L, H, W = P.shape
    out = np.zeros((B, L, len(distances), H, W), np.complex128)
    for b in range(B):
        for li, lam in enumerate(wavelengths):
            for k, z in enumerate(distances):
                out[b, li, k] = propagate(P[b, li], lam, -z, pitch, pad, mode)
    return out


def phase_only_loss(targets, phi, wavelengths, distances, pitch, pad=2, mode=2, weight=SSIM_WEIGHT):
    """Loss and dL/dphi for targets U = layer_fields(P) and phases phi [B, wavelengths, H, W]."""
    phi = np.asarray(phi, np.float64)
    V = layer_fields(np.exp(1j * phi), wavelengths, distances, pitch, pad, mode)
    U = np.asarray(targets, np.complex128)
    n = U.size
    D = V - U
    loss = float(np.mean(np.abs(D) ** 2))
    G = 2.0 * D / n
    flatU = U.reshape((-1,) + U.shape[-2:])
    flatV = V.reshape((-1,) + V.shape[-2:])
    Gs = np.zeros_like(flatV)
    n_img = flatU.shape[0]
    s = 0.0
    for i in range(n_img):
        s += ssim(flatV[i].real, flatU[i].real) + ssim(flatV[i].imag, flatU[i].imag)
        Gs[i] = ssim_grad(flatV[i].real, flatU[i].real) + 1j * ssim_grad(flatV[i].imag, flatU[i].imag)
    loss += weight * (1.0 - s / (2 * n_img))
    G = G - (weight / (2 * n_img)) * Gs.reshape(G.shape)
    B, L = phi.shape[:2]
    dphi = np.zeros_like(phi)
    for b in range(B):
        for li, lam in enumerate(wavelengths):
            GP = sum(propagate_adjoint(G[b, li, k], lam, -z, pitch, pad, mode) for k, z in enumerate(distances))
            dphi[b, li] = np.imag(GP * np.exp(-1j * phi[b, li]))
    return loss, dphi
