"""FP64 band-limited angular-spectrum propagation (Eqs. 7, 14, 16).

  u = crop_{H x W}( IDFT2( H_z . DFT2( pad_{pH x pW}(U) ) ) )

DFT2 is the unnormalised forward transform with kernel exp(-2 pi i k n / N),
IDFT2 its inverse with 1/N (readings: the paper fixes neither convention; the
plane-wave test pins the sign, the phase after propagation by z being
+2 pi z / lambda).  U is zero-padded at the top-left corner and the first H x W
samples are kept; after a matching crop the pad placement is unobservable.

Transfer function (Eq. 7):
  H_z(fx, fy) = exp(j 2 pi z sqrt(1/lambda^2 - fx^2 - fy^2)) where
  fx^2 + fy^2 <= 1/lambda^2, else 0;
with band mode 2 the band limit of Matsushima and Shimobaba (2009, cited with
Eq. 6) is applied on top: |fx| <= 1/(lambda sqrt((2 dfx z)^2 + 1)),
dfx = 1/(pW pitch), and likewise in y.  fx, fy are the DFT frequencies of the
padded grid, k/(n pitch) with k the signed bin index.

The adjoint of the crop-propagate-pad map is crop(IDFT2(conj(H) DFT2(pad g))),
since the unnormalised DFT's adjoint is N times its inverse; it carries the
loss gradient from u back to U (Supplementary D: dP/dU "via band-limited
propagation").
"""
from __future__ import annotations

import numpy as np


def frequencies(n, pitch):
    return np.fft.fftfreq(n, d=pitch)


def band_mask(pH, pW, pitch, lam, z, mode):
    fy = frequencies(pH, pitch)[:, None]
    fx = frequencies(pW, pitch)[None, :]
    mask = np.ones((pH, pW), bool)
    if mode >= 1:
        mask &= (fx * fx + fy * fy) <= 1.0 / (lam * lam)
    if mode >= 2:
        dfx = 1.0 / (pW * pitch)
        dfy = 1.0 / (pH * pitch)
        fxl = 1.0 / (lam * np.sqrt((2.0 * dfx * z) ** 2 + 1.0))
        fyl = 1.0 / (lam * np.sqrt((2.0 * dfy * z) ** 2 + 1.0))
        mask &= (np.abs(fx) <= fxl) & (np.abs(fy) <= fyl)
    return mask


def transfer_function(pH, pW, pitch, lam, z, mode=2):
    """Modes 1 and 2 cut the bins beyond 1/lambda (Eq. 7).  Mode 0 cuts
    nothing: those bins keep the continuation of Eq. 7 that decays away from
    the source plane, exp(-2 pi |z| sqrt(f^2 - 1/lambda^2)) (reading: the
    paper always band-limits; the decaying branch is taken for either sign of
    z so that backward propagation stays bounded)."""
    fy = frequencies(pH, pitch)[:, None]
    fx = frequencies(pW, pitch)[None, :]
    arg = 1.0 / (lam * lam) - fx * fx - fy * fy
    mask = band_mask(pH, pW, pitch, lam, z, mode) & (arg >= 0.0)
    phase = 2.0 * np.pi * z * np.sqrt(np.where(arg >= 0.0, arg, 0.0))
    H = np.where(mask, np.exp(1j * phase), 0.0)
    if mode == 0:
        H = np.where(arg < 0.0, np.exp(-2.0 * np.pi * abs(z) * np.sqrt(np.where(arg < 0.0, -arg, 0.0))), H)
    return H


def _pad(U, pad):
    H, W = U.shape[-2:]
    P = np.zeros(U.shape[:-2] + (pad * H, pad * W), np.complex128)
    P[..., :H, :W] = U
    return P


def propagate(U, lam, z, pitch, pad=2, mode=2, crop=True, padded_input=False):
    """Propagate U [..., H, W] by distance z (signed).

    With crop=False the full padded result is returned; with padded_input=True
    U is already on the padded grid (used by the round-trip and semigroup pins).
    """
    U = np.asarray(U, np.complex128)
    P = U if padded_input else _pad(U, pad)
    pH, pW = P.shape[-2:]
    Hz = transfer_function(pH, pW, pitch, lam, z, mode)
    out = np.fft.ifft2(Hz * np.fft.fft2(P))
    if crop and not padded_input:
        H, W = U.shape[-2:]
        out = out[..., :H, :W]
    return out


def propagate_adjoint(G, lam, z, pitch, pad=2, mode=2):
    """Adjoint of ``propagate`` (cropped) applied to G [..., H, W]."""
    G = np.asarray(G, np.complex128)
    H, W = G.shape[-2:]
    P = _pad(G, pad)
    Hz = transfer_function(P.shape[-2], P.shape[-1], pitch, lam, z, mode)
    return np.fft.ifft2(np.conj(Hz) * np.fft.fft2(P))[..., :H, :W]
