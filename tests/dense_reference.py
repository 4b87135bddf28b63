"""Dense torch float64 formulation of the hologram map, for the oracle pins.

Every pixel is paired with every Gaussian (no tiles, no per-Gaussian loops):
an all-pairs alpha matrix in depth order, transmittance as an exclusive
cumulative product, the early stop of Algorithm 2 as a mask computed from
that product (a pair is kept while the transmittance in front of it is still
>= T_min, so the Gaussian that crosses T_min is kept), and the angular
spectrum with torch.fft.  The stop mask and the alpha clamp enter as
constants, so autograd differentiates the map with the set of included pairs
held fixed, which is what the analytic backward computes.  Shares no code
with the oracle's compositing and gradient; the single-precision footprint
(depth key and support rectangle) and the transfer function are taken from
the oracle, where they are pinned separately.
"""
import numpy as np
import torch

import oracle
from oracle import binning


def dense_alpha(params, sc, cam, thr):
    """alpha [pixels, Gaussians] in (depth key, index) order, the values
    v = c exp(j phi) [Gaussians, wavelengths] in the same order, and H, W."""
    means, log_scales, quats, opacity, amp, phase = params
    fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam, k_sigma=thr.k_sigma)
    vis = torch.as_tensor(fp["visible"])
    order = np.lexsort((np.arange(sc.n), fp["key"].astype(np.int64)))
    q = quats / torch.linalg.norm(quats, dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)
    S = torch.diag_embed(torch.exp(log_scales))
    RS = R @ S
    Sigma = RS @ RS.transpose(1, 2)
    Wc = torch.as_tensor(np.asarray(cam.R, np.float64))
    tcam = means @ Wc.T + torch.as_tensor(np.asarray(cam.t, np.float64))
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    tx, ty, tz = tcam.unbind(1)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * tx / tz ** 2], -1),
                     torch.stack([zero, fy / tz, -fy * ty / tz ** 2], -1)], 1)
    JW = J @ Wc
    cov = JW @ Sigma @ JW.transpose(1, 2)
    conic = torch.linalg.inv(cov)
    mu = torch.stack([fx * tx / tz + cx, fy * ty / tz + cy], -1)
    H, Wd = cam.height, cam.width
    py, px = torch.meshgrid(torch.arange(H, dtype=torch.float64) + 0.5, torch.arange(Wd, dtype=torch.float64) + 0.5,
                            indexing="ij")
    pix = torch.stack([px.reshape(-1), py.reshape(-1)], -1)
    d = pix[:, None, :] - mu[None]
    power = 0.5 * torch.einsum("pgi,gij,pgj->pg", d, conic, d)
    rect = torch.as_tensor(fp["rect"])
    inrect = ((pix[:, None, 0] >= rect[None, :, 0] + 0.5) & (pix[:, None, 0] <= rect[None, :, 1] + 0.5)
              & (pix[:, None, 1] >= rect[None, :, 2] + 0.5) & (pix[:, None, 1] <= rect[None, :, 3] + 0.5))
    oG = opacity[None] * torch.exp(-power)
    a = torch.where(oG > thr.alpha_max, torch.full_like(oG, thr.alpha_max), oG)
    sup = inrect & vis[None] & (power <= 0.5 * thr.k_sigma ** 2) & (a >= thr.alpha_min)
    a = torch.where(sup, a, torch.zeros_like(a))
    v = torch.polar(amp, phase)
    return a[:, order], v[order], order, H, Wd


def exclusive_transmittance(a):
    """T in front of every pair: prod over earlier pairs of (1 - a)."""
    return torch.cumprod(torch.cat([torch.ones_like(a[:, :1]), 1 - a[:, :-1]], 1), 1)


def stop_mask(a, t_min):
    """Pairs that composite: the transmittance in front is still >= T_min."""
    with torch.no_grad():
        return exclusive_transmittance(a) >= t_min


def composite(a, v, t_min, H, W):
    """U [wavelengths, H, W] of one plane with the early stop."""
    a = torch.where(stop_mask(a, t_min), a, torch.zeros_like(a))
    T = exclusive_transmittance(a)
    return torch.einsum("pg,gl->lp", (a * T).to(v.dtype), v).reshape(-1, H, W)


def asm(U, lam, z, pitch, band_limit):
    """Padded (2x, top-left) propagation by z with the oracle's transfer function."""
    H, W = U.shape
    P = torch.zeros((2 * H, 2 * W), dtype=U.dtype)
    P[:H, :W] = U
    Hz = torch.as_tensor(oracle.transfer_function(2 * H, 2 * W, pitch, lam, z, band_limit))
    return torch.fft.ifft2(Hz * torch.fft.fft2(P))[:H, :W]


def stop_fraction(a, t_min):
    """Fraction of pixels whose walk stops (some pair is cut by the stop)."""
    keep = stop_mask(a, t_min)
    cut = (~keep) & (a > 0)
    return float(cut.any(dim=1).double().mean())
