"""FP64 front-to-back complex compositing and its reverse-order backward.

Forward (Algorithm 2 with one plane, rho = 1; Supplementary D forward pass):
for every pixel p the supported Gaussians are taken in ascending
(depth key, index) order and

    a_g   = min(alpha_max, o_g exp(-power_g(p))),   power = 0.5 d^T conic d
    U_l  += v_{g,l} a_g T,     T <- T (1 - a_g)

with T = 1 at the start; the pixel stops after the Gaussian that brings T below
T_min (that Gaussian is included).  A Gaussian supports p iff p lies in its
single-precision support rectangle, power <= k^2/2 and a_g >= alpha_min.
Depth order is front to back: the loop starts at T = 1 and terminates early,
so the "back-to-front" wording of the algorithm's comments is read as the
order of the backward replay (reading listed in the design notes).

The loop over pixels is vectorised per Gaussian over its rectangle; visiting
Gaussians in the global sorted order gives every pixel the same sequence as a
per-pixel loop.

Backward (Supplementary D backward pass and Sec. 4.2): reverse order from each
pixel's last contributor.  T_g, the transmittance in front of g, is taken from
a forward replay that keeps it for every included (pixel, Gaussian) pair (the
GPU recovers it by dividing by 1 - a_g instead; the oracle does not mirror
that), and with B the field accumulated behind g,

    dL/da_g = T_g * sum_l Re(conj(G_l) (v_{g,l} - B_l)),
    B_l    <- a_g v_{g,l} + (1 - a_g) B_l,
    dL/dv  += a_g T_g G_l,   dL/do += exp(-power) dL/da,  dL/dpower = -a dL/da

(the last two only where a is not clamped at alpha_max).  G is the gradient of
the loss w.r.t. the field in the convention dL/dRe + j dL/dIm.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class RasterResult:
    U: np.ndarray          # [L,H,W] complex128
    T_final: np.ndarray    # [H,W]
    last: np.ndarray       # [H,W] position in ``order`` of the last included Gaussian, -1 if none
    order: np.ndarray      # visible Gaussian indices sorted by (depth key, index)
    n_contrib: np.ndarray  # [H,W] number of included Gaussians


def _support(g, proj, opacity, rect, thr, window=None):
    c0, c1, r0, r1 = (int(v) for v in rect[g])
    if window is not None:   # restrict the pixel loop to rows [wr0, wr1) x columns [wc0, wc1)
        wr0, wr1, wc0, wc1 = window
        c0, c1, r0, r1 = max(c0, wc0), min(c1, wc1 - 1), max(r0, wr0), min(r1, wr1 - 1)
        if c0 > c1 or r0 > r1:
            return None
    px = np.arange(c0, c1 + 1, dtype=np.float64) + 0.5
    py = np.arange(r0, r1 + 1, dtype=np.float64) + 0.5
    dx = px[None, :] - proj.mu[g, 0]
    dy = py[:, None] - proj.mu[g, 1]
    A, B, C = proj.conic[g]
    power = 0.5 * (A * dx * dx + 2.0 * B * dx * dy + C * dy * dy)
    G = np.exp(-power)
    oG = float(opacity[g]) * G
    clamped = oG > thr.alpha_max
    a = np.where(clamped, thr.alpha_max, oG)
    sup = (power <= 0.5 * thr.k_sigma ** 2) & (a >= thr.alpha_min)
    return (slice(r0, r1 + 1), slice(c0, c1 + 1)), dx, dy, power, G, a, clamped, sup


def depth_order(footprint):
    vis = np.nonzero(footprint["visible"])[0]
    keys = footprint["key"][vis].astype(np.int64)
    return vis[np.lexsort((vis, keys))]


def render_field(proj, opacity, footprint, width, height, thr, window=None) -> RasterResult:
    """Composite every pixel (or only those in ``window`` = (r0, r1, c0, c1),
    half-open, the rest staying at U = 0, T = 1)."""
    L = proj.v.shape[1]
    U = np.zeros((L, height, width), np.complex128)
    T = np.ones((height, width))
    active = np.ones((height, width), bool)
    last = np.full((height, width), -1, np.int64)
    ncon = np.zeros((height, width), np.int64)
    order = depth_order(footprint)
    rect = footprint["rect"]
    for pos, g in enumerate(order):
        sp = _support(g, proj, opacity, rect, thr, window)
        if sp is None:
            continue
        sl, _, _, _, _, a, _, sup = sp
        inc = sup & active[sl]
        if not inc.any():
            continue
        Tl = T[sl]
        w = np.where(inc, a * Tl, 0.0)
        U[(slice(None),) + sl] += proj.v[g][:, None, None] * w[None]
        Tn = np.where(inc, Tl * (1.0 - a), Tl)
        T[sl] = Tn
        last[sl] = np.where(inc, pos, last[sl])
        ncon[sl] += inc
        active[sl] &= ~(inc & (Tn < thr.t_min))
    return RasterResult(U, T, last, order, ncon)


def transmittance_in_front(proj, opacity, footprint, res: RasterResult, thr, window=None):
    """T in front of every included (pixel, Gaussian) pair, by replaying the
    front-to-back product: {order position: T over that Gaussian's support
    rectangle (clipped to ``window``), meaningful where it was included}."""
    T = np.ones_like(res.T_final)
    out = {}
    for pos, g in enumerate(res.order):
        sp = _support(g, proj, opacity, footprint["rect"], thr, window)
        if sp is None:
            continue
        sl, _, _, _, _, a, _, sup = sp
        inc = sup & (pos <= res.last[sl])
        if not inc.any():
            continue
        out[pos] = T[sl].copy()
        T[sl] = np.where(inc, T[sl] * (1.0 - a), T[sl])
    return out


def render_field_backward(proj, opacity, footprint, res: RasterResult, G_U, thr, window=None):
    """Per-Gaussian 2D gradients for one view (over ``window`` only, if given).

    G_U: [L,H,W] complex gradient of the loss w.r.t. the rendered field.
    Returns d_mu [N,2], d_conic [N,3], d_opacity [N], d_v [N,L] complex.
    """
    N, L = proj.v.shape
    d_mu = np.zeros((N, 2))
    d_conic = np.zeros((N, 3))
    d_op = np.zeros(N)
    d_v = np.zeros((N, L), np.complex128)
    Bacc = np.zeros_like(G_U)
    rect = footprint["rect"]
    T_front = transmittance_in_front(proj, opacity, footprint, res, thr, window)
    for pos in range(len(res.order) - 1, -1, -1):
        g = res.order[pos]
        sp = _support(g, proj, opacity, rect, thr, window)
        if sp is None:
            continue
        sl, dx, dy, power, G, a, clamped, sup = sp
        # included: supported and not behind the pixel's last contributor
        # (the Gaussian that crossed T_min is itself included)
        inc = sup & (pos <= res.last[sl])
        if not inc.any():
            continue
        Tg = np.where(inc, T_front[pos], 0.0)
        Gs = G_U[(slice(None),) + sl]
        Bs = Bacc[(slice(None),) + sl]
        v = proj.v[g][:, None, None]
        dLda = np.where(inc, Tg * np.sum((np.conj(Gs) * (v - Bs)).real, axis=0), 0.0)
        d_v[g] += np.sum(np.where(inc[None], a * Tg * Gs, 0.0), axis=(1, 2))
        Bacc[(slice(None),) + sl] = np.where(inc[None], a * v + (1.0 - a) * Bs, Bs)
        free = inc & ~clamped
        d_op[g] += np.sum(np.where(free, G * dLda, 0.0))
        dpow = np.where(free, -a * dLda, 0.0)
        A, B, C = proj.conic[g]
        d_conic[g, 0] += np.sum(0.5 * dx * dx * dpow)
        d_conic[g, 1] += np.sum(dx * dy * dpow)
        d_conic[g, 2] += np.sum(0.5 * dy * dy * dpow)
        d_mu[g, 0] += np.sum(-(A * dx + B * dy) * dpow)
        d_mu[g, 1] += np.sum(-(B * dx + C * dy) * dpow)
    return d_mu, d_conic, d_op, d_v
