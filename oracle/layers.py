"""FP64 multi-layer hologram: hard plane assignment, per-layer compositing,
forward recording and inverse propagation (test infrastructure only).

Layer construction (Sec. 4.1, Eqs. 11-13, and the per-layer transmittance
of Supplementary D).  Every Gaussian n carries layer logits rho'_n, one per
layer.  The forward pass uses the hard assignment

    rho_n = OneHot(argmax_l rho'_n)                                  (Eq. 12)

(ties go to the lowest layer index; reading).  Layer l composites, front to
back in the global depth order, only what is assigned to it, with its own
transmittance T_l = prod over earlier j of (1 - rho_{j,l} a_j):

    U_l += rho_{n,l} v_n a_n T_l,     T_l <- T_l (1 - rho_{n,l} a_n)  (Eq. 13)

Reading of the early termination of Algorithm 2 for several layers: the test
T < T_min is applied to each layer's own transmittance; after the Gaussian
that brings T_l below T_min (that Gaussian included) layer l takes no more
contributions.  ``render_layers`` accepts any weight matrix rho [N, layers]
(the finite-difference pins perturb it off the one-hot point).

Forward recording and inverse propagation (Eqs. 14-16): for each wavelength
the layer fields are propagated to the hologram plane and summed,
P = sum_l ASM(U_l; +Z_l), and P is propagated back to every layer,
u_k = ASM(P; -Z_k), I_k = |u_k|^2.  ASM is ``asm.propagate`` (pad, transfer
function, crop to the layer grid).

Backward.  Per layer the reverse-order replay of raster.py with that layer's
T (taken, as in raster.py, from a forward replay that keeps the transmittance
in front of every Gaussian), accumulated field B_l and loss gradient G_l.
With w = rho_{n,l} and T_l the transmittance of layer l in front of n,

    dL/drho_{n,l} = a_n T_l sum_lambda Re(conj(G_l) (v_n - B_l))

for every layer l that had not terminated before n: for the Gaussian's own
layer this is a_n dL/da_n; for the other layers (w = 0) it is the derivative
of inserting n into layer l, whose T_l and B_l are then unchanged by n.  The
straight-through estimator (Eq. 12, backward) gives
dL/drho'_{n,l} = dL/drho_{n,l} softmax(rho'_n / tau)_l with tau = 1e-3
(reading: the product is elementwise).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .asm import propagate, propagate_adjoint
from .binning import fp32_footprint
from .pipeline import DEFAULT, mse_loss
from .projection import project, project_backward
from .raster import _support, depth_order

STE_TAU = 1e-3
NEVER = np.iinfo(np.int64).max


def hard_assignment(logits):
    """Eq. 12: one-hot of the argmax of each Gaussian's layer logits."""
    logits = np.asarray(logits, np.float64)
    w = np.zeros_like(logits)
    w[np.arange(logits.shape[0]), np.argmax(logits, axis=1)] = 1.0
    return w


def ste_softmax(logits, tau=STE_TAU):
    """softmax(rho' / tau) per Gaussian, the surrogate gradient weight of Eq. 12."""
    x = np.asarray(logits, np.float64) / tau
    x = x - x.max(axis=1, keepdims=True)
    e = np.exp(x)
    return e / e.sum(axis=1, keepdims=True)


@dataclass
class LayerRaster:
    U: np.ndarray        # [layers, wavelengths, H, W] complex128
    T_final: np.ndarray  # [layers, H, W]
    stop: np.ndarray     # [layers, H, W] order position where the layer terminated, NEVER if it did not
    order: np.ndarray    # visible Gaussians by (depth key, index)


def render_layers(proj, opacity, footprint, weights, width, height, thr=DEFAULT, window=None) -> LayerRaster:
    """Eq. 13 for every layer at once; ``weights`` [N, layers] (one-hot in the
    method, continuous in the finite-difference pins)."""
    w_all = np.asarray(weights, np.float64)
    nl = w_all.shape[1]
    lam = proj.v.shape[1]
    U = np.zeros((nl, lam, height, width), np.complex128)
    T = np.ones((nl, height, width))
    stop = np.full((nl, height, width), NEVER, np.int64)
    order = depth_order(footprint)
    for pos, g in enumerate(order):
        sp = _support(g, proj, opacity, footprint["rect"], thr, window)
        if sp is None:
            continue
        sl, _, _, _, _, a, _, sup = sp
        for l in range(nl):
            w = w_all[g, l]
            if w == 0.0:
                continue
            inc = sup & (stop[l][sl] == NEVER)
            if not inc.any():
                continue
            Tl = T[l][sl]
            U[(l, slice(None)) + sl] += proj.v[g][:, None, None] * np.where(inc, w * a * Tl, 0.0)[None]
            Tn = np.where(inc, Tl * (1.0 - w * a), Tl)
            T[l][sl] = Tn
            stop[l][sl] = np.where(inc & (Tn < thr.t_min), pos, stop[l][sl])
    return LayerRaster(U, T, stop, order)


def layer_transmittance_in_front(proj, opacity, footprint, weights, res: LayerRaster, thr=DEFAULT, window=None):
    """Per layer, the transmittance in front of every Gaussian over its support
    rectangle, by replaying each layer's front-to-back product up to the
    position where the layer stopped: {order position: [layers, rows, cols]}."""
    w_all = np.asarray(weights, np.float64)
    nl = w_all.shape[1]
    T = np.ones_like(res.T_final)
    out = {}
    for pos, g in enumerate(res.order):
        sp = _support(g, proj, opacity, footprint["rect"], thr, window)
        if sp is None:
            continue
        sl, _, _, _, _, a, _, sup = sp
        out[pos] = np.stack([T[l][sl] for l in range(nl)])
        for l in range(nl):
            live = sup & (pos <= res.stop[l][sl])
            T[l][sl] = np.where(live, T[l][sl] * (1.0 - w_all[g, l] * a), T[l][sl])
    return out


def render_layers_backward(proj, opacity, footprint, weights, res: LayerRaster, G_layers, thr=DEFAULT,
                           window=None):
    """Reverse replay of every layer.  G_layers [layers, wavelengths, H, W]
    complex (dL/dRe + j dL/dIm).  Returns d_mu [N,2], d_conic [N,3],
    d_opacity [N], d_v [N,wavelengths] complex and d_rho [N, layers]."""
    w_all = np.asarray(weights, np.float64)
    N, lam = proj.v.shape
    nl = w_all.shape[1]
    d_mu = np.zeros((N, 2))
    d_conic = np.zeros((N, 3))
    d_op = np.zeros(N)
    d_v = np.zeros((N, lam), np.complex128)
    d_rho = np.zeros((N, nl))
    T_front = layer_transmittance_in_front(proj, opacity, footprint, w_all, res, thr, window)
    Bacc = np.zeros((nl, lam) + res.T_final.shape[1:], np.complex128)
    for pos in range(len(res.order) - 1, -1, -1):
        g = res.order[pos]
        sp = _support(g, proj, opacity, footprint["rect"], thr, window)
        if sp is None:
            continue
        sl, dx, dy, power, G, a, clamped, sup = sp
        v = proj.v[g][:, None, None]
        dLda = np.zeros(a.shape)
        for l in range(nl):
            live = sup & (pos <= res.stop[l][sl])
            if not live.any():
                continue
            w = w_all[g, l]
            Tb = np.where(live, T_front[pos][l], 0.0)
            Gs = G_layers[(l, slice(None)) + sl]
            Bs = Bacc[(l, slice(None)) + sl]
            s = np.where(live, Tb * np.sum((np.conj(Gs) * (v - Bs)).real, axis=0), 0.0)
            d_rho[g, l] += np.sum(a * s)
            dLda += w * s
            d_v[g] += np.sum(np.where(live[None], w * a * Tb * Gs, 0.0), axis=(1, 2))
            Bacc[(l, slice(None)) + sl] = np.where(live[None], w * a * v + (1.0 - w * a) * Bs, Bs)
        free = sup & ~clamped
        d_op[g] += np.sum(np.where(free, G * dLda, 0.0))
        dpow = np.where(free, -a * dLda, 0.0)
        A, B, C = proj.conic[g]
        d_conic[g, 0] += np.sum(0.5 * dx * dx * dpow)
        d_conic[g, 1] += np.sum(dx * dy * dpow)
        d_conic[g, 2] += np.sum(0.5 * dy * dy * dpow)
        d_mu[g, 0] += np.sum(-(A * dx + B * dy) * dpow)
        d_mu[g, 1] += np.sum(-(B * dx + C * dy) * dpow)
    return d_mu, d_conic, d_op, d_v, d_rho


def record(U_layers, lam, distances, pitch, pad=2, mode=2):
    """Forward recording (Eqs. 14-15): P = sum_l ASM(U_l; +Z_l)."""
    return sum(propagate(U_layers[l], lam, z, pitch, pad, mode) for l, z in enumerate(distances))


def forward_layers(scene, logits, cameras, optics, thr=DEFAULT, targets=None, weights=None):
    """Multi-layer forward for every view.  ``optics.distances`` are the layer
    distances Z_l (layer l to the hologram plane); the intensities are those
    of the inverse propagation to every layer, I [B, wavelengths, layers, H, W]."""
    w = hard_assignment(logits) if weights is None else np.asarray(weights, np.float64)
    B, L, K = len(cameras), scene.n_lambda, len(optics.distances)
    assert w.shape == (scene.n, K)
    H, W = cameras[0].height, cameras[0].width
    u = np.zeros((B, L, K, H, W), np.complex128)
    P = np.zeros((B, L, H, W), np.complex128)
    views = []
    for b, cam in enumerate(cameras):
        proj = project(scene.means, scene.log_scales, scene.quats, scene.amp, scene.phase, cam)
        fp = fp32_footprint(scene.means, scene.log_scales, scene.quats, cam, 16, 16, thr.k_sigma, scene.opacity,
                            thr.alpha_min)
        res = render_layers(proj, scene.opacity, fp, w, W, H, thr)
        for li, lam in enumerate(optics.wavelengths):
            P[b, li] = record(res.U[:, li], lam, optics.distances, optics.pitch, optics.pad, optics.band_limit)
            for k, z in enumerate(optics.distances):
                u[b, li, k] = propagate(P[b, li], lam, -z, optics.pitch, optics.pad, optics.band_limit)
        views.append({"proj": proj, "fp": fp, "res": res, "cam": cam})
    I = np.abs(u) ** 2
    out = {"views": views, "u": u, "I": I, "P": P, "weights": w, "logits": np.asarray(logits, np.float64),
           "scene": scene, "optics": optics, "thr": thr}
    if targets is not None:
        out["loss"] = mse_loss(I, targets)
        out["targets"] = np.asarray(targets, np.float64)
    return out


def backward_layers(state, dL_dI=None):
    """Gradients w.r.t. the scene parameters, the continuous weights rho
    ("rho") and, through the straight-through estimator, the logits."""
    scene, optics, thr, w = state["scene"], state["optics"], state["thr"], state["weights"]
    u, I = state["u"], state["I"]
    if dL_dI is None:
        dL_dI = 2.0 * (I - state["targets"]) / I.size
    G_u = 2.0 * u * dL_dI
    names = ("means", "log_scales", "quats", "opacity", "amp", "phase")
    grads = {k: np.zeros(a.shape, np.float64) for k, a in zip(names, scene.arrays())}
    d_rho = np.zeros(w.shape)
    for b, view in enumerate(state["views"]):
        res = view["res"]
        G_layers = np.zeros_like(res.U)
        for li, lam in enumerate(optics.wavelengths):
            G_P = sum(propagate_adjoint(G_u[b, li, k], lam, -z, optics.pitch, optics.pad, optics.band_limit)
                      for k, z in enumerate(optics.distances))
            for l, z in enumerate(optics.distances):
                G_layers[l, li] = propagate_adjoint(G_P, lam, z, optics.pitch, optics.pad, optics.band_limit)
        d_mu, d_conic, d_op, d_v, d_r = render_layers_backward(view["proj"], scene.opacity, view["fp"], w, res,
                                                                G_layers, thr)
        g = project_backward(view["proj"], scene.quats, scene.amp, scene.phase, view["cam"], d_mu, d_conic, d_op,
                             d_v)
        vis = view["fp"]["visible"]
        for k in grads:
            m = vis.reshape((-1,) + (1,) * (g[k].ndim - 1))
            grads[k] += np.where(m, np.nan_to_num(g[k]), 0.0)
        d_rho += d_r
        view["G_layers"] = G_layers
    grads["rho"] = d_rho
    grads["logits"] = d_rho * ste_softmax(state["logits"])
    return grads
