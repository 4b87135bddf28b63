"""FP64 optimiser and densification of the training loop (test infrastructure only).

Optimiser (Sec. 5): Adan, the adaptive Nesterov momentum method of Xie et
al., written in the decay-coefficient form (each moment keeps the fraction
b of its previous value).  For a parameter theta with gradient g_k at step
k = 1, 2, ...:

    d_k   = g_k - g_{k-1}                  (d_1 = 0)
    m_k   = b1 m_{k-1} + (1 - b1) g_k
    v_k   = b2 v_{k-1} + (1 - b2) d_k
    n_k   = b3 n_{k-1} + (1 - b3) (g_k + b2 d_k)^2
    theta_k = (theta_{k-1} - lr (m_k / c1 + b2 v_k / c2) / (sqrt(n_k / c3) + eps)) / (1 + lr wd)

with the bias corrections c_i = 1 - b_i^k.  Readings: the paper gives two
coefficients, 0.9 and 0.99, for a method that has three; they are taken as
the decay of the first moment (b1) and of the squared moment (b3), and the
moment of the gradient difference keeps Adan's own default b2 = 0.92.
eps = 1e-8 and no weight decay unless given.

Densification (Supplementary, optimisation and densification algorithm: the
3DGS strategy with phase-preserving perturbations).  Per Gaussian i, a_i is
the sum over the visible views of the training steps since the last
densification of the norm of dL/d mu_2D (the projected mean, in pixels) and
c_i the number of those views.  With s_i the log-scales:

    grow_i  = c_i > 0 and a_i >= tau_grad * c_i    (mean gradient reaches tau_grad)
    big_i   = max_j s_ij > sigma_split             (log of the split scale)
    split_i = grow_i and big_i                     (over-reconstruction)
    clone_i = grow_i and not big_i                 (under-reconstruction)

Outputs in the order of i, each Gaussian giving at most two:
  * not split: the Gaussian itself (kind 0), then, if clone_i, its copy
    (kind 1) whose phases are perturbed, phase + sigma_phi zeta_i0;
  * split: two children (kind 2), c = 0, 1, with
        mean      mu_i + R(q_i) (exp(s_i) * xi_ic)   (a sample of the Gaussian)
        log-scale s_i - shrink                       (shrink = log 1.6: two
                                                      children, each 1/(0.8 * 2))
        phase     phi_i + sigma_phi zeta_ic
    and every other parameter copied.
xi [N, 2, 3] and zeta [N, 2, Lambda] are standard normal draws passed in.
Every candidate is then pruned if its opacity < min_opacity or
max_j s_j > sigma_prune (too large).  Readings: the pruning and splitting
thresholds, the split factor and the 1.6 shrink are the 3DGS ones; the
paper states neither the perturbation law nor its size, so it is a normal
draw with a configurable sigma_phi; the clone keeps the position and the
scale of its source, as in 3DGS.

The grow/split/prune decisions are integers that floating point decides, so
they are taken here in single precision exactly as stated above: fl32(tau_grad
* c) against the fl32 sum, and the fl32 log-scales (fl32(s - shrink) for
split children) against the fl32 thresholds.  The new means, log-scales and
phases themselves are computed in FP64.
"""
from __future__ import annotations

import numpy as np

from .projection import quat_to_rotmat

ADAN_BETAS = (0.9, 0.92, 0.99)
SPLIT_SHRINK = float(np.log(1.6))

KIND_KEPT, KIND_CLONE, KIND_SPLIT = 0, 1, 2


def adan_step(theta, g, state, lr, step, betas=ADAN_BETAS, eps=1e-8, weight_decay=0.0):
    """One Adan update of theta (returned) from gradient g; ``state`` is a dict
    with m, v, n and g_prev (created on the first step) and is updated in place."""
    b1, b2, b3 = betas
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    if step == 1 or "m" not in state:
        state["m"] = np.zeros_like(g)
        state["v"] = np.zeros_like(g)
        state["n"] = np.zeros_like(g)
        state["g_prev"] = g.copy()
    d = g - state["g_prev"]
    state["m"] = b1 * state["m"] + (1 - b1) * g
    state["v"] = b2 * state["v"] + (1 - b2) * d
    state["n"] = b3 * state["n"] + (1 - b3) * (g + b2 * d) ** 2
    state["g_prev"] = g.copy()
    c1, c2, c3 = 1 - b1 ** step, 1 - b2 ** step, 1 - b3 ** step
    upd = (state["m"] / c1 + b2 * state["v"] / c2) / (np.sqrt(state["n"] / c3) + eps)
    return (theta - lr * upd) / (1 + lr * weight_decay)


def accumulate_stats(accum, count, d_mu, visible):
    """Add ||dL/d mu_2D|| of one view to the statistics of its visible Gaussians."""
    accum = accum + np.where(visible, np.linalg.norm(np.asarray(d_mu, np.float64), axis=-1), 0.0)
    count = count + visible.astype(np.float64)
    return accum, count


def densify(means, log_scales, quats, opacity, phase, grad_accum, grad_count, xi, zeta, tau_grad, sigma_split,
            sigma_prune, min_opacity, phase_sigma, shrink=SPLIT_SHRINK):
    """Returns (src, kind, means, log_scales, phase) of the output Gaussians:
    output j comes from input src[j]; kind is KIND_KEPT, KIND_CLONE or
    KIND_SPLIT; the three arrays hold the new values (FP64) of the fields that
    densification changes.  Every other per-Gaussian array is gathered by src."""
    f32 = np.float32
    means = np.asarray(means, np.float64)
    s64 = np.asarray(log_scales, np.float64)
    s32 = np.asarray(log_scales, f32)
    phase = np.asarray(phase, np.float64)
    op32 = np.asarray(opacity, f32)
    a32 = np.asarray(grad_accum, f32)
    c32 = np.asarray(grad_count, f32)
    xi = np.asarray(xi, np.float64)
    zeta = np.asarray(zeta, np.float64)
    R = quat_to_rotmat(np.asarray(quats, np.float64))
    tau32, split32, prune32, minop32, shrink32 = (f32(tau_grad), f32(sigma_split), f32(sigma_prune),
                                                  f32(min_opacity), f32(shrink))
    src, kind, out_m, out_s, out_p = [], [], [], [], []

    def emit(i, k, m, s, p, s_for_test):
        if op32[i] < minop32 or s_for_test.max() > prune32:
            return
        src.append(i)
        kind.append(k)
        out_m.append(m)
        out_s.append(s)
        out_p.append(p)

    for i in range(means.shape[0]):
        grow = c32[i] > 0 and a32[i] >= f32(tau32 * c32[i])
        big = s32[i].max() > split32
        if grow and big:
            child32 = (s32[i] - shrink32).astype(f32)
            for c in range(2):
                m = means[i] + R[i] @ (np.exp(s64[i]) * xi[i, c])
                emit(i, KIND_SPLIT, m, s64[i] - shrink, phase[i] + phase_sigma * zeta[i, c], child32)
            continue
        emit(i, KIND_KEPT, means[i], s64[i], phase[i], s32[i])
        if grow:
            emit(i, KIND_CLONE, means[i], s64[i], phase[i] + phase_sigma * zeta[i, 0], s32[i])
    n_lam = phase.shape[1]
    return (np.asarray(src, np.int64), np.asarray(kind, np.int64), np.asarray(out_m, np.float64).reshape(-1, 3),
            np.asarray(out_s, np.float64).reshape(-1, 3), np.asarray(out_p, np.float64).reshape(-1, n_lam))


def gather_rows(values, src, kind, zero_new):
    """Per-Gaussian array carried through densification: row j is values[src[j]],
    or zero for new Gaussians (kind != KIND_KEPT) when zero_new (optimiser state)."""
    values = np.asarray(values)
    out = values[np.asarray(src, np.int64)].copy()
    if zero_new:
        out[np.asarray(kind) != KIND_KEPT] = 0
    return out


def cosine_lr(step, total, lr0, lr_min):
    """Cosine annealing from lr0 at step 0 to lr_min at step ``total``."""
    t = min(max(step, 0), total) / float(total)
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + np.cos(np.pi * t))
