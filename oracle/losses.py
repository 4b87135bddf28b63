"""FP64 training losses of the paper (test infrastructure only).

Reconstruction loss (Sec. 4.1, the three-term focal-stack loss):

    L_recon = (1/L) sum_l ( ||I_l - T_l||^2 + ||I_l M_l - T_l M_l||^2
                            + ||I_l T_l - T_l T_l||^2 )

with binary masks M_l of the pixels whose quantised target depth falls on
plane l.  Reading: every squared norm is a mean over its elements (as for the
MSE), and the average runs over views, wavelengths and planes, so with
binary M the loss is the mean of (I - T)^2 (1 + M + T^2).

Structural similarity term:  L_SSIM = lambda_1 (1 - mean SSIM(I_l, T_l)),
lambda_1 = 0.005.  SSIM is the index of Wang et al. (2004): with Gaussian
window averages mu_x = G*x, mu_y = G*y, sigma_x^2 = G*(x^2) - mu_x^2,
sigma_y^2 = G*(y^2) - mu_y^2, sigma_xy = G*(xy) - mu_x mu_y,

    S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) /
        ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),

C1 = 0.01^2, C2 = 0.03^2 (unit dynamic range), an 11 x 11 Gaussian window
with sigma = 1.5, zero padding at the image border (output of the image's
size) and the mean of S over the pixels of each image (readings: the paper
names the fused SSIM of its rasteriser without restating these constants;
they are the standard ones).

Gradients.  With the five window averages as intermediate variables, the
derivative of the mean SSIM w.r.t. x is
    (1/N) [ G*(dS/dmu_x) + 2 x G*(dS/de_xx) + y G*(dS/de_xy) ],
where e_xx = G*(x^2), e_xy = G*(xy) and the window is symmetric, so the
adjoint of the zero-padded filtering is the same filtering.
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5
SSIM_WEIGHT = 0.005


def gaussian_window(size=WINDOW, sigma=SIGMA):
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-r * r / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def filter2(img, win=None):
    """Zero-padded 'same' window average: out[p] = sum_o win[o] img[p + o - c]."""
    win = gaussian_window() if win is None else win
    k = win.shape[0]
    c = k // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * c, W + 2 * c))
    pad[c:c + H, c:c + W] = img
    out = np.zeros((H, W))
    for i in range(k):
        for j in range(k):
            out += win[i, j] * pad[i:i + H, j:j + W]
    return out


def _moments(x, y):
    mx, my = filter2(x), filter2(y)
    exx, eyy, exy = filter2(x * x), filter2(y * y), filter2(x * y)
    return mx, my, exx, eyy, exy


def ssim_map(x, y):
    mx, my, exx, eyy, exy = _moments(np.asarray(x, np.float64), np.asarray(y, np.float64))
    a1 = 2 * mx * my + C1
    a2 = 2 * (exy - mx * my) + C2
    b1 = mx * mx + my * my + C1
    b2 = (exx - mx * mx) + (eyy - my * my) + C2
    return a1 * a2 / (b1 * b2)


def ssim(x, y):
    return float(np.mean(ssim_map(x, y)))


def ssim_grad(x, y):
    """d mean(SSIM(x, y)) / dx for one image."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my, exx, eyy, exy = _moments(x, y)
    a1 = 2 * mx * my + C1
    a2 = 2 * (exy - mx * my) + C2
    b1 = mx * mx + my * my + C1
    b2 = (exx - mx * mx) + (eyy - my * my) + C2
    S = a1 * a2 / (b1 * b2)
    d_mx = (2 * my * a2 - 2 * my * a1) / (b1 * b2) - S * (2 * mx / b1 - 2 * mx / b2)
    d_exx = -S / b2
    d_exy = 2 * a1 / (b1 * b2)
    n = x.size
    return (filter2(d_mx) + 2 * x * filter2(d_exx) + y * filter2(d_exy)) / n


def recon_loss(I, T, M):
    I, T, M = (np.asarray(a, np.float64) for a in (I, T, M))
    return float(np.mean((I - T) ** 2 * (1.0 + M + T * T)))


def recon_grad(I, T, M):
    I, T, M = (np.asarray(a, np.float64) for a in (I, T, M))
    return 2.0 * (I - T) * (1.0 + M + T * T) / I.size


def paper_loss(I, T, M, weight=SSIM_WEIGHT):
    """L_recon + L_SSIM over intensities I, targets T [B, wavelengths, planes, H, W]
    and masks M [B, planes, H, W]; returns (loss, dL/dI)."""
    I = np.asarray(I, np.float64)
    T = np.asarray(T, np.float64)
    Mb = np.broadcast_to(np.asarray(M, np.float64)[:, None], I.shape)
    loss = recon_loss(I, T, Mb)
    grad = recon_grad(I, T, Mb)
    imgs = I.reshape((-1,) + I.shape[-2:])
    tgts = T.reshape((-1,) + T.shape[-2:])
    n_img = imgs.shape[0]
    s = 0.0
    g = np.zeros_like(imgs)
    for i in range(n_img):
        s += ssim(imgs[i], tgts[i])
        g[i] = ssim_grad(imgs[i], tgts[i])
    loss += weight * (1.0 - s / n_img)
    grad += (-weight / n_img) * g.reshape(I.shape)
    return loss, grad


def plane_masks(depth, n_planes, d_min, d_max):
    """Binary masks of a depth map quantised into n_planes equal bins over
    [d_min, d_max] (the target's quantised depth of the recon loss)."""
    q = np.clip(((np.asarray(depth, np.float64) - d_min) / (d_max - d_min) * n_planes).astype(np.int64), 0,
                n_planes - 1)
    return np.stack([(q == l) for l in range(n_planes)], axis=-3).astype(np.uint8)
