"""Pins for the training-loss oracle (reconstruction loss with plane masks and
the SSIM term of Sec. 4.1).

* the window average equals scipy's zero-padded correlation with the same
  normalised Gaussian;
* SSIM(x, x) = 1 at every pixel; symmetry; constant images give the
  luminance term (2ab + C1)/(a^2 + b^2 + C1) away from the border;
* SSIM and loss gradients against central differences;
* the reconstruction loss reduces to the MSE for zero masks and zero targets,
  and each extra term doubles or scales it as its closed form says;
* plane masks partition the pixels.
"""
import numpy as np
import scipy.ndimage as ndi

from oracle import losses


def test_window_average_is_zero_padded_gaussian_correlation():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(23, 31))
    w = losses.gaussian_window()
    assert np.isclose(w.sum(), 1.0) and w.shape == (11, 11)
    assert np.isclose(w[5, 5] / w[5, 6], np.exp(1.0 / (2 * 1.5 ** 2)))
    ref = ndi.correlate(x, w, mode="constant", cval=0.0)
    assert np.allclose(losses.filter2(x), ref, rtol=0, atol=1e-14)


def test_ssim_identity_symmetry_and_constant_images():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(20, 24))
    y = rng.uniform(size=(20, 24))
    assert np.allclose(losses.ssim_map(x, x), 1.0, atol=1e-12)
    assert np.isclose(losses.ssim(x, y), losses.ssim(y, x), rtol=0, atol=1e-14)
    assert losses.ssim(x, y) < 0.5
    a, b = 0.3, 0.7
    S = losses.ssim_map(np.full((30, 30), a), np.full((30, 30), b))
    inner = S[5:-5, 5:-5]
    assert np.allclose(inner, (2 * a * b + losses.C1) / (a * a + b * b + losses.C1), rtol=1e-12)


def test_ssim_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(13, 15))
    y = rng.uniform(size=(13, 15))
    g = losses.ssim_grad(x, y)
    h = 1e-6
    for (r, c) in [(0, 0), (6, 7), (12, 14), (3, 11), (9, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[r, c] += h
        xm[r, c] -= h
        fd = (losses.ssim(xp, y) - losses.ssim(xm, y)) / (2 * h)
        assert abs(fd - g[r, c]) < 1e-7 * max(1.0, abs(fd)) + 1e-9, (r, c, fd, g[r, c])


def test_recon_loss_closed_forms_and_gradient():
    rng = np.random.default_rng(3)
    I = rng.uniform(size=(2, 3, 8, 9))
    T = rng.uniform(size=I.shape)
    zero = np.zeros_like(I)
    assert np.isclose(losses.recon_loss(I, zero, zero), np.mean(I ** 2))
    ones = np.ones_like(I)
    # mask everywhere doubles the first term; unit targets add a third copy of it
    assert np.isclose(losses.recon_loss(I, zero, ones), 2 * np.mean(I ** 2))
    assert np.isclose(losses.recon_loss(I, ones, zero), 2 * np.mean((I - 1) ** 2))
    M = (rng.uniform(size=I.shape) < 0.4).astype(float)
    g = losses.recon_grad(I, T, M)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 7, 8), (0, 1, 3, 4)]:
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += h
        Im[idx] -= h
        fd = (losses.recon_loss(Ip, T, M) - losses.recon_loss(Im, T, M)) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8, idx


def test_paper_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    I = rng.uniform(size=(1, 2, 2, 12, 13))
    T = rng.uniform(size=I.shape)
    M = (rng.uniform(size=(1, 2, 12, 13)) < 0.5).astype(np.uint8)
    loss, g = losses.paper_loss(I, T, M)
    h = 1e-6
    for idx in [(0, 0, 0, 0, 0), (0, 1, 1, 6, 6), (0, 0, 1, 11, 12), (0, 1, 0, 2, 9)]:
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += h
        Im[idx] -= h
        fd = (losses.paper_loss(Ip, T, M)[0] - losses.paper_loss(Im, T, M)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8, (idx, fd, g[idx])
    # the SSIM term is active: weight 0 changes the loss
    assert losses.paper_loss(I, T, M, weight=0.0)[0] < loss


def test_plane_masks_partition_pixels():
    rng = np.random.default_rng(5)
    depth = rng.uniform(1.0, 3.0, size=(2, 10, 12))
    m = losses.plane_masks(depth, 4, 1.0, 3.0)
    assert m.shape == (2, 4, 10, 12) and m.dtype == np.uint8
    assert np.array_equal(m.sum(axis=1), np.ones((2, 10, 12)))
    lay = np.argmax(m, axis=1)
    assert np.array_equal(lay, np.clip(((depth - 1.0) / 2.0 * 4).astype(int), 0, 3))
