"""The raster kernels skip an 8x8 pixel block for a Gaussian when a lower
bound of its power over the block's pixel centres exceeds the largest power
at which it can support a pixel (min(k^2/2, ln(o / alpha_min))).  The bound
minimises the quadratic form over the box of pixel centres on the box edges
that face the centre.  This checks, in single precision as the kernels
compute it, that the bound never exceeds the power of any pixel of the block
(brute force over every pixel), so that a skipped block never holds a
supported pixel, on random and on needle-thin rotated Gaussians."""
import numpy as np

f32 = np.float32


def block_bound(mx, my, A, B, C, xlo, xhi, ylo, yhi):
    """Single-precision lower bound of power = 0.5 (A dx^2 + C dy^2) + B dx dy
    over pixel centres x in [xlo, xhi] + 0.5, y in [ylo, yhi] + 0.5, and the
    rounding margin's magnitude term (as in the raster kernels)."""
    x0, x1 = f32(f32(xlo) + f32(0.5)) - mx, f32(f32(xhi) + f32(0.5)) - mx
    y0, y1 = f32(f32(ylo) + f32(0.5)) - my, f32(f32(yhi) + f32(0.5)) - my
    xin, yin = (x0 <= 0) & (x1 >= 0), (y0 <= 0) & (y1 >= 0)
    xe = np.where(x0 > 0, x0, x1)
    ys = np.minimum(np.maximum(-B * xe * (f32(1) / C), y0), y1)
    qx = f32(0.5) * (A * xe * xe + C * ys * ys) + B * xe * ys
    ye = np.where(y0 > 0, y0, y1)
    xs = np.minimum(np.maximum(-B * ye * (f32(1) / A), x0), x1)
    qy = f32(0.5) * (A * xs * xs + C * ye * ye) + B * xs * ye
    lb = np.where(xin, np.where(yin, f32(0), qy), np.where(yin, qx, np.minimum(qx, qy)))
    xm, ym = np.maximum(-x0, x1), np.maximum(-y0, y1)
    mag = f32(0.5) * (A * xm * xm + C * ym * ym) + np.abs(B) * xm * ym
    return lb.astype(f32), mag.astype(f32)


def _conics(rng, n, aniso):
    sig = np.exp(rng.normal(1.5, 1.0, size=(n, 2)))
    if aniso:
        sig[:, 1] = sig[:, 0] * rng.uniform(1e-3, 2e-2, size=n)   # needles
    th = rng.uniform(0, np.pi, size=n)
    c, s = np.cos(th), np.sin(th)
    cov = np.empty((n, 2, 2))
    cov[:, 0, 0] = c * c * sig[:, 0] ** 2 + s * s * sig[:, 1] ** 2
    cov[:, 1, 1] = s * s * sig[:, 0] ** 2 + c * c * sig[:, 1] ** 2
    cov[:, 0, 1] = cov[:, 1, 0] = c * s * (sig[:, 0] ** 2 - sig[:, 1] ** 2)
    Q = np.linalg.inv(cov)
    return Q[:, 0, 0].astype(f32), Q[:, 0, 1].astype(f32), Q[:, 1, 1].astype(f32)


def test_block_bound_never_exceeds_any_pixel_power():
    rng = np.random.default_rng(7)
    for aniso in (False, True):
        n = 4000
        A, B, C = _conics(rng, n, aniso)
        mx = rng.uniform(-20, 28, size=n).astype(f32)
        my = rng.uniform(-20, 28, size=n).astype(f32)
        # the block [0, 7]^2 clipped by a random support rectangle
        xlo = rng.integers(0, 4, size=n)
        xhi = np.maximum(xlo, rng.integers(3, 8, size=n))
        ylo = rng.integers(0, 4, size=n)
        yhi = np.maximum(ylo, rng.integers(3, 8, size=n))
        lb, mag = block_bound(mx, my, A, B, C, xlo, xhi, ylo, yhi)
        worst = np.inf
        for i in range(n):
            px = np.arange(xlo[i], xhi[i] + 1, dtype=f32) + f32(0.5)
            py = np.arange(ylo[i], yhi[i] + 1, dtype=f32) + f32(0.5)
            dx = (px[None, :] - mx[i]).astype(f32)
            dy = (py[:, None] - my[i]).astype(f32)
            power = f32(0.5) * (A[i] * dx * dx + C[i] * dy * dy) + B[i] * dx * dy   # the kernels' formula
            slack = (power.min() + f32(1e-4) + f32(4e-6) * mag[i]) - lb[i]
            worst = min(worst, float(slack))
        assert worst >= 0.0, f"bound above a pixel's power (aniso={aniso}): slack {worst}"


def test_block_bound_is_tight_when_the_centre_is_outside():
    """The bound is the exact minimum for an isotropic Gaussian: the distance
    to the nearest pixel centre (so that the cull is useful, not only safe)."""
    A = C = np.array([1.0], f32)
    B = np.array([0.0], f32)
    lb, _ = block_bound(np.array([-3.0], f32), np.array([4.0], f32), A, B, C, 0, 7, 0, 7)
    assert abs(float(lb[0]) - 0.5 * 3.5 ** 2) < 1e-5
    lb, _ = block_bound(np.array([-3.0], f32), np.array([-4.0], f32), A, B, C, 0, 7, 0, 7)
    assert abs(float(lb[0]) - 0.5 * (3.5 ** 2 + 4.5 ** 2)) < 1e-5
