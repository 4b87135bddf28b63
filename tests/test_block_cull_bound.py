"""The raster kernels skip an 8x8 pixel block for a Gaussian when a lower
bound of its power over the block's pixel centres exceeds the largest power
at which it can support a pixel (min(k^2/2, ln(o / alpha_min))).  The bound
minimises the quadratic form over the box of pixel centres on the box edges
that face the centre.  This checks, in single precision as the kernels
compute it, that the bound never exceeds the power of any pixel of the block
(brute force over every pixel), so that a skipped block never holds a
supported pixel, on random and on needle-thin rotated Gaussians.

Tile binning drops tiles by a related rule, the column span of the ellipse
per tile row (oracle.binning.row_span, which the library reproduces bit for
bit); the same brute force pins it, with tightness and closed-form cases."""
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


def _span_fp(mu, conic, pmax, rect):
    return {"mu": mu.astype(f32), "conic": conic.astype(f32), "pmax": pmax.astype(f32), "rect": rect}


def _row_bands(rect, tile_h):
    """(Gaussian, tile row) pairs of the rectangles: index, row, band rows."""
    gi, ty = [], []
    for i, (c0, c1, r0, r1) in enumerate(rect):
        for t in range(r0 // tile_h, r1 // tile_h + 1):
            gi.append(i)
            ty.append(t)
    return np.array(gi), np.array(ty)


def _random_spans(rng, n, aniso):
    A, B, C = _conics(rng, n, aniso)
    conic = np.stack([A, B, C], axis=1)
    mu = np.stack([rng.uniform(-20, 84, size=n), rng.uniform(-20, 84, size=n)], axis=1).astype(f32)
    pmax = rng.uniform(-0.2, 4.5, size=n).astype(f32)
    c0 = rng.integers(0, 24, size=n)
    r0 = rng.integers(0, 24, size=n)
    rect = np.stack([c0, c0 + rng.integers(0, 40, size=n), r0, r0 + rng.integers(0, 40, size=n)], axis=1)
    return _span_fp(mu, conic, pmax, rect)


def test_row_spans_hold_every_supported_pixel():
    """The tile-binning rule (per tile row, the column span of the ellipse
    power <= pmax plus margin) against brute force over every pixel centre:
    a pixel whose exact power is within the per-pixel rounding allowance of
    pmax (1e-4 plus 4e-6 times the form's size over the rectangle) lies in
    its row's span; also for needle-thin Gaussians."""
    from oracle import binning
    rng = np.random.default_rng(11)
    for aniso in (False, True):
        for tile_h in (16, 8):
            fp = _random_spans(rng, 1500, aniso)
            gi, ty = _row_bands(fp["rect"], tile_h)
            lo, hi = binning.row_span(binning.span_geometry(fp, gi), ty, 16, tile_h)
            for k in range(gi.size):
                i = gi[k]
                c0, c1, r0, r1 = fp["rect"][i]
                mx, my = (float(v) for v in fp["mu"][i])
                a, b, c = (float(v) for v in fp["conic"][i])
                xs = np.arange(c0, c1 + 1) + 0.5 - mx
                ys = np.arange(max(ty[k] * tile_h, r0), min(ty[k] * tile_h + tile_h - 1, r1) + 1) + 0.5 - my
                xm = max(-(c0 + 0.5 - mx), c1 + 0.5 - mx)
                ym = max(-(r0 + 0.5 - my), r1 + 0.5 - my)
                mag = 0.5 * (a * xm * xm + c * ym * ym) + abs(b) * xm * ym
                power = 0.5 * (a * xs[None, :] ** 2 + c * ys[:, None] ** 2) + b * xs[None, :] * ys[:, None]
                cols = np.nonzero((power <= float(fp["pmax"][i]) + 1e-4 + 4e-6 * mag).any(axis=0))[0] + c0
                if cols.size:
                    assert lo[k] <= cols.min() and cols.max() <= hi[k], (aniso, tile_h, k)
            assert np.mean(lo > hi) > 0.05      # rows the ellipse misses are dropped


def test_row_spans_are_tight():
    """Each span end is a column whose centre comes within the margin of the
    ellipse over the row's band (exact minimum of the power along the column,
    FP64): the span is no wider than the ellipse plus rounding."""
    from oracle import binning
    rng = np.random.default_rng(12)
    for aniso in (False, True):
        fp = _random_spans(rng, 1500, aniso)
        gi, ty = _row_bands(fp["rect"], 16)
        geo = binning.span_geometry(fp, gi)
        lo, hi = binning.row_span(geo, ty, 16, 16)
        for k in np.nonzero((lo <= hi) & ~geo["full"])[0]:
            i = gi[k]
            c0, c1, r0, r1 = fp["rect"][i]
            mx, my = (float(v) for v in fp["mu"][i])
            a, b, c = (float(v) for v in fp["conic"][i])
            y0 = max(ty[k] * 16, r0) + 0.5 - my
            y1 = min(ty[k] * 16 + 15, r1) + 0.5 - my
            pmax = float(fp["pmax"][i])
            xm = max(-(c0 + 0.5 - mx), c1 + 0.5 - mx)
            ym = max(-(r0 + 0.5 - my), r1 + 0.5 - my)
            mag = 0.5 * (a * xm * xm + c * ym * ym) + abs(b) * xm * ym
            pm = pmax + 1e-4 + 1e-3 * abs(pmax) + 4e-6 * mag
            for col in (lo[k], hi[k]):
                dx = col + 0.5 - mx
                dy = min(max(-b * dx / c, y0), y1)      # minimiser along the column within the band
                pw = 0.5 * (a * dx * dx + c * dy * dy) + b * dx * dy
                assert pw <= pm * (1 + 1e-3) + 1e-3 + 1e-5 * mag, (aniso, k, pw, pm)


def test_row_span_of_a_circle():
    """Unit conic, pmax = 8: the ellipse is the circle of radius 4 around mu.
    Band of centres y - my in [1.5, 2.5]: nearest row at 1.5, half-width
    sqrt(16 - 2.25) = 3.708, so with mu_x = 10.0 the centres 6.29 .. 13.71,
    i.e. pixel columns 6 .. 13 (centres 6.5 .. 13.5)."""
    from oracle import binning
    fp = _span_fp(np.array([[10.0, 0.0]]), np.array([[1.0, 0.0, 1.0]]), np.array([8.0]),
                  np.array([[0, 31, 0, 31]]))
    geo = binning.span_geometry(fp, np.array([0]))
    fp2 = _span_fp(np.array([[10.0, -1.0]]), np.array([[1.0, 0.0, 1.0]]), np.array([8.0]),
                   np.array([[0, 31, 0, 1]]))
    lo, hi = binning.row_span(binning.span_geometry(fp2, np.array([0])), np.array([0]), 16, 16)
    assert (int(lo[0]), int(hi[0])) == (6, 13)
    # the band holding mu's row (dy from 0.5): half-width sqrt(16 - 0.25) = 3.97, columns 6 .. 13
    lo, hi = binning.row_span(geo, np.array([0]), 16, 16)
    assert (int(lo[0]), int(hi[0])) == (6, 13)
    # a tilted needle: conic of a Gaussian stretched along x = y; rows far from
    # mu keep only the columns near the diagonal
    th = np.pi / 4
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    Q = np.linalg.inv(R @ np.diag([20.0 ** 2, 0.5 ** 2]) @ R.T)
    fp3 = _span_fp(np.array([[40.0, 40.0]]), np.array([[Q[0, 0], Q[0, 1], Q[1, 1]]]), np.array([4.5]),
                   np.array([[0, 80, 0, 80]]))
    lo, hi = binning.row_span(binning.span_geometry(fp3, np.array([0])), np.array([1]), 16, 16)
    assert 14 <= lo[0] and hi[0] <= 34          # rows 16..31: the diagonal runs through columns ~16..31


def test_support_power_limit_closed_forms():
    """pmax = min(k^2/2, ln(o / alpha_min)); k^2/2 alone when alpha_min = 0."""
    from oracle import binning
    a = f32(1.0 / 255.0)
    o = np.array([float(a) * np.e ** 2, float(a) * np.e ** 6, float(a) / np.e, 0.0, 0.05], np.float64).astype(f32)
    got = binning.support_power_limit(o, 3.0, 1.0 / 255.0)
    assert abs(float(got[0]) - 2.0) < 1e-6
    assert got[1] == f32(4.5)
    assert abs(float(got[2]) + 1.0) < 1e-6
    assert got[3] == -np.inf
    assert abs(float(got[4]) - np.log(float(f32(0.05)) / float(a))) < 1e-6
    assert np.all(binning.support_power_limit(o, 3.0, 0.0) == f32(4.5))
