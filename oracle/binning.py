"""Single-precision footprint recipe and tile binning (oracle side).

Algorithm 2 culls Gaussians, computes screen-space extents, duplicates each
Gaussian once per covered 16x16 tile with a depth key, sorts, and finds tile
ranges.  The paper fixes neither the precision nor the extent rule, so the
choices below are readings (listed in the design notes):

* the depth key is the camera-space depth in IEEE single precision, computed
  in the fixed order below with round-to-nearest and no fused multiply-add;
* the support rectangle of a Gaussian is its k-sigma axis-aligned box
  (half-extent k*sqrt(Sigma'_xx) + 0.01 px, likewise in y), intersected with
  the pixel centres of the image; a pixel outside it never receives the
  Gaussian, so the field cannot depend on the tile shape;
* a Gaussian is kept iff depth > z_near, det Sigma' > 0, every quantity is
  finite and the rectangle holds at least one pixel centre;
* a kept Gaussian is binned only to the tiles of its rectangle that can hold
  a pixel it supports: power = d^T conic d / 2 <= pmax with
  pmax = min(k^2/2, ln(o / alpha_min)) (o exp(-power) < alpha_min takes the
  pixel out of the support).  Per tile row, the pixel centres of the row's
  band that lie in the ellipse power <= pm form one column interval, found in
  closed form; the row keeps the tiles that interval touches.  pm exceeds
  pmax by a margin that covers rounding, so a dropped tile never holds a
  supported pixel and the field is unchanged.

These are integer decisions taken from floating point, so the oracle takes
them in the same precision as the GPU: every operation below is one float32
operation, in the order written.  The result is compared bit for bit.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def _rot_f32(q):
    qw, qx, qy, qz = (q[:, i] for i in range(4))
    n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz
    n = np.sqrt(n2)
    w, x, y, z = qw / n, qx / n, qy / n, qz / n
    xx, yy, zz = x * x, y * y, z * z
    xy, xz, yz = x * y, x * z, y * z
    wx, wy, wz = w * x, w * y, w * z
    one, two = f32(1.0), f32(2.0)
    R = np.empty((q.shape[0], 3, 3), np.float32)
    R[:, 0, 0] = one - two * (yy + zz)
    R[:, 0, 1] = two * (xy - wz)
    R[:, 0, 2] = two * (xz + wy)
    R[:, 1, 0] = two * (xy + wz)
    R[:, 1, 1] = one - two * (xx + zz)
    R[:, 1, 2] = two * (yz - wx)
    R[:, 2, 0] = two * (xz - wy)
    R[:, 2, 1] = two * (yz + wx)
    R[:, 2, 2] = one - two * (xx + yy)
    return R


def fp32_footprint(means, log_scales, quats, cam, tile_w=16, tile_h=16, k_sigma=3.0, opacity=None,
                   alpha_min=None):
    """Per-Gaussian depth key, visibility, pixel rectangle and tile rectangle.

    Returns a dict of arrays: ``key`` (uint32 bits of the float32 depth),
    ``visible`` (bool), ``rect`` (int64 [N,4] = c0, c1, r0, r1, inclusive pixel
    indices), ``tiles`` (int64 [N,4] = tx0, tx1, ty0, ty1, the tiles the
    rectangle touches) and ``count`` (their number).  With ``opacity`` and
    ``alpha_min`` also the single-precision ``mu`` [N,2], ``conic`` [N,3]
    (A, B, C of power = (A dx^2 + C dy^2) / 2 + B dx dy) and ``pmax`` that
    decide which of those tiles the Gaussian is binned to (``binned_tiles``).
    """
    m = np.asarray(means, np.float32)
    s = np.asarray(log_scales, np.float32)
    q = np.asarray(quats, np.float32)
    Rc = np.asarray(cam.R, np.float32).reshape(3, 3)
    tc = np.asarray(cam.t, np.float32)
    fx, fy, cx, cy = f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy)
    W, H = int(cam.width), int(cam.height)
    k = f32(k_sigma)

    # camera-space centre; the depth key is tcz
    tcam = [((Rc[i, 0] * m[:, 0] + Rc[i, 1] * m[:, 1]) + Rc[i, 2] * m[:, 2]) + tc[i] for i in range(3)]
    tcx, tcy, tcz = tcam
    Rq = _rot_f32(q)
    A = np.empty_like(Rq)
    for i in range(3):
        for j in range(3):
            A[:, i, j] = (Rc[i, 0] * Rq[:, 0, j] + Rc[i, 1] * Rq[:, 1, j]) + Rc[i, 2] * Rq[:, 2, j]
    with np.errstate(all="ignore"):
        ux = tcx / tcz
        uy = tcy / tcz
        gx = fx / tcz
        gy = fy / tcz
        es = np.exp(s.astype(np.float64)).astype(np.float32)
        T0 = [(gx * (A[:, 0, j] - ux * A[:, 2, j])) * es[:, j] for j in range(3)]
        T1 = [(gy * (A[:, 1, j] - uy * A[:, 2, j])) * es[:, j] for j in range(3)]
        sxx = (T0[0] * T0[0] + T0[1] * T0[1]) + T0[2] * T0[2]
        syy = (T1[0] * T1[0] + T1[1] * T1[1]) + T1[2] * T1[2]
        sxy = (T0[0] * T1[0] + T0[1] * T1[1]) + T0[2] * T1[2]
        det = sxx * syy - sxy * sxy
        mux = fx * ux + cx
        muy = fy * uy + cy
        ex = k * np.sqrt(sxx) + f32(0.01)
        ey = k * np.sqrt(syy) + f32(0.01)
        ok = (tcz > f32(cam.z_near)) & (det > f32(0.0))
        ok &= np.isfinite(ex) & np.isfinite(ey) & np.isfinite(mux) & np.isfinite(muy)
        half = f32(0.5)
        xl = np.clip((mux - ex) - half, f32(-1.0), f32(W))
        xh = np.clip((mux + ex) - half, f32(-1.0), f32(W))
        yl = np.clip((muy - ey) - half, f32(-1.0), f32(H))
        yh = np.clip((muy + ey) - half, f32(-1.0), f32(H))
    xl = np.where(ok, xl, 0)
    xh = np.where(ok, xh, 0)
    yl = np.where(ok, yl, 0)
    yh = np.where(ok, yh, 0)
    c0 = np.maximum(np.ceil(xl).astype(np.int64), 0)
    c1 = np.minimum(np.floor(xh).astype(np.int64), W - 1)
    r0 = np.maximum(np.ceil(yl).astype(np.int64), 0)
    r1 = np.minimum(np.floor(yh).astype(np.int64), H - 1)
    visible = ok & (c0 <= c1) & (r0 <= r1)
    rect = np.stack([c0, c1, r0, r1], axis=1)
    tiles = np.stack([c0 // tile_w, c1 // tile_w, r0 // tile_h, r1 // tile_h], axis=1)
    count = np.where(visible, (tiles[:, 1] - tiles[:, 0] + 1) * (tiles[:, 3] - tiles[:, 2] + 1), 0)
    key = np.asarray(tcz, np.float32).view(np.uint32).copy()
    out = {"key": key, "visible": visible, "rect": rect, "tiles": tiles, "count": count}
    if opacity is not None:
        with np.errstate(all="ignore"):
            # the conic is the inverse of the 2D covariance
            out["conic"] = np.stack([syy / det, -sxy / det, sxx / det], axis=1).astype(np.float32)
            out["mu"] = np.stack([mux, muy], axis=1).astype(np.float32)
            out["pmax"] = support_power_limit(opacity, k_sigma, alpha_min)
    return out


def support_power_limit(opacity, k_sigma, alpha_min):
    """Largest power at which a Gaussian can support a pixel, per Gaussian:
    power <= k^2/2, and o exp(-power) >= alpha_min means power <= ln(o /
    alpha_min).  The logarithm is taken in double precision and rounded once
    to single precision; fmin ignores a NaN logarithm."""
    k = f32(k_sigma)
    half_k2 = (f32(0.5) * k) * k
    o = np.asarray(opacity, np.float32)
    a = f32(0.0 if alpha_min is None else alpha_min)
    if not a > 0:
        return np.full(o.shape, half_k2, np.float32)
    with np.errstate(all="ignore"):
        lg = np.log(o.astype(np.float64) / np.float64(a))
    return np.fmin(np.float64(half_k2), lg).astype(np.float32)


def span_geometry(fp, g):
    """Per-Gaussian quantities of the row-span rule for Gaussians ``g``.

    The centres of a tile row's band dy in [y0, y1] that lie in the ellipse
    power <= pm form one interval of dx (the projection of a convex set).
    Its right end is the largest root of power(dx, dy) = pm over the band,
    dx(dy) = (sqrt(2 pm A - D dy^2) - B dy) / A with D = AC - B^2, a concave
    function that peaks at the ellipse's rightmost point dy = -B xr / C,
    xr = sqrt(2 pm C / D); the maximum over the band is at that dy clamped to
    the band (and to the ellipse's height +-ymax, ymax = sqrt(2 pm A / D)).
    The left end mirrors it.  pm = pmax + 1e-4 + 1e-3 |pmax| + 4e-6 mag
    (mag: the size of the form's terms over the rectangle) covers the
    rounding of the per-pixel power and of these steps.  ``none``: no tile;
    ``full``: every tile of the rectangle (a degenerate or non-finite form).
    """
    if "pmax" not in fp:
        raise ValueError("binning needs footprints computed with opacity and alpha_min")
    half, two = f32(0.5), f32(2.0)
    mx, my = fp["mu"][g, 0], fp["mu"][g, 1]
    A, B, C = fp["conic"][g, 0], fp["conic"][g, 1], fp["conic"][g, 2]
    P = fp["pmax"][g]
    c0, c1, r0, r1 = (fp["rect"][g, i] for i in range(4))
    with np.errstate(all="ignore"):
        x0 = (c0.astype(np.float32) + half) - mx
        x1 = (c1.astype(np.float32) + half) - mx
        y0 = (r0.astype(np.float32) + half) - my
        y1 = (r1.astype(np.float32) + half) - my
        xm = np.fmax(-x0, x1)
        ym = np.fmax(-y0, y1)
        mag = half * ((A * xm) * xm + (C * ym) * ym) + (np.abs(B) * xm) * ym
        pm = P + ((f32(1e-4) + f32(1e-3) * np.abs(P)) + f32(4e-6) * mag)
        # A C and B^2 are exact in double precision: D is rounded once
        D = (A.astype(np.float64) * C.astype(np.float64) - B.astype(np.float64) * B.astype(np.float64)).astype(
            np.float32)
        w = (two * pm) / D
        t = (two * pm) * A
        ymax = np.sqrt(w * A)
        xr = np.sqrt(w * C)
        ytip = -(B * xr) / C
    none = ~(pm > 0)
    full = ~none & ~((D > 0) & (A > 0) & (C > 0) & np.isfinite(t) & np.isfinite(ymax) & np.isfinite(ytip))
    return {"mx": mx, "my": my, "A": A, "B": B, "D": D, "t": t, "ymax": ymax, "ytip": ytip,
            "c0": c0, "c1": c1, "r0": r0, "r1": r1, "none": none, "full": full}


def row_span(geo, ty, tile_w, tile_h):
    """Pixel columns [lo, hi] of tile row ``ty`` (arrays aligned with the
    Gaussians of ``geo``) whose centres the ellipse reaches; lo > hi: none."""
    half = f32(0.5)
    c0, c1, r0, r1 = geo["c0"], geo["c1"], geo["r0"], geo["r1"]
    ylo = np.maximum(ty * tile_h, r0)
    yhi = np.minimum(ty * tile_h + tile_h - 1, r1)
    with np.errstate(all="ignore"):
        y0 = (ylo.astype(np.float32) + half) - geo["my"]
        y1 = (yhi.astype(np.float32) + half) - geo["my"]
        a = np.fmax(y0, -geo["ymax"])
        b = np.fmin(y1, geo["ymax"])
        miss = ~(a <= b)
        dr = np.fmin(np.fmax(geo["ytip"], a), b)
        dl = np.fmin(np.fmax(-geo["ytip"], a), b)
        D, t, A, B = geo["D"], geo["t"], geo["A"], geo["B"]
        sr = np.sqrt(np.fmax(t - (D * dr) * dr, f32(0.0)))
        sl = np.sqrt(np.fmax(t - (D * dl) * dl, f32(0.0)))
        xh = (geo["mx"] + (sr - B * dr) / A) - half
        xl = (geo["mx"] + ((-sl) - B * dl) / A) - half
        nan = np.isnan(xl) | np.isnan(xh)
        cl = c0.astype(np.float32) - f32(1.0)
        ch = c1.astype(np.float32) + f32(1.0)
        lo = np.ceil(np.fmin(np.fmax(xl, cl), ch)).astype(np.int64)
        hi = np.floor(np.fmin(np.fmax(xh, cl), ch)).astype(np.int64)
    lo = np.maximum(lo, c0)
    hi = np.minimum(hi, c1)
    whole = geo["full"] | (~geo["none"] & ~miss & nan)
    lo = np.where(whole, c0, lo)
    hi = np.where(whole, c1, np.where(geo["none"] | (miss & ~geo["full"]), c0 - 1, hi))
    return lo, hi


def binned_tiles(fp, g, tile_w=16, tile_h=16):
    """The (Gaussian, tile) pairs of Gaussians ``g``: per Gaussian, per tile
    row of its rectangle, the tiles its column span touches, in row-major
    order.  Returns index arrays (gauss, tx, ty)."""
    g = np.asarray(g, np.int64)
    r0, r1 = fp["rect"][g, 2], fp["rect"][g, 3]
    nrow = r1 // tile_h - r0 // tile_h + 1
    rep = np.repeat(np.arange(g.size), nrow)
    ty = r0[rep] // tile_h + (np.arange(rep.size) - np.repeat(np.cumsum(nrow) - nrow, nrow))
    geo = span_geometry(fp, g[rep])
    lo, hi = row_span(geo, ty, tile_w, tile_h)
    n = np.where(lo <= hi, hi // tile_w - lo // tile_w + 1, 0)
    rr = np.repeat(np.arange(rep.size), n)
    tx = lo[rr] // tile_w + (np.arange(rr.size) - np.repeat(np.cumsum(n) - n, n))
    return g[rep[rr]], tx, ty[rr]


def tile_members(fp, tx, ty, tile_w=16, tile_h=16):
    """Visible Gaussians binned to tile (tx, ty), in depth order (depth key,
    then index)."""
    g = np.nonzero(fp["visible"])[0]
    t = fp["tiles"][g]
    g = g[(t[:, 0] <= tx) & (tx <= t[:, 1]) & (t[:, 2] <= ty) & (ty <= t[:, 3])]
    lo, hi = row_span(span_geometry(fp, g), np.full(g.size, ty), tile_w, tile_h)
    g = g[(lo <= hi) & (lo // tile_w <= tx) & (tx <= hi // tile_w)]
    return g[np.lexsort((g, fp["key"][g].astype(np.int64)))]


def bin_pairs(footprints, width, height, tile_w=16, tile_h=16):
    """Duplicate-with-keys, sort and tile ranges for a batch of views.

    ``footprints`` is a list (one per view) of ``fp32_footprint`` results
    computed with opacity and alpha_min; each visible Gaussian goes to the
    tiles ``binned_tiles`` gives it.
    Returns ``tile_key`` (view * n_tiles + tile, uint32), ``gauss`` (Gaussian
    index, uint32) sorted by (tile_key, depth key, Gaussian index), and
    ``ranges`` [n_views * n_tiles, 2] (start, end) into that list.
    """
    tx = (width + tile_w - 1) // tile_w
    ty = (height + tile_h - 1) // tile_h
    n_tiles = tx * ty
    keys, depth, gid = [], [], []
    for v, fp in enumerate(footprints):
        gg, xx, yy = binned_tiles(fp, np.nonzero(fp["visible"])[0], tile_w, tile_h)
        keys.append(v * n_tiles + yy * tx + xx)
        depth.append(fp["key"][gg].astype(np.int64))
        gid.append(gg)
    keys = np.concatenate(keys).astype(np.int64) if keys else np.zeros(0, np.int64)
    depth = np.concatenate(depth) if depth else np.zeros(0, np.int64)
    gid = np.concatenate(gid).astype(np.int64) if gid else np.zeros(0, np.int64)
    order = np.lexsort((gid, depth, keys))
    keys, gid = keys[order], gid[order]
    ranges = np.zeros((len(footprints) * n_tiles, 2), np.int64)
    if keys.size:
        starts = np.r_[0, np.nonzero(np.diff(keys))[0] + 1]
        ends = np.r_[starts[1:], keys.size]
        ranges[keys[starts], 0] = starts
        ranges[keys[starts], 1] = ends
    return {"tile_key": keys.astype(np.uint32), "gauss": gid.astype(np.uint32), "ranges": ranges,
            "tiles_x": tx, "tiles_y": ty}
