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
  finite and the rectangle holds at least one pixel centre.

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


def fp32_footprint(means, log_scales, quats, cam, tile_w=16, tile_h=16, k_sigma=3.0):
    """Per-Gaussian depth key, visibility, pixel rectangle and tile rectangle.

    Returns a dict of arrays: ``key`` (uint32 bits of the float32 depth),
    ``visible`` (bool), ``rect`` (int64 [N,4] = c0, c1, r0, r1, inclusive pixel
    indices), ``tiles`` (int64 [N,4] = tx0, tx1, ty0, ty1) and ``count``.
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
    return {"key": key, "visible": visible, "rect": rect, "tiles": tiles, "count": count}


def bin_pairs(footprints, width, height, tile_w=16, tile_h=16):
    """Duplicate-with-keys, sort and tile ranges for a batch of views.

    ``footprints`` is a list (one per view) of ``fp32_footprint`` results.
    Returns ``tile_key`` (view * n_tiles + tile, uint32), ``gauss`` (Gaussian
    index, uint32) sorted by (tile_key, depth key, Gaussian index), and
    ``ranges`` [n_views * n_tiles, 2] (start, end) into that list.
    """
    tx = (width + tile_w - 1) // tile_w
    ty = (height + tile_h - 1) // tile_h
    n_tiles = tx * ty
    keys, depth, gid = [], [], []
    for v, fp in enumerate(footprints):
        g = np.nonzero(fp["visible"])[0]
        x0, x1, y0, y1 = (fp["tiles"][g, i] for i in range(4))
        cnt = fp["count"][g]
        wdt = x1 - x0 + 1
        first = np.cumsum(cnt) - cnt
        rep = np.repeat(np.arange(g.size), cnt)
        j = np.arange(int(cnt.sum())) - first[rep]
        xx = x0[rep] + j % wdt[rep]
        yy = y0[rep] + j // wdt[rep]
        keys.append(v * n_tiles + yy * tx + xx)
        depth.append(fp["key"][g][rep].astype(np.int64))
        gid.append(g[rep])
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
