"""Pins for the oracle's projection, single-precision binning and compositing.

Closed forms (Eqs. 3, 4, 8, 10), the textbook alpha-blending special case
(Eq. 5), hand-computed compositing of stacked Gaussians including early
termination (Algorithm 2), invariances of the quaternion parameterisation, and
structural properties of the tile lists.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import binning, projection, raster
from scenegen import Camera, Scene, identity_camera, make_gaussians

F = 800.0


def _scene(means, log_scales, quats, opacity, amp, phase):
    a = lambda x: np.asarray(x, np.float32).reshape(len(means), -1)
    return Scene(a(means), a(log_scales), a(quats), np.asarray(opacity, np.float32), a(amp), a(phase))


def _render(scene, cam, thr=oracle.DEFAULT):
    p = projection.project(scene.means, scene.log_scales, scene.quats, scene.amp, scene.phase, cam)
    fp = binning.fp32_footprint(scene.means, scene.log_scales, scene.quats, cam, k_sigma=thr.k_sigma)
    r = raster.render_field(p, scene.opacity, fp, cam.width, cam.height, thr)
    return p, fp, r


def _pix(cam):
    x = np.arange(cam.width) + 0.5
    y = np.arange(cam.height) + 0.5
    return x[None, :], y[:, None]


def test_isotropic_on_axis_closed_form():
    cam = identity_camera(32, 32, f=F)
    s = np.float32(math.log(0.01))
    sc = _scene([[0, 0, 2]], [[s, s, s]], [[1, 0, 0, 0]], [0.8], [[0.6]], [[1.1]])
    p, fp, r = _render(sc, cam)
    sig = F * math.exp(float(s)) / 2.0
    assert np.allclose(p.cov2d[0], sig ** 2 * np.eye(2), rtol=1e-12, atol=0)
    assert np.allclose(p.mu[0], [16, 16])
    x, y = _pix(cam)
    power = ((x - 16) ** 2 + (y - 16) ** 2) / (2 * sig ** 2)
    a = np.minimum(0.99, float(np.float32(0.8)) * np.exp(-power))
    sup = (power <= 4.5) & (a >= 1 / 255)
    expected = np.where(sup, float(np.float32(0.6)) * np.exp(1j * float(np.float32(1.1))) * a, 0)
    assert np.max(np.abs(r.U[0] - expected)) < 1e-12
    assert np.allclose(r.T_final, np.where(sup, 1 - a, 1.0), atol=1e-12)


def test_anisotropic_off_axis_closed_form():
    cam = identity_camera(64, 48, f=F)
    x0, z0 = 0.05, 2.0
    sx, sy, sz = 0.02, 0.01, 0.03
    sc = _scene([[x0, 0, z0]], [np.log([sx, sy, sz])], [[1, 0, 0, 0]], [0.5], [[1]], [[0]])
    p = projection.project(sc.means, sc.log_scales, sc.quats, sc.amp, sc.phase, cam)
    m = sc.means.astype(np.float64)[0]
    e = np.exp(sc.log_scales.astype(np.float64)[0])
    xx = (F / m[2]) ** 2 * e[0] ** 2 + (F * m[0] / m[2] ** 2) ** 2 * e[2] ** 2
    yy = (F / m[2]) ** 2 * e[1] ** 2
    assert np.allclose(p.cov2d[0], [[xx, 0], [0, yy]], rtol=1e-12, atol=1e-12)
    assert np.allclose(p.mu[0], [F * m[0] / m[2] + 32, 24], rtol=1e-14)


def test_quaternion_sign_and_norm_invariance():
    sc = make_gaussians(40, 2, seed=3)
    cam = identity_camera(48, 40, f=60)
    base = _render(sc, cam)[2].U
    for k in (-1.0, 4.0, 0.25):   # exact in float32: inputs differ only in sign and norm
        sc2 = Scene(sc.means, sc.log_scales, (sc.quats * np.float32(k)).astype(np.float32),
                    sc.opacity, sc.amp, sc.phase)
        U = _render(sc2, cam)[2].U
        assert np.max(np.abs(U - base)) < 1e-12


def test_rotation_matrix_closed_form():
    h = math.sqrt(0.5)
    R = projection.quat_to_rotmat(np.array([[h, 0, 0, h]]))[0]   # 90 degrees about z
    assert np.allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    q = np.random.default_rng(0).normal(size=(100, 4))
    Rs = projection.quat_to_rotmat(q)
    assert np.allclose(np.einsum("nij,nkj->nik", Rs, Rs), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(Rs), 1.0)


def _iso(z, sig_px, op, amp, ph, x=0.0):
    s = math.log(sig_px * z / F)
    return [x, 0, z], [s, s, s], [1, 0, 0, 0], op, [amp], [ph]


def test_two_gaussians_front_to_back():
    cam = identity_camera(32, 32, f=F)
    g1 = _iso(1.0, 3.0, 0.7, 0.9, 0.3)
    g2 = _iso(2.0, 5.0, 0.6, 0.5, 2.0)
    for first, second in ((g1, g2), (g2, g1)):
        sc = _scene(*[np.array(v, dtype=object) for v in zip(first, second)])
        p, fp, r = _render(sc, cam)
        # pixel (16,16) has its centre at (16.5, 16.5), 0.5 px off both axes
        a = []
        for k in range(2):
            sig2 = p.cov2d[k, 0, 0]
            a.append(min(0.99, float(sc.opacity[k]) * math.exp(-0.25 / sig2)))
        v = [float(sc.amp[k, 0]) * np.exp(1j * float(sc.phase[k, 0])) for k in range(2)]
        front = 0 if sc.means[0, 2] < sc.means[1, 2] else 1
        back = 1 - front
        expected = a[front] * v[front] + (1 - a[front]) * a[back] * v[back]
        assert abs(r.U[0, 16, 16] - expected) < 1e-12
        assert abs(r.T_final[16, 16] - (1 - a[0]) * (1 - a[1])) < 1e-12


def test_early_termination_includes_the_crossing_gaussian():
    cam = identity_camera(32, 32, f=F)
    gs = [_iso(1.0 + 0.1 * i, 4.0, 0.95, 0.2 + 0.1 * i, 0.5 * i) for i in range(6)]
    sc = _scene(*[np.array(v, dtype=object) for v in zip(*gs)])
    p, fp, r = _render(sc, cam)
    T, U = 1.0, 0j
    n = 0
    for k in range(6):
        a = min(0.99, float(sc.opacity[k]) * math.exp(-0.25 / p.cov2d[k, 0, 0]))
        U += float(sc.amp[k, 0]) * np.exp(1j * float(sc.phase[k, 0])) * a * T
        T *= 1 - a
        n += 1
        if T < 1e-4:
            break
    assert n == 4          # the fourth Gaussian brings T below 1e-4 and is the last one in
    assert abs(r.U[0, 16, 16] - U) < 1e-12
    assert r.n_contrib[16, 16] == 4
    assert abs(r.T_final[16, 16] - T) < 1e-15


def test_zero_phase_reduces_to_alpha_blending():
    """phi = 0, one wavelength: U is the alpha-blended amplitude of Eq. 5 (per-pixel loop)."""
    sc = make_gaussians(30, 1, seed=5, log_scale_mean=-3.0)
    sc.phase[:] = 0
    cam = identity_camera(24, 20, f=40)
    thr = oracle.DEFAULT
    p, fp, r = _render(sc, cam, thr)
    assert np.max(np.abs(r.U.imag)) == 0
    for row in range(cam.height):
        for col in range(cam.width):
            cand = []
            for g in np.nonzero(fp["visible"])[0]:
                c0, c1, r0, r1 = fp["rect"][g]
                if c0 <= col <= c1 and r0 <= row <= r1:
                    cand.append((int(fp["key"][g]), g))
            C, T = 0.0, 1.0
            for _, g in sorted(cand):
                d = np.array([col + 0.5, row + 0.5]) - p.mu[g]
                A, B, Cc = p.conic[g]
                power = 0.5 * (A * d[0] ** 2 + 2 * B * d[0] * d[1] + Cc * d[1] ** 2)
                alpha = min(thr.alpha_max, float(sc.opacity[g]) * math.exp(-power))
                if power > 0.5 * thr.k_sigma ** 2 or alpha < thr.alpha_min:
                    continue
                C += float(sc.amp[g, 0]) * alpha * T
                T *= 1 - alpha
                if T < thr.t_min:
                    break
            assert abs(r.U[0, row, col].real - C) < 1e-12
            assert abs(r.T_final[row, col] - T) < 1e-12


def test_fp32_footprint_encloses_support_and_keys_match_depth():
    sc = make_gaussians(300, 1, seed=11, log_scale_mean=-3.5)
    cam = identity_camera(64, 48, f=64)
    p = projection.project(sc.means, sc.log_scales, sc.quats, sc.amp, sc.phase, cam)
    fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam)
    depth32 = fp["key"].view(np.float32).astype(np.float64)
    assert np.all(np.abs(depth32 - p.t[:, 2]) <= 2 * np.spacing(np.float32(3.0)))
    x, y = _pix(cam)
    for g in range(sc.n):
        d = (x - p.mu[g, 0], y - p.mu[g, 1])
        A, B, C = p.conic[g]
        power = 0.5 * (A * d[0] ** 2 + 2 * B * d[0] * d[1] + C * d[1] ** 2)
        inside = power <= 4.5 * (1 - 1e-9)
        if not fp["visible"][g]:
            assert not inside.any()
            continue
        rows, cols = np.nonzero(inside)
        c0, c1, r0, r1 = fp["rect"][g]
        if rows.size:
            assert c0 <= cols.min() and cols.max() <= c1 and r0 <= rows.min() and rows.max() <= r1


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_bin_pairs_structure(tile):
    """Every tile holding a pixel that a Gaussian supports (FP64 oracle
    compositing rule) lists it; it is listed only in tiles of its rectangle;
    each list is in depth order and the ranges delimit it."""
    thr = oracle.DEFAULT
    sc = make_gaussians(200, 1, seed=12, log_scale_mean=-3.5)
    cams = [identity_camera(70, 45, f=64), identity_camera(70, 45, f=90)]
    fps = [binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, c, *tile, thr.k_sigma, sc.opacity,
                                  thr.alpha_min) for c in cams]
    out = binning.bin_pairs(fps, 70, 45, *tile)
    key, gid, ranges = out["tile_key"].astype(np.int64), out["gauss"].astype(np.int64), out["ranges"]
    assert np.all(np.diff(key) >= 0)
    tx = out["tiles_x"]
    n_tiles = tx * out["tiles_y"]
    n_rect_pairs = 0
    for v, (fp, cam) in enumerate(zip(fps, cams)):
        p = projection.project(sc.means, sc.log_scales, sc.quats, sc.amp, sc.phase, cam)
        for g in np.nonzero(fp["visible"])[0]:
            c0, c1, r0, r1 = fp["rect"][g]
            in_rect = set()
            for ty_ in range(r0 // tile[1], r1 // tile[1] + 1):
                for tx_ in range(c0 // tile[0], c1 // tile[0] + 1):
                    in_rect.add(v * n_tiles + ty_ * tx + tx_)
            n_rect_pairs += len(in_rect)
            listed = set(int(t) for t in key[gid == g] if t // n_tiles == v)
            assert listed <= in_rect
            sp = raster._support(g, p, sc.opacity, fp["rect"], thr)
            rows, cols = np.nonzero(sp[7])
            rows, cols = rows + sp[0][0].start, cols + sp[0][1].start
            needed = set((v * n_tiles + (rows // tile[1]) * tx + cols // tile[0]).tolist())
            assert needed <= listed, (v, g)
    assert key.size < n_rect_pairs          # tiles the ellipse cannot reach are dropped
    for t in range(len(ranges)):
        s, e = ranges[t]
        assert np.all(key[s:e] == t)
        v = t // n_tiles
        d = fps[v]["key"][gid[s:e]].astype(np.int64)
        order = np.lexsort((gid[s:e], d))
        assert np.all(order == np.arange(e - s))
    assert ranges[:, 1].max() == key.size


def test_tile_members_match_bin_pairs():
    thr = oracle.DEFAULT
    sc = make_gaussians(300, 1, seed=13, log_scale_mean=-3.0)
    cam = identity_camera(64, 48, f=70)
    fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam, 16, 16, thr.k_sigma, sc.opacity,
                                thr.alpha_min)
    out = binning.bin_pairs([fp], 64, 48)
    for t, (s, e) in enumerate(out["ranges"]):
        got = binning.tile_members(fp, t % out["tiles_x"], t // out["tiles_x"])
        assert np.array_equal(got, out["gauss"][s:e].astype(np.int64))


def test_bin_pairs_requires_the_support_limit():
    sc = make_gaussians(20, 1, seed=14)
    cam = identity_camera(32, 32, f=40)
    fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam)
    with pytest.raises(ValueError):
        binning.bin_pairs([fp], 32, 32)
