"""Pins for the oracle's analytic gradient (Supplementary D backward pass).

* central finite differences (h = 1e-4) of the oracle's own FP64 forward, in
  the smooth threshold mode where the map is differentiable;
* an independent dense formulation written with torch float64 ops
  (all-pairs alpha matrix, exclusive cumulative product for transmittance,
  torch.fft for the angular spectrum) differentiated by autograd;
* the per-parameter amplitude and phase formulas printed in Supplementary D.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import binning
from scenegen import Optics, Scene, identity_camera, make_gaussians, make_targets, yaw_cameras
from tests import dense_reference as dense



@pytest.fixture(autouse=True)
def _float64_default():
    """The dense torch formulation works in float64; the default dtype is set
    for this module's tests only, so that no other test in the process
    creates float64 tensors by accident."""
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


def _small_problem(n=30, H=40, W=48, seed=21, log_scale_mean=-2.8):
    sc = make_gaussians(n, 2, seed, log_scale_mean=log_scale_mean, log_scale_std=0.3)
    sc = Scene(*(a.astype(np.float64) for a in sc.arrays()))
    cams = yaw_cameras((0.0, 8.0), (0.0, 0.0, 2.0), W, H, f=64)
    opt = Optics((639e-9, 473e-9), (0.5e-3, 1.5e-3), 8e-6, 2, 2)
    tg = make_targets((2, 2, 2, H, W), seed + 1)
    return sc, cams, opt, tg


def _loss(sc, cams, opt, tg, thr):
    return oracle.forward(sc, cams, opt, thr, targets=tg)["loss"]


def test_gradient_matches_central_differences():
    sc, cams, opt, tg = _small_problem()
    thr = oracle.SMOOTH
    st = oracle.forward(sc, cams, opt, thr, targets=tg)
    # depth keys must not swap under a perturbation of h (a depth moves by at most h)
    for v in st["views"]:
        k = np.sort(v["proj"].t[:, 2])
        assert np.min(np.diff(k)) > 2.5e-4
    grads = oracle.backward(st)
    rng = np.random.default_rng(0)
    names = ("means", "log_scales", "quats", "opacity", "amp", "phase")
    h = 1e-4
    checked = 0
    for name in names:
        arr = getattr(sc, name)
        flat = arr.reshape(-1)
        picks = rng.choice(flat.size, size=min(flat.size, 8), replace=False)
        for i in picks:
            old = flat[i]
            flat[i] = old + h
            lp = _loss(sc, cams, opt, tg, thr)
            flat[i] = old - h
            lm = _loss(sc, cams, opt, tg, thr)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[i]
            scale = max(abs(fd), 1e-3 * np.max(np.abs(grads[name])), 1e-12)
            assert abs(an - fd) <= 2e-5 * scale, (name, i, an, fd)
            checked += 1
    assert checked >= 40


def _torch_dense_loss(params, sc, cams, opt, tg, thr):
    """Independent dense formulation: every pixel against every Gaussian,
    with the early stop of Algorithm 2 as a fixed mask."""
    total = 0.0
    n_el = 0
    for b, cam in enumerate(cams):
        a, v, _, H, Wd = dense.dense_alpha(params, sc, cam, thr)
        U = dense.composite(a, v, thr.t_min, H, Wd)
        for li, lam in enumerate(opt.wavelengths):
            for ki, zz in enumerate(opt.distances):
                u = dense.asm(U[li], lam, zz, opt.pitch, opt.band_limit)
                I = u.real ** 2 + u.imag ** 2
                total = total + torch.sum((I - torch.as_tensor(tg[b, li, ki], dtype=torch.float64)) ** 2)
                n_el += I.numel()
    return total / n_el


@pytest.mark.parametrize("mode", ["smooth", "default"])
def test_gradient_matches_torch_dense_autograd(mode):
    sc, cams, opt, tg = _small_problem(n=25, H=32, W=40, seed=31)
    if mode == "smooth":
        thr = oracle.SMOOTH
    else:
        # default support test and alpha clamp (some opacities clamp at alpha_max);
        # the dense form has no early stop, so the scene must never reach T_min
        thr = oracle.DEFAULT
        sc.opacity[:6] = 0.9995
    st = oracle.forward(sc, cams, opt, thr, targets=tg)
    if mode == "default":
        assert min(v["res"].T_final.min() for v in st["views"]) > thr.t_min
        clamped = [np.any(sc.opacity[g] * 1.0 > thr.alpha_max) for g in range(6)]
        assert any(clamped)
    grads = oracle.backward(st)
    params = [torch.tensor(a, requires_grad=True) for a in sc.arrays()]
    loss = _torch_dense_loss(params, sc, cams, opt, tg, thr)
    assert abs(loss.item() - st["loss"]) < 1e-12 * abs(st["loss"])
    loss.backward()
    for name, p in zip(("means", "log_scales", "quats", "opacity", "amp", "phase"), params):
        ref = p.grad.numpy()
        err = np.linalg.norm(grads[name] - ref) / np.linalg.norm(ref)
        assert err < 1e-9, (name, err)


def test_amplitude_and_phase_formulas_single_gaussian():
    """dL/dc = a T (cos(phi) dL/dRe + sin(phi) dL/dIm);
    dL/dphi = a T c (-sin(phi) dL/dRe + cos(phi) dL/dIm)   (Supplementary D)."""
    cam = identity_camera(24, 24, f=300)
    sc = Scene(np.array([[0.0, 0.0, 2.0]]), np.full((1, 3), math.log(0.05)), np.array([[1.0, 0, 0, 0]]),
               np.array([0.7]), np.array([[0.8]]), np.array([[0.9]]))
    thr = oracle.DEFAULT
    p = oracle.project(sc.means, sc.log_scales, sc.quats, sc.amp, sc.phase, cam)
    fp = oracle.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam)
    r = oracle.render_field(p, sc.opacity, fp, 24, 24, thr)
    rng = np.random.default_rng(4)
    G = rng.normal(size=(1, 24, 24)) + 1j * rng.normal(size=(1, 24, 24))
    d_mu, d_conic, d_op, d_v = oracle.render_field_backward(p, sc.opacity, fp, r, G, thr)
    from oracle.projection import project_backward
    g = project_backward(p, sc.quats, sc.amp, sc.phase, cam, d_mu, d_conic, d_op, d_v)
    aT = np.abs(r.U[0]) / 0.8           # a * T with T = 1 for the only Gaussian
    c, ph = 0.8, 0.9
    dc = np.sum(aT * (math.cos(ph) * G[0].real + math.sin(ph) * G[0].imag))
    dphi = np.sum(aT * c * (-math.sin(ph) * G[0].real + math.cos(ph) * G[0].imag))
    assert abs(g["amp"][0, 0] - dc) < 1e-12 * max(1, abs(dc))
    assert abs(g["phase"][0, 0] - dphi) < 1e-12 * max(1, abs(dphi))


def _saturated_problem(seed=31):
    """Dense near-opaque Gaussians: most pixel walks end early (T < T_min)
    and a fifth of the Gaussians clamp at alpha_max somewhere."""
    sc = make_gaussians(80, 2, seed, x_range=(-0.25, 0.25), y_range=(-0.25, 0.25), log_scale_mean=-1.8,
                        log_scale_std=0.3, opacity_logit_mean=3.5, opacity_logit_std=1.5)
    sc = Scene(*(a.astype(np.float64) for a in sc.arrays()))
    cams = yaw_cameras((0.0, 8.0), (0.0, 0.0, 2.0), 40, 32, f=64)
    opt = Optics((639e-9, 473e-9), (0.5e-3, 1.5e-3), 8e-6, 2, 2)
    tg = make_targets((2, 2, 2, 32, 40), seed + 1)
    return sc, cams, opt, tg


def test_gradient_with_early_termination_and_clamp_matches_dense_autograd():
    """Default thresholds on a saturated scene: the backward replay from each
    pixel's last contributor (Sec. 4.2), the crossing Gaussian included
    (Algorithm 2's stop after T < T_min), and the zero gradient of clamped
    alphas, against the dense formulation whose stop mask comes from its own
    cumulative product."""
    sc, cams, opt, tg = _saturated_problem()
    thr = oracle.DEFAULT
    st = oracle.forward(sc, cams, opt, thr, targets=tg)
    params = [torch.tensor(a, requires_grad=True) for a in sc.arrays()]
    for v, cam in zip(st["views"], cams):
        assert np.mean(v["res"].T_final < thr.t_min) >= 0.5
        with torch.no_grad():
            a, _, _, _, _ = dense.dense_alpha(params, sc, cam, thr)
        assert dense.stop_fraction(a, thr.t_min) >= 0.5
        assert float((a >= thr.alpha_max).any(0).double().mean()) >= 0.1   # clamped Gaussians
    grads = oracle.backward(st)
    loss = _torch_dense_loss(params, sc, cams, opt, tg, thr)
    assert abs(loss.item() - st["loss"]) < 1e-12 * abs(st["loss"])
    loss.backward()
    for name, p in zip(("means", "log_scales", "quats", "opacity", "amp", "phase"), params):
        ref = p.grad.numpy()
        err = np.linalg.norm(grads[name] - ref) / np.linalg.norm(ref)
        assert err < 1e-9, (name, err)


def test_dense_pin_detects_a_dropped_crossing_gaussian():
    """The pin above is sensitive to the cut: a replay that stops one
    contributor early at every terminated pixel (the crossing Gaussian
    dropped) is far outside its tolerance."""
    sc, cams, opt, tg = _saturated_problem()
    thr = oracle.DEFAULT
    st = oracle.forward(sc, cams, opt, thr, targets=tg)
    ref = oracle.backward(st)
    for v in st["views"]:
        res = v["res"]
        done = res.T_final < thr.t_min
        last = res.last.copy()
        for r, c in zip(*np.nonzero(done)):
            # the previous included position of this pixel
            prev = [pos for pos in range(last[r, c]) if _includes(v, sc, thr, pos, r, c)]
            last[r, c] = prev[-1] if prev else -1
        v["res"] = oracle.RasterResult(res.U, res.T_final, last, res.order, res.n_contrib)
    bad = oracle.backward(st)
    worst = max(np.linalg.norm(bad[k] - ref[k]) / np.linalg.norm(ref[k]) for k in ref)
    assert worst > 1e-4


def _includes(view, sc, thr, pos, r, c):
    from oracle import raster
    g = view["res"].order[pos]
    sp = raster._support(g, view["proj"], sc.opacity, view["fp"]["rect"], thr, (r, r + 1, c, c + 1))
    return sp is not None and bool(sp[-1].any())
