"""Pins for the multi-layer oracle (Sec. 4.1, Eqs. 12-16; Supplementary D).

* one layer reduces to the single-plane compositing of raster.py;
* every layer equals the single-plane compositing of only the Gaussians
  assigned to it (Eq. 13: a Gaussian neither contributes to nor occludes
  another layer);
* closed forms for two Gaussians on one pixel in the same / in different
  layers, and per-layer early termination;
* forward recording and inverse propagation of constant fields without
  padding, where every transfer function acts on the DC bin only:
  P = sum_l c_l exp(i 2 pi Z_l / lambda), u_k = P exp(-i 2 pi Z_k / lambda);
* central finite differences of the full multi-layer loss in the smooth
  threshold mode w.r.t. the continuous assignment weights (own and other
  layers) and the Gaussian parameters;
* the hard assignment and the straight-through softmax weights.
"""
import numpy as np

import oracle
from oracle import binning, layers, projection, raster
from scenegen import Camera, Optics, Scene, identity_camera, make_gaussians, make_targets, yaw_cameras


def _scene(n=40, nl=1, seed=5, log_scale_mean=-2.8):
    sc = make_gaussians(n, nl, seed, log_scale_mean=log_scale_mean, log_scale_std=0.3)
    return Scene(*(a.astype(np.float64) for a in sc.arrays()))


def _view(sc, cam, thr=oracle.DEFAULT):
    p = projection.project(sc.means, sc.log_scales, sc.quats, sc.amp, sc.phase, cam)
    fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam, k_sigma=thr.k_sigma)
    return p, fp


def test_one_layer_is_the_single_plane_compositing():
    sc = _scene(nl=2)
    cam = identity_camera(48, 40, f=64)
    p, fp = _view(sc, cam)
    ref = raster.render_field(p, sc.opacity, fp, 48, 40, oracle.DEFAULT)
    got = layers.render_layers(p, sc.opacity, fp, np.ones((sc.n, 1)), 48, 40, oracle.DEFAULT)
    assert np.allclose(got.U[0], ref.U, rtol=0, atol=1e-13)
    assert np.allclose(got.T_final[0], ref.T_final, rtol=0, atol=1e-13)


def test_each_layer_is_the_compositing_of_its_own_gaussians():
    sc = _scene(n=60, nl=2, seed=8, log_scale_mean=-2.5)
    cam = identity_camera(48, 40, f=64)
    thr = oracle.DEFAULT
    p, fp = _view(sc, cam)
    logits = np.random.default_rng(1).normal(size=(sc.n, 3))
    w = layers.hard_assignment(logits)
    got = layers.render_layers(p, sc.opacity, fp, w, 48, 40, thr)
    for l in range(3):
        sub = dict(fp)
        sub["visible"] = fp["visible"] & (np.argmax(logits, axis=1) == l)
        ref = raster.render_field(p, sc.opacity, sub, 48, 40, thr)
        assert np.allclose(got.U[l], ref.U, rtol=0, atol=1e-13), l
        assert np.allclose(got.T_final[l], ref.T_final, rtol=0, atol=1e-13), l
    # the layers are not all trivial
    assert all(np.abs(got.U[l]).max() > 1e-3 for l in range(3))


def _two_on_axis(opacities, amps, phases):
    """Two isotropic Gaussians on the optical axis at depths 1 and 2 (front first)."""
    means = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 2.0]])
    ls = np.full((2, 3), np.log(0.05))
    quats = np.tile([1.0, 0.0, 0.0, 0.0], (2, 1))
    sc = Scene(means, ls, quats, np.asarray(opacities, float), np.asarray(amps, float)[:, None],
               np.asarray(phases, float)[:, None])
    cam = identity_camera(9, 9, f=9)
    return sc, cam


def test_two_gaussians_same_and_different_layers():
    sc, cam = _two_on_axis([0.6, 0.5], [0.8, 0.3], [0.4, 2.0])
    thr = oracle.DEFAULT
    p, fp = _view(sc, cam)
    v = p.v[:, 0]
    r, c = 4, 4   # centre pixel
    dx = np.array([c + 0.5, c + 0.5]) - p.mu[:, 0]
    dy = np.array([r + 0.5, r + 0.5]) - p.mu[:, 1]
    power = 0.5 * (p.conic[:, 0] * dx * dx + 2 * p.conic[:, 1] * dx * dy + p.conic[:, 2] * dy * dy)
    a = np.minimum(thr.alpha_max, sc.opacity * np.exp(-power))
    same = layers.render_layers(p, sc.opacity, fp, np.array([[1.0, 0.0], [1.0, 0.0]]), 9, 9, thr)
    assert np.isclose(same.U[0, 0, r, c], a[0] * v[0] + (1 - a[0]) * a[1] * v[1], rtol=1e-12)
    assert np.isclose(same.T_final[0, r, c], (1 - a[0]) * (1 - a[1]), rtol=1e-12)
    assert same.U[1, 0, r, c] == 0 and same.T_final[1, r, c] == 1
    diff = layers.render_layers(p, sc.opacity, fp, np.array([[1.0, 0.0], [0.0, 1.0]]), 9, 9, thr)
    assert np.isclose(diff.U[0, 0, r, c], a[0] * v[0], rtol=1e-12)
    assert np.isclose(diff.U[1, 0, r, c], a[1] * v[1], rtol=1e-12)   # not occluded by the front Gaussian


def test_termination_is_per_layer():
    # a saturating stack in layer 0 in front of one Gaussian in layer 1 and one more in layer 0
    n = 6
    means = np.array([[0.0, 0.0, 1.0 + 0.1 * i] for i in range(n)])
    ls = np.full((n, 3), np.log(0.3))
    quats = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    opac = np.array([0.99, 0.99, 0.99, 0.5, 0.5, 0.5])
    sc = Scene(means, ls, quats, opac, np.ones((n, 1)), np.zeros((n, 1)))
    cam = identity_camera(5, 5, f=5)
    thr = oracle.DEFAULT
    p, fp = _view(sc, cam)
    w = np.zeros((n, 2))
    w[[0, 1, 2, 4], 0] = 1
    w[[3, 5], 1] = 1
    res = layers.render_layers(p, sc.opacity, fp, w, 5, 5, thr)
    r = c = 2
    a = np.minimum(thr.alpha_max, opac * np.exp(-0.5 * ((c + 0.5 - p.mu[:, 0]) ** 2 * p.conic[:, 0]
                                                        + (r + 0.5 - p.mu[:, 1]) ** 2 * p.conic[:, 2])))
    # layer 0: T after three 0.99 Gaussians < 1e-4, so the fourth (index 4) is dropped
    T0 = (1 - a[0]) * (1 - a[1]) * (1 - a[2])
    assert T0 < thr.t_min
    assert np.isclose(res.U[0, 0, r, c], a[0] + (1 - a[0]) * a[1] + (1 - a[0]) * (1 - a[1]) * a[2], rtol=1e-12)
    assert np.isclose(res.T_final[0, r, c], T0, rtol=1e-12)
    assert res.stop[0, r, c] == 2
    # layer 1 is untouched by layer 0's termination
    assert np.isclose(res.U[1, 0, r, c], a[3] + (1 - a[3]) * a[5], rtol=1e-12)
    assert res.stop[1, r, c] == layers.NEVER


def test_recording_and_inverse_propagation_of_constant_fields():
    """pad = 1: a constant field lives on the DC bin, where H = exp(i 2 pi z / lambda)."""
    lam, pitch = 515e-9, 8e-6
    Z = (0.7e-3, 1.3e-3, 2.9e-3)
    c = np.array([0.3 + 0.1j, -0.2 + 0.5j, 0.05 - 0.4j])
    U = np.stack([np.full((6, 10), ci) for ci in c])
    P = layers.record(U, lam, Z, pitch, pad=1, mode=2)
    P_ref = sum(ci * np.exp(2j * np.pi * z / lam) for ci, z in zip(c, Z))
    assert np.allclose(P, P_ref, rtol=0, atol=1e-12)
    for z in Z:
        u = oracle.propagate(P, lam, -z, pitch, pad=1, mode=2)
        assert np.allclose(u, P_ref * np.exp(-2j * np.pi * z / lam), rtol=0, atol=1e-12)


def _layer_problem(seed=34):
    sc = _scene(n=24, nl=2, seed=seed, log_scale_mean=-2.6)
    cams = yaw_cameras((0.0, 9.0), (0.0, 0.0, 2.0), 32, 28, f=48)
    opt = Optics((639e-9, 473e-9), (0.6e-3, 1.1e-3, 1.6e-3), 8e-6, 2, 2)
    logits = np.random.default_rng(seed).normal(size=(sc.n, 3))
    tg = make_targets((2, 2, 3, 28, 32), seed + 2)
    return sc, cams, opt, logits, tg


def test_layer_gradients_match_central_differences():
    sc, cams, opt, logits, tg = _layer_problem()
    thr = oracle.SMOOTH
    st = layers.forward_layers(sc, logits, cams, opt, thr, targets=tg)
    for v in st["views"]:
        k = np.sort(v["proj"].t[:, 2])
        assert np.min(np.diff(k)) > 2.5e-4
    g = layers.backward_layers(st)
    w0 = st["weights"]
    h = 1e-4

    def loss_w(w):
        return layers.forward_layers(sc, logits, cams, opt, thr, targets=tg, weights=w)["loss"]

    rng = np.random.default_rng(3)
    checked = 0
    # assignment weights: own layer and the other layers of several Gaussians
    for n in rng.choice(sc.n, size=6, replace=False):
        for l in range(3):
            wp, wm = w0.copy(), w0.copy()
            wp[n, l] += h
            wm[n, l] -= h
            fd = (loss_w(wp) - loss_w(wm)) / (2 * h)
            an = g["rho"][n, l]
            scale = max(abs(fd), 1e-3 * np.max(np.abs(g["rho"])), 1e-12)
            assert abs(an - fd) <= 2e-5 * scale, (n, l, an, fd)
            checked += 1
    assert np.count_nonzero(np.abs(g["rho"][w0 == 0]) > 1e-9) > 10   # other-layer terms are live
    for name in ("means", "log_scales", "quats", "opacity", "amp", "phase"):
        flat = getattr(sc, name).reshape(-1)
        for i in rng.choice(flat.size, size=min(flat.size, 5), replace=False):
            old = flat[i]
            flat[i] = old + h
            lp = layers.forward_layers(sc, logits, cams, opt, thr, targets=tg)["loss"]
            flat[i] = old - h
            lm = layers.forward_layers(sc, logits, cams, opt, thr, targets=tg)["loss"]
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            scale = max(abs(fd), 1e-3 * np.max(np.abs(g[name])), 1e-12)
            assert abs(an - fd) <= 2e-5 * scale, (name, i, an, fd)
            checked += 1
    assert checked >= 40


def test_hard_assignment_and_straight_through_weights():
    logits = np.array([[0.1, 0.5, 0.5], [2.0, -1.0, 0.0], [0.3, 0.3, 0.3]])
    w = layers.hard_assignment(logits)
    assert np.array_equal(w, [[0, 1, 0], [1, 0, 0], [1, 0, 0]])   # ties: lowest index
    s = layers.ste_softmax(logits, tau=1e-3)
    assert np.allclose(s.sum(axis=1), 1.0)
    assert np.allclose(s[1], [1, 0, 0]) and np.allclose(s[2], [1 / 3] * 3)
    assert np.allclose(s[0], [0, 0.5, 0.5])
    # a logit gap of tau ln 3 gives weights 3:1
    s2 = layers.ste_softmax(np.array([[1e-3 * np.log(3.0), 0.0]]), tau=1e-3)
    assert np.allclose(s2, [[0.75, 0.25]])
    sc, cams, opt, lg, tg = _layer_problem(seed=33)
    st = layers.forward_layers(sc, lg, cams[:1], opt, oracle.DEFAULT, targets=tg[:1])
    g = layers.backward_layers(st)
    assert np.allclose(g["logits"], g["rho"] * layers.ste_softmax(lg))


def test_layer_gradients_with_termination_match_dense_autograd():
    """Default thresholds, three layers of dense near-opaque Gaussians (about
    half the pixels end each layer's walk early; some alphas clamp): the
    oracle's per-layer reverse replay against a dense torch formulation of
    Eqs. 13-16 whose per-layer stop masks come from its own cumulative
    products, differentiated by autograd w.r.t. the Gaussian parameters and
    the assignment weights rho at the one-hot point."""
    import torch

    from tests import dense_reference as dense

    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    try:
        sc = make_gaussians(160, 2, 35, x_range=(-0.25, 0.25), y_range=(-0.25, 0.25), log_scale_mean=-1.8,
                            log_scale_std=0.3, opacity_logit_mean=3.5, opacity_logit_std=1.5)
        sc = Scene(*(a.astype(np.float64) for a in sc.arrays()))
        cams = yaw_cameras((0.0, 9.0), (0.0, 0.0, 2.0), 32, 28, f=48)
        opt = Optics((639e-9, 473e-9), (0.6e-3, 1.1e-3, 1.6e-3), 8e-6, 2, 2)
        logits = np.random.default_rng(35).normal(size=(sc.n, 3))
        tg = make_targets((2, 2, 3, 28, 32), 37)
        thr = oracle.DEFAULT
        st = layers.forward_layers(sc, logits, cams, opt, thr, targets=tg)
        for v in st["views"]:
            stopped = np.any(v["res"].stop != layers.NEVER, axis=0)
            assert np.mean(stopped) >= 0.5
        g = layers.backward_layers(st)

        params = [torch.tensor(a, requires_grad=True) for a in sc.arrays()]
        w = torch.tensor(st["weights"], requires_grad=True)
        total, n_el, clamped = 0.0, 0, 0.0
        for b, cam in enumerate(cams):
            a, v, order, H, W = dense.dense_alpha(params, sc, cam, thr)
            clamped = max(clamped, float((a >= thr.alpha_max).any(0).double().mean()))
            wl = w[order]
            U = [dense.composite(a * wl[:, l][None], v, thr.t_min, H, W) for l in range(3)]
            for li, lam in enumerate(opt.wavelengths):
                P = sum(dense.asm(U[l][li], lam, z, opt.pitch, opt.band_limit) for l, z in enumerate(opt.distances))
                for k, z in enumerate(opt.distances):
                    u = dense.asm(P, lam, -z, opt.pitch, opt.band_limit)
                    I = u.real ** 2 + u.imag ** 2
                    total = total + torch.sum((I - torch.as_tensor(tg[b, li, k])) ** 2)
                    n_el += I.numel()
        assert clamped >= 0.1
        loss = total / n_el
        assert abs(loss.item() - st["loss"]) < 1e-12 * st["loss"]
        loss.backward()
        for name, p in zip(("means", "log_scales", "quats", "opacity", "amp", "phase"), params):
            ref = p.grad.numpy()
            err = np.linalg.norm(g[name] - ref) / np.linalg.norm(ref)
            assert err < 1e-9, (name, err)
        err = np.linalg.norm(g["rho"] - w.grad.numpy()) / np.linalg.norm(w.grad.numpy())
        assert err < 1e-9, ("rho", err)
    finally:
        torch.set_default_dtype(old)
