"""Layered plans (multi-layer hologram with hard plane assignment, forward
recording and inverse propagation; Sec. 4.1, Eqs. 12-16) through the C ABI
against the FP64 oracle in ``oracle/layers.py``.

Bars: layer fields, the hologram P and the propagated planes within relative
L2 1e-4; intensities 2e-4; loss 1e-4; gradients (including the
straight-through logits gradient) 1e-3 per tensor.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import layers
from paper_2506_08350_amd import _lib, api
from scenegen import Optics, identity_camera, make_gaussians, make_targets, yaw_cameras
from tests.gpu_helpers import announce, cplx, make_renderer, rel_l2, to_device

pytestmark = pytest.mark.gpu


def _problem(n=300, H=40, W=60, nlay=3, seed=71, views=(0.0, 11.0), logit_scale=1.0, n_lambda=2):
    sc = make_gaussians(n, n_lambda, seed, log_scale_mean=-3.0, log_scale_std=0.4)
    cams = yaw_cameras(views, (0.0, 0.0, 2.0), W, H, f=0.8 * W)
    lams = (639e-9, 532e-9, 473e-9)[:n_lambda]
    Z = tuple(float(z) for z in np.linspace(0.5e-3, 2.0e-3, nlay))
    opt = Optics(lams, Z, 8e-6, 2, 2)
    logits = (np.random.default_rng(seed + 1).normal(size=(n, nlay)) * logit_scale).astype(np.float32)
    tg = make_targets((len(cams), n_lambda, nlay, H, W), seed + 2)
    return sc, cams, opt, logits, tg


def _params(sc, logits):
    p = to_device(sc)
    p[api.LAYER_LOGITS] = torch.from_numpy(logits).cuda()
    return p


@pytest.mark.parametrize("nlay", [1, 2, 3, 4])
def test_layer_fields_hologram_and_planes_match_oracle(nlay):
    announce(f"layered forward, {nlay} layers")
    sc, cams, opt, logits, tg = _problem(nlay=nlay, seed=70 + nlay)
    r = make_renderer(cams, opt, sc.n, tile=None, layered=True)
    params = _params(sc, logits)
    out = r.forward(params, api.pack_cameras(cams), want_field=True, want_prop=True, want_intensity=True,
                    target=torch.from_numpy(tg).cuda())
    torch.cuda.synchronize()
    assert r.read_status()[0] == 0
    st = layers.forward_layers(sc, logits.astype(np.float64), cams, opt, oracle.DEFAULT, targets=tg)
    B, L, K, H, W = r.B, r.L, r.K, r.H, r.W
    U = cplx(r.region(_lib.REGION_LAYER_FIELDS, torch.float32).view(B, L, K, H, W, 2))
    Tf = r.region(_lib.REGION_LAYER_T_FINAL, torch.float32).view(B, K, H, W).cpu().numpy()
    for b, v in enumerate(st["views"]):
        for q in range(K):
            assert rel_l2(U[b, :, q], v["res"].U[q]) < 1e-4, (b, q)
            assert rel_l2(Tf[b, q], v["res"].T_final[q]) < 1e-4, (b, q)
    assert rel_l2(cplx(out["field"]), st["P"]) < 1e-4
    assert rel_l2(cplx(out["prop"]), st["u"]) < 1e-4
    assert rel_l2(out["intensity"].cpu().numpy(), st["I"]) < 2e-4
    assert abs(float(out["loss"]) - st["loss"]) < 1e-4 * st["loss"]


@pytest.mark.parametrize("logit_scale", [1.0, 2e-3])
def test_layered_gradients_match_oracle(logit_scale):
    """logit_scale 2e-3 puts the logits within a few tau of each other, so the
    straight-through weights spread over every layer and the gradients of
    inserting a Gaussian into the other layers are exercised."""
    announce(f"layered gradients, logit scale {logit_scale}")
    sc, cams, opt, logits, tg = _problem(n=250, logit_scale=logit_scale, seed=81)
    r = make_renderer(cams, opt, sc.n, tile=None, layered=True)
    params = _params(sc, logits)
    loss, grads, _ = r.train_step(params, api.pack_cameras(cams), torch.from_numpy(tg).cuda())
    torch.cuda.synchronize()
    st = layers.forward_layers(sc, logits.astype(np.float64), cams, opt, oracle.DEFAULT, targets=tg)
    ref = layers.backward_layers(st)
    assert abs(float(loss) - st["loss"]) < 1e-4 * st["loss"]
    for k in api.PARAM_NAMES + (api.LAYER_LOGITS,):
        err = rel_l2(grads[k].cpu().numpy(), ref[k])
        assert err < 1e-3, (k, err)
    if logit_scale < 1.0:
        w = layers.ste_softmax(logits.astype(np.float64))
        assert np.mean(w.max(axis=1)) < 0.9   # the weights really are spread


@pytest.mark.parametrize("logit_scale", [1.0, 2e-3])
def test_layered_gradients_four_layers_three_wavelengths(logit_scale):
    """The layer and wavelength counts of the benchmarked four-layer step
    (each of the four own-layer copies of the backward's pair step runs)."""
    announce(f"layered gradients, 4 layers x 3 wavelengths, logit scale {logit_scale}")
    sc, cams, opt, logits, tg = _problem(n=250, nlay=4, n_lambda=3, logit_scale=logit_scale, seed=87)
    assert set(np.argmax(logits, axis=1)) == {0, 1, 2, 3}
    r = make_renderer(cams, opt, sc.n, tile=None, layered=True)
    loss, grads, _ = r.train_step(_params(sc, logits), api.pack_cameras(cams), torch.from_numpy(tg).cuda())
    torch.cuda.synchronize()
    st = layers.forward_layers(sc, logits.astype(np.float64), cams, opt, oracle.DEFAULT, targets=tg)
    ref = layers.backward_layers(st)
    assert abs(float(loss) - st["loss"]) < 1e-4 * st["loss"]
    for k in api.PARAM_NAMES + (api.LAYER_LOGITS,):
        err = rel_l2(grads[k].cpu().numpy(), ref[k])
        assert err < 1e-3, (k, err)


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (32, 8)])
def test_layered_gradients_match_oracle_at_other_tiles(tile):
    """One 8x8 block per tile takes one pixel per lane; two or four blocks
    take two pixels per lane, in one or two waves.  Every layout matches the
    oracle, on a frame whose edges cut tiles short."""
    announce(f"layered gradients, tile {tile}")
    sc, cams, opt, logits, tg = _problem(n=250, logit_scale=2e-3, seed=83, H=36, W=54)
    r = make_renderer(cams, opt, sc.n, tile=tile, layered=True)
    loss, grads, _ = r.train_step(_params(sc, logits), api.pack_cameras(cams), torch.from_numpy(tg).cuda())
    torch.cuda.synchronize()
    st = layers.forward_layers(sc, logits.astype(np.float64), cams, opt, oracle.DEFAULT, targets=tg)
    ref = layers.backward_layers(st)
    assert abs(float(loss) - st["loss"]) < 1e-4 * st["loss"]
    for k in api.PARAM_NAMES + (api.LAYER_LOGITS,):
        err = rel_l2(grads[k].cpu().numpy(), ref[k])
        assert err < 1e-3, (k, tile, err)


def test_layered_autograd_path_matches_fused_path():
    announce("layered autograd vs fused")
    sc, cams, opt, logits, tg = _problem(n=200, seed=91, logit_scale=2e-3)
    r = make_renderer(cams, opt, sc.n, tile=None, layered=True)
    cam_t = api.pack_cameras(cams)
    target = torch.from_numpy(tg).cuda()
    loss_f, grads_f, _ = r.train_step(_params(sc, logits), cam_t, target)
    leaves = {k: v.clone().requires_grad_(True) for k, v in _params(sc, logits).items()}
    I = api.render_intensity(r, cam_t, *(leaves[k] for k in api.PARAM_NAMES), leaves[api.LAYER_LOGITS])
    loss = torch.mean((I - target) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    assert abs(float(loss) - float(loss_f)) <= 1e-5 * float(loss_f)
    for k in api.PARAM_NAMES + (api.LAYER_LOGITS,):
        err = rel_l2(leaves[k].grad.cpu().numpy(), grads_f[k].cpu().numpy())
        assert err < 1e-4, (k, err)


def test_recording_is_the_adjoint_of_inverse_propagation():
    """chrf_propagate of a layered plan maps P to the layers (-Z_k) and
    chrf_propagate_adjoint records layer fields into P (+Z_l); both against
    the oracle, and their dot-product identity."""
    announce("layered propagate / record")
    H, W = 36, 48
    opt = Optics((639e-9, 473e-9), (0.4e-3, 1.2e-3, 2.5e-3), 8e-6, 2, 2)
    r = make_renderer([identity_camera(W, H)], opt, 1, tile=None, layered=True)
    rng = np.random.default_rng(5)
    P = rng.normal(size=(1, 2, H, W)) + 1j * rng.normal(size=(1, 2, H, W))
    Ul = rng.normal(size=(1, 2, 3, H, W)) + 1j * rng.normal(size=(1, 2, 3, H, W))

    def dev(z):
        return torch.from_numpy(np.stack([z.real, z.imag], -1).astype(np.float32)).cuda()

    u, _ = r.propagate(dev(P), want_intensity=False)
    rec = r.propagate_adjoint(dev(Ul))
    torch.cuda.synchronize()
    for li, lam in enumerate(opt.wavelengths):
        ref_P = layers.record(Ul[0, li], lam, opt.distances, opt.pitch, opt.pad, opt.band_limit)
        assert rel_l2(cplx(rec[0, li]), ref_P) < 1e-4
        for k, z in enumerate(opt.distances):
            ref_u = oracle.propagate(P[0, li], lam, -z, opt.pitch, opt.pad, opt.band_limit)
            assert rel_l2(cplx(u[0, li, k]), ref_u) < 1e-4
    lhs = np.vdot(Ul, cplx(u))
    rhs = np.vdot(cplx(rec), P)
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (32, 8)])
def test_layered_fields_do_not_depend_on_the_tile(tile):
    """Waves of one workgroup share a tile's records; every tile shape gives
    the same layer fields, bit for bit, as 16 x 16."""
    announce(f"layered tile invariance {tile}")
    sc, cams, opt, logits, tg = _problem(seed=77)
    outs = []
    for tl in ((16, 16), tile):
        r = make_renderer(cams, opt, sc.n, tile=tl, layered=True)
        r.forward(_params(sc, logits), api.pack_cameras(cams), want_field=True)
        torch.cuda.synchronize()
        outs.append(r.region(_lib.REGION_LAYER_FIELDS, torch.float32).clone())
    assert torch.equal(outs[0], outs[1])


def test_layered_plan_rejects_too_many_layers():
    opt5 = Optics((515e-9,), tuple(np.linspace(1e-3, 3e-3, 5)), 8e-6, 2, 2)
    with pytest.raises(_lib.ChrfError):
        make_renderer([identity_camera(32, 32)], opt5, 10, tile=None, layered=True)
