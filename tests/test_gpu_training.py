"""The training loop's library kernels against ``oracle/training.py`` and the
FP64 pipeline oracle: Adan updates (relative 1e-5 over several steps),
densification (index map and kinds bit-exact, new means / log-scales /
phases within 1e-5), the carried arrays (bit-exact), the view-space gradient
statistics (relative L2 1e-3, counts exact), and a short training run whose
loss falls across a densification."""
import numpy as np
import pytest
import torch

import oracle
from oracle import training
from paper_2506_08350_amd import api
from scenegen import Optics, identity_camera, make_gaussians, make_targets, yaw_cameras
from tests.gpu_helpers import announce, make_renderer, rel_l2, to_device

pytestmark = pytest.mark.gpu


def test_adan_matches_oracle():
    announce("adan steps")
    rng = np.random.default_rng(5)
    n = 3000
    x0 = rng.normal(size=n).astype(np.float32)
    grads = [rng.normal(size=n).astype(np.float32) for _ in range(6)]
    xt = torch.from_numpy(x0.copy()).cuda()
    st_gpu, st_ref, x = {}, {}, x0.astype(np.float64)
    for k, g in enumerate(grads, 1):
        api.adan_step(xt, torch.from_numpy(g).cuda(), st_gpu, lr=0.01, step=k, weight_decay=0.02)
        x = training.adan_step(x, g.astype(np.float64), st_ref, lr=0.01, step=k, weight_decay=0.02)
    torch.cuda.synchronize()
    assert np.allclose(xt.cpu().numpy(), x, rtol=1e-5, atol=1e-6)
    for key in ("m", "v", "n"):
        assert np.allclose(st_gpu[key].cpu().numpy(), st_ref[key], rtol=1e-5, atol=1e-7), key


def _densify_inputs(n, n_lam, rng):
    means = rng.normal(size=(n, 3)).astype(np.float32)
    log_scales = rng.normal(np.log(0.03), 1.0, size=(n, 3)).astype(np.float32)
    quats = rng.normal(size=(n, 4)).astype(np.float32)
    opacity = rng.uniform(0.0, 0.05, size=n).astype(np.float32)
    phase = rng.uniform(0, 2 * np.pi, size=(n, n_lam)).astype(np.float32)
    count = rng.integers(0, 4, size=n).astype(np.float32)
    accum = (count * rng.uniform(0.0, 2.0, size=n) * 2e-4).astype(np.float32)
    # exact ties of the grow test: accum == fl(tau * count)
    tie = rng.uniform(size=n) < 0.05
    accum[tie] = (np.float32(2e-4) * count[tie]).astype(np.float32)
    xi = rng.normal(size=(n, 2, 3)).astype(np.float32)
    zeta = rng.normal(size=(n, 2, n_lam)).astype(np.float32)
    return dict(means=means, log_scales=log_scales, quats=quats, opacity=opacity, phase=phase, accum=accum,
                count=count, xi=xi, zeta=zeta)


@pytest.mark.parametrize("n", [0, 1, 7, 5000])
def test_densify_matches_oracle(n):
    announce(f"densify n={n}")
    rng = np.random.default_rng(100 + n)
    a = _densify_inputs(n, 3, rng)
    cfg = api.DensifyConfig(tau_grad=2e-4, split_scale=0.05, prune_scale=0.5, min_opacity=0.005, phase_sigma=0.02)
    dev = {k: torch.from_numpy(v).cuda() for k, v in a.items()}
    params = {k: dev[k] for k in ("means", "log_scales", "quats", "phase")}
    m, src, kind, means, ls, ph, n_out = api.densify(params, dev["opacity"], dev["accum"], dev["count"], dev["xi"],
                                                     dev["zeta"], cfg)
    r_src, r_kind, r_m, r_s, r_p = training.densify(
        a["means"], a["log_scales"], a["quats"], a["opacity"], a["phase"], a["accum"], a["count"], a["xi"], a["zeta"],
        tau_grad=cfg.tau_grad, sigma_split=float(np.float32(np.log(cfg.split_scale))),
        sigma_prune=float(np.float32(np.log(cfg.prune_scale))), min_opacity=cfg.min_opacity,
        phase_sigma=cfg.phase_sigma, shrink=float(np.float32(cfg.shrink)))
    assert m == len(r_src)
    assert np.array_equal(src.cpu().numpy(), r_src) and np.array_equal(kind.cpu().numpy(), r_kind)
    if n > 100:
        assert {0, 1, 2} <= set(r_kind.tolist()) and m != n   # every case occurs
    assert np.allclose(means.cpu().numpy(), r_m, rtol=1e-5, atol=1e-6)
    assert np.allclose(ls.cpu().numpy(), r_s, rtol=1e-6, atol=1e-6)
    assert np.allclose(ph.cpu().numpy(), r_p, rtol=1e-6, atol=1e-5)
    # carried arrays: the quaternions (kept for every kind) and fresh optimiser state
    q = api.gather_rows(dev["quats"], src, kind, n_out, zero_new=False)
    st = api.gather_rows(dev["quats"], src, kind, n_out, zero_new=True)
    torch.cuda.synchronize()
    assert np.array_equal(q.cpu().numpy(), training.gather_rows(a["quats"], r_src, r_kind, False))
    assert np.array_equal(st.cpu().numpy(), training.gather_rows(a["quats"], r_src, r_kind, True))


def test_densify_stats_match_oracle_mean_gradient():
    announce("densify statistics")
    H, W = 40, 60
    opt = Optics((639e-9, 515e-9), (0.5e-3, 1.2e-3), 8e-6, 2, 2)
    cams = [identity_camera(W, H, f=0.8 * W)] + yaw_cameras((10.0,), (0.0, 0.0, 2.0), W, H, f=0.8 * W)
    scene = make_gaussians(60, 2, 21, log_scale_mean=-2.6, log_scale_std=0.3)
    targets = make_targets((2, 2, 2, H, W), 22)
    r = make_renderer(cams, opt, scene.n)
    params = to_device(scene)
    cam_t = api.pack_cameras(cams)
    r.train_step(params, cam_t, torch.from_numpy(targets).cuda())
    accum = torch.zeros(scene.n, dtype=torch.float32, device="cuda")
    count = torch.zeros_like(accum)
    r.densify_stats(scene.n, accum, count)
    r.densify_stats(scene.n, accum, count)   # accumulates
    torch.cuda.synchronize()
    st = oracle.forward(scene, cams, opt, oracle.DEFAULT, targets=targets)
    oracle.backward(st)
    ref_a = np.zeros(scene.n)
    ref_c = np.zeros(scene.n)
    for view in st["views"]:
        ref_a, ref_c = training.accumulate_stats(ref_a, ref_c, np.nan_to_num(view["d_mu"]), view["fp"]["visible"])
    assert np.array_equal(count.cpu().numpy(), 2 * ref_c)
    assert rel_l2(accum.cpu().numpy(), 2 * ref_a) < 1e-3


def test_training_loop_lowers_the_loss_across_densification():
    """A scene renders the targets; a perturbed copy is trained towards them
    for 40 steps with densification at step 20."""
    announce("training loop")
    H, W = 48, 64
    opt = Optics((639e-9, 515e-9, 473e-9), (1e-3, 2e-3), 8e-6, 2, 2)
    cams = [identity_camera(W, H)]
    truth = make_gaussians(300, 3, 31, log_scale_mean=-3.0, log_scale_std=0.3)
    r0 = make_renderer(cams, opt, truth.n)
    cam_t = api.pack_cameras(cams)
    target = r0.forward(to_device(truth), cam_t, want_field=False, want_intensity=True)["intensity"].contiguous()
    start = make_gaussians(300, 3, 32, log_scale_mean=-3.0, log_scale_std=0.3)
    params = to_device(start)
    params["opacity"] = torch.logit(params["opacity"].clamp(1e-4, 1 - 1e-4)).contiguous()
    r = make_renderer(cams, opt, 2 * start.n)
    cfg = api.DensifyConfig(tau_grad=1e-6, split_scale=0.05, prune_scale=1.0, min_opacity=0.005)
    tr = api.Trainer(r, params, cam_t, target, total_steps=40, densify_every=20, densify_until=20, densify_cfg=cfg)
    losses = [float(tr.step()) for _ in range(40)]
    assert np.all(np.isfinite(losses))
    assert tr.n != start.n
    assert np.mean(losses[-5:]) < 0.8 * np.mean(losses[:5]), (losses[:5], losses[-5:])
