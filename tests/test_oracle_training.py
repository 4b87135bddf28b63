"""Pins of the optimiser and densification oracle (``oracle/training.py``).

Adan with the gradient-difference moment switched off (b2 = 0) is Adam, so
it must agree with torch.optim.Adam; a constant gradient has the closed form
theta_k = theta_0 - k lr g / (|g| + eps).  Split children are samples of
their Gaussian, so their offsets must have its covariance
R diag(exp(2 s)) R^T (taken from the projection oracle's camera-space
covariance, an independent route); counts, order and the thresholds are checked on
hand-made cases.
"""
import numpy as np
import pytest
import torch

from oracle import training
from oracle.projection import quat_to_rotmat
from scenegen import identity_camera


def test_adan_without_difference_moment_is_adam():
    rng = np.random.default_rng(0)
    x0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(8)]
    st, x = {}, x0.copy()
    for k, g in enumerate(grads, 1):
        x = training.adan_step(x, g, st, lr=0.01, step=k, betas=(0.9, 0.0, 0.99))
    p = torch.nn.Parameter(torch.tensor(x0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.99), eps=1e-8)
    for g in grads:
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    assert np.allclose(x, p.detach().numpy(), rtol=0, atol=1e-12)


def test_adan_constant_gradient_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    st, x = {}, np.zeros(3)
    for k in range(1, 6):
        x = training.adan_step(x, g, st, lr=0.1, step=k)
    assert np.allclose(x, -5 * 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adan_uses_the_gradient_difference():
    """With b2 > 0 the update differs from Adam's exactly through v and the
    corrected second moment; on a quadratic it still converges."""
    st, x = {}, np.array([3.0, -1.0])
    for k in range(1, 400):
        x = training.adan_step(x, 2.0 * (x - np.array([1.0, 2.0])), st, lr=0.05, step=k)
    assert np.allclose(x, [1.0, 2.0], atol=1e-2)
    st1, st2 = {}, {}
    a = training.adan_step(np.zeros(1), np.ones(1), st1, 0.1, 1)
    b = training.adan_step(a, 3 * np.ones(1), st1, 0.1, 2)
    a2 = training.adan_step(np.zeros(1), np.ones(1), st2, 0.1, 1, betas=(0.9, 0.0, 0.99))
    b2 = training.adan_step(a2, 3 * np.ones(1), st2, 0.1, 2, betas=(0.9, 0.0, 0.99))
    assert a[0] == a2[0] and b[0] != b2[0]


def _scene(n, rng):
    return dict(
        means=rng.normal(size=(n, 3)),
        log_scales=rng.normal(-3.0, 0.3, size=(n, 3)),
        quats=rng.normal(size=(n, 4)),
        opacity=rng.uniform(0.2, 0.9, size=n),
        phase=rng.uniform(0, 2 * np.pi, size=(n, 3)),
    )


KW = dict(tau_grad=2e-4, sigma_split=float(np.log(0.05)), sigma_prune=float(np.log(1.0)), min_opacity=0.005,
          phase_sigma=0.01)


def _run(sc, accum, count, xi, zeta, **kw):
    args = dict(KW)
    args.update(kw)
    return training.densify(sc["means"], sc["log_scales"], sc["quats"], sc["opacity"], sc["phase"], accum, count, xi,
                            zeta, **args)


def test_densify_identity_when_nothing_grows():
    rng = np.random.default_rng(1)
    n = 40
    sc = _scene(n, rng)
    src, kind, m, s, p = _run(sc, np.zeros(n), np.zeros(n), rng.normal(size=(n, 2, 3)), rng.normal(size=(n, 2, 3)))
    assert np.array_equal(src, np.arange(n)) and np.all(kind == training.KIND_KEPT)
    assert np.array_equal(m, sc["means"]) and np.array_equal(s, sc["log_scales"]) and np.array_equal(p, sc["phase"])


def test_densify_clone_split_prune_cases():
    rng = np.random.default_rng(2)
    sc = _scene(5, rng)
    sc["log_scales"][:] = -4.0
    sc["log_scales"][2, 1] = -2.0          # large: splits when it grows
    sc["opacity"][3] = 0.001               # pruned
    sc["log_scales"][4, 0] = 0.5           # too large: pruned
    accum = np.array([1e-3, 1e-5, 1e-3, 1e-3, 0.0])
    count = np.array([2.0, 2.0, 2.0, 2.0, 0.0])
    xi = rng.normal(size=(5, 2, 3))
    zeta = rng.normal(size=(5, 2, 3))
    src, kind, m, s, p = _run(sc, accum, count, xi, zeta)
    # 0 grows and is small: kept + clone; 1 does not grow; 2 splits into two; 3 and 4 are pruned
    # (3 would have cloned, but the clone has the same opacity and is pruned too)
    assert src.tolist() == [0, 0, 1, 2, 2]
    assert kind.tolist() == [0, 1, 0, 2, 2]
    assert np.array_equal(m[1], sc["means"][0]) and np.array_equal(s[1], sc["log_scales"][0])
    assert np.allclose(p[1], sc["phase"][0] + 0.01 * zeta[0, 0], rtol=0, atol=1e-15)
    assert np.allclose(np.exp(s[3]), np.exp(sc["log_scales"][2]) / 1.6, rtol=1e-14)
    R = quat_to_rotmat(sc["quats"][2:3])[0]
    for c in range(2):
        off = np.linalg.solve(R, m[3 + c] - sc["means"][2]) / np.exp(sc["log_scales"][2])
        assert np.allclose(off, xi[2, c], rtol=1e-12, atol=1e-12)
        assert np.allclose(p[3 + c], sc["phase"][2] + 0.01 * zeta[2, c], rtol=0, atol=1e-15)


def test_densify_grow_threshold_is_the_mean_gradient():
    sc = _scene(2, np.random.default_rng(3))
    sc["log_scales"][:] = -4.0
    z = np.zeros((2, 2, 3))
    src, kind, *_ = _run(sc, np.array([4e-4, 3.9e-4]), np.array([2.0, 2.0]), z, z)
    assert src.tolist() == [0, 0, 1] and kind.tolist() == [0, 1, 0]


def test_split_children_sample_the_gaussian_covariance():
    """20,000 children of one anisotropic, rotated Gaussian: the covariance of
    their offsets is Sigma = R S S^T R^T of the projection oracle."""
    from oracle import projection
    rng = np.random.default_rng(4)
    n = 10_000
    q = np.array([[0.8, 0.3, -0.4, 0.2]])
    ls = np.array([[-1.0, -2.0, -0.5]])
    sc = dict(means=np.tile([[0.5, -0.2, 2.0]], (n, 1)), log_scales=np.tile(ls, (n, 1)), quats=np.tile(q, (n, 1)),
              opacity=np.full(n, 0.5), phase=np.zeros((n, 1)))
    src, kind, m, *_ = _run(sc, np.ones(n), np.ones(n), rng.normal(size=(n, 2, 3)), np.zeros((n, 2, 1)),
                            sigma_split=float(np.log(0.01)), sigma_prune=10.0)
    assert m.shape == (2 * n, 3) and np.all(kind == training.KIND_SPLIT)
    d = m - sc["means"][0]
    emp = d.T @ d / d.shape[0]
    # the projection oracle's camera-space covariance W Sigma W^T with W = I
    proj = projection.project(np.array([[0.0, 0.0, 2.0]]), ls, q, np.ones((1, 1)), np.zeros((1, 1)),
                              identity_camera(64, 64))
    Sig = proj.M[0]
    assert np.allclose(emp, Sig, rtol=0, atol=0.03 * np.abs(Sig).max())


def test_gather_rows_zeroes_new_state():
    v = np.arange(12.0).reshape(4, 3)
    out = training.gather_rows(v, [0, 0, 2, 3, 3], [0, 1, 0, 2, 2], zero_new=True)
    assert out.tolist() == [[0, 1, 2], [0, 0, 0], [6, 7, 8], [0, 0, 0], [0, 0, 0]]
    out = training.gather_rows(v, [0, 0, 2], [0, 1, 0], zero_new=False)
    assert out.tolist() == [[0, 1, 2], [0, 1, 2], [6, 7, 8]]


def test_cosine_lr_endpoints():
    assert training.cosine_lr(0, 100, 0.01, 1e-5) == pytest.approx(0.01)
    assert training.cosine_lr(100, 100, 0.01, 1e-5) == pytest.approx(1e-5)
    assert training.cosine_lr(50, 100, 0.01, 1e-5) == pytest.approx(0.5 * (0.01 + 1e-5))
