"""GPU angular-spectrum propagation and its adjoint against the FP64 oracle.

Tolerance: complex-field relative L2 <= 1e-4 (FP32 on the GPU against FP64).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from scenegen import Optics, identity_camera
from tests.gpu_helpers import announce, cplx, make_renderer, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def _to_gpu(U):
    return torch.from_numpy(np.stack([U.real, U.imag], -1).astype(np.float32)).cuda()


@pytest.mark.parametrize("H,W,pad,mode,lams,zs,pitch", [
    (24, 40, 2, 2, (639e-9, 473e-9), (0.5e-3, 1e-3, -2e-3), 8e-6),     # ragged, several planes
    (45, 36, 2, 1, (515e-9,), (1e-3,), 8e-6),                           # odd height: radix 3, 5
    (64, 64, 1, 2, (515e-9,), (2e-3,), 8e-6),                           # no padding
    (30, 50, 2, 2, (515e-9, 639e-9, 473e-9), (4e-6, 1e-5), 0.3e-6),     # both band masks active
    (128, 128, 2, 2, (515e-9,), (1e-3,), 8e-6),                         # the 128x128 workload
])
def test_propagate_matches_oracle(H, W, pad, mode, lams, zs, pitch):
    announce(f"propagate H={H} W={W} pad={pad} mode={mode} L={len(lams)} K={len(zs)}")
    opt = Optics(lams, zs, pitch, pad, mode)
    cam = identity_camera(W, H)
    r = make_renderer([cam], opt, 1)
    U = _field((1, len(lams), H, W), 11)
    prop, inten = r.propagate(_to_gpu(U))
    torch.cuda.synchronize()
    u_gpu = cplx(prop)
    for li, lam in enumerate(lams):
        for ki, z in enumerate(zs):
            ref = oracle.propagate(U[0, li], lam, z, pitch, pad, mode)
            err = rel_l2(u_gpu[0, li, ki], ref)
            assert err < TOL, (li, ki, err)
            ierr = rel_l2(inten[0, li, ki].cpu().numpy(), np.abs(ref) ** 2)
            assert ierr < 2 * TOL, (li, ki, ierr)


def test_plane_wave_phase():
    announce("plane wave")
    H, W = 32, 48
    lam = 515e-9
    opt = Optics((lam,), (0.5e-3, 1.7e-3), 8e-6, 1, 2)
    r = make_renderer([identity_camera(W, H)], opt, 1)
    U = np.full((1, 1, H, W), 0.6 - 0.3j)
    prop, _ = r.propagate(_to_gpu(U))
    u = cplx(prop)
    for ki, z in enumerate(opt.distances):
        expected = U[0, 0] * np.exp(2j * math.pi * z / lam)
        assert np.max(np.abs(u[0, 0, ki] - expected)) < 1e-5


def test_adjoint_matches_oracle_and_dot_product():
    announce("adjoint")
    H, W = 36, 20
    lams, zs = (639e-9, 515e-9), (0.5e-3, 1.5e-3, 2e-3)
    opt = Optics(lams, zs, 8e-6, 2, 2)
    r = make_renderer([identity_camera(W, H)], opt, 1)
    G = _field((1, 2, 3, H, W), 5)
    gU = cplx(r.propagate_adjoint(_to_gpu(G)))
    for li, lam in enumerate(lams):
        ref = sum(oracle.propagate_adjoint(G[0, li, ki], lam, z, 8e-6, 2, 2) for ki, z in enumerate(zs))
        assert rel_l2(gU[0, li], ref) < TOL
    # <A u, v> = <u, A^H v> with the GPU on both sides
    U = _field((1, 2, H, W), 6)
    prop, _ = r.propagate(_to_gpu(U), want_intensity=False)
    lhs = np.vdot(G, cplx(prop))
    rhs = np.vdot(gU, U)
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


@pytest.mark.parametrize("cols", [1, 2, 4])
def test_full_size_workload_geometry(cols):
    """1080 x 1920 field, padded 2160 x 3840, three wavelengths, four planes,
    with each column-pass variant (columns per workgroup); one wavelength and
    two planes of the propagation, and the adjoint of one wavelength, are
    checked against the oracle in full."""
    announce(f"propagate 1080x1920, {cols} columns per workgroup")
    H, W = 1080, 1920
    lams, zs = (639e-9, 515e-9, 473e-9), (0.5e-3, 1e-3, 1.5e-3, 2e-3)
    opt = Optics(lams, zs, 8e-6, 2, 2)
    r = make_renderer([identity_camera(W, H)], opt, 1, cols_per_block=cols)
    rng = np.random.default_rng(3)
    U = (rng.uniform(0, 1, (1, 3, H, W)) * np.exp(2j * np.pi * rng.uniform(0, 1, (1, 3, H, W))))
    prop, inten = r.propagate(_to_gpu(U))
    torch.cuda.synchronize()
    for li, ki in ((0, 0), (2, 3)):
        ref = oracle.propagate(U[0, li], lams[li], zs[ki], 8e-6, 2, 2)
        got = cplx(prop[0, li, ki])
        assert rel_l2(got, ref) < TOL
    G = (rng.normal(size=(1, 3, 4, H, W)) + 1j * rng.normal(size=(1, 3, 4, H, W)))
    back = r.propagate_adjoint(torch.from_numpy(np.stack([G.real, G.imag], -1).astype(np.float32)).cuda())
    torch.cuda.synchronize()
    ref = sum(oracle.propagate_adjoint(G[0, 1, k], lams[1], zs[k], 8e-6, 2, 2) for k in range(4))
    assert rel_l2(cplx(back[0, 1]), ref) < TOL


@pytest.mark.parametrize("W", [2560, 3840])
def test_wide_rows_propagation_and_fused_loss(W):
    """Rows whose two LDS buffers exceed 64 KiB (generic transforms of 5120 and
    7680 points): one propagated plane against the oracle, and the fused MSE
    row sums of an empty scene, whose intensities are zero, against the sums of
    the squared targets."""
    from paper_2506_08350_amd import _lib, api
    from scenegen import make_gaussians
    from tests.gpu_helpers import to_device

    announce(f"wide rows W={W}")
    H = 6
    opt = Optics((515e-9,), (1e-3, 2e-3), 8e-6, 2, 2)
    cam = identity_camera(W, H)
    r = make_renderer([cam], opt, 4)
    U = _field((1, 1, H, W), 11)
    prop, _ = r.propagate(_to_gpu(U), want_intensity=False)
    torch.cuda.synchronize()
    assert rel_l2(cplx(prop[0, 0, 1]), oracle.propagate(U[0, 0], 515e-9, 2e-3, 8e-6, 2, 2)) < TOL
    gen = torch.Generator(device="cuda").manual_seed(3)
    tgt = torch.rand((1, 1, 2, H, W), generator=gen, device="cuda")
    sums_before = [float(t.double().sum()) for t in (tgt, prop)]
    out = r.forward(to_device(make_gaussians(0, 1, 9)), api.pack_cameras([cam]), want_field=False,
                    want_intensity=True, target=tgt)
    torch.cuda.synchronize()
    # the forward writes none of the caller's buffers it was not given
    assert [float(t.double().sum()) for t in (tgt, prop)] == sums_before
    assert float(out["intensity"].abs().max()) == 0.0
    part = r.region(_lib.REGION_LOSS_PARTIAL, torch.float32)[:2 * H].double()
    rows = (tgt.double() ** 2).sum(-1).reshape(-1)
    assert torch.allclose(part, rows, rtol=1e-5), (part[:4].tolist(), rows[:4].tolist())
    assert abs(float(out["loss"]) - float((tgt.double() ** 2).mean())) < 1e-5


def test_tuned_rows_without_padding():
    """Rows of 3840 with pad factor 1 (the tuned row transforms with every
    input live and every output kept; rows of 7680 always come from a padded
    width of 3840, the largest the plans take): one propagated plane and the
    adjoint against the oracle."""
    announce("tuned rows, no padding, W=3840")
    H, W, lam, zs = 4, 3840, 515e-9, (1e-3, 2e-3)
    opt = Optics((lam,), zs, 8e-6, 1, 2)
    r = make_renderer([identity_camera(W, H)], opt, 1)
    U = _field((1, 1, H, W), 41)
    prop, _ = r.propagate(_to_gpu(U), want_intensity=False)
    torch.cuda.synchronize()
    assert rel_l2(cplx(prop[0, 0, 1]), oracle.propagate(U[0, 0], lam, zs[1], 8e-6, 1, 2)) < TOL
    G = _field((1, 1, 2, H, W), 42)
    back = r.propagate_adjoint(_to_gpu(G))
    torch.cuda.synchronize()
    ref = sum(oracle.propagate_adjoint(G[0, 0, k], lam, z, 8e-6, 1, 2) for k, z in enumerate(zs))
    assert rel_l2(cplx(back[0, 0]), ref) < TOL


@pytest.mark.parametrize("views,zs", [
    (1, (1e-3,)),                                                  # one plane: no copy in flight
    (2, (0.4e-3, 0.9e-3, 1.3e-3, 1.7e-3, 2.2e-3, 2.6e-3, 3e-3)),   # seven planes, two views
])
def test_full_size_plane_counts_and_views(views, zs):
    """At 1080 x 1920 with two columns per workgroup the adjoint copies each
    plane's input into LDS while the previous plane's transform runs, and
    the plane parameters are read by scalar loads: one plane, seven planes,
    and two views (group indexing across views).  Sampled planes of the
    propagation and the full adjoint of the last view against the oracle."""
    announce(f"propagate 1080x1920, {views} views, {len(zs)} planes")
    H, W = 1080, 1920
    lam, K = 515e-9, len(zs)
    opt = Optics((lam,), zs, 8e-6, 2, 2)
    r = make_renderer([identity_camera(W, H)] * views, opt, 1, cols_per_block=2)
    rng = np.random.default_rng(9)
    U = rng.uniform(0, 1, (views, 1, H, W)) * np.exp(2j * np.pi * rng.uniform(0, 1, (views, 1, H, W)))
    prop, _ = r.propagate(_to_gpu(U), want_intensity=False)
    torch.cuda.synchronize()
    for v, k in {(0, 0), (views - 1, K - 1)}:
        ref = oracle.propagate(U[v, 0], lam, zs[k], 8e-6, 2, 2)
        assert rel_l2(cplx(prop[v, 0, k]), ref) < TOL, (v, k)
    del prop
    G = rng.normal(size=(views, 1, K, H, W)).astype(np.float32) + 1j * rng.normal(size=(views, 1, K, H, W)).astype(
        np.float32)
    back = r.propagate_adjoint(torch.from_numpy(np.stack([G.real, G.imag], -1)).cuda())
    torch.cuda.synchronize()
    v = views - 1
    ref = sum(oracle.propagate_adjoint(G[v, 0, k].astype(np.complex128), lam, zs[k], 8e-6, 2, 2) for k in range(K))
    assert rel_l2(cplx(back[v, 0]), ref) < TOL


@pytest.mark.parametrize("plans", [(1, 0), (2, 0), (0, 1), (0, 2), (0, 3)])
def test_radix_schedules_at_full_size(plans):
    """Every non-default radix schedule of the tuned transforms (rows of 3840,
    columns of 2160) at the 1080 x 1920 x 3 wavelengths x 4 planes geometry:
    one propagated plane against the oracle, and the fused training step's
    dL/dU for one wavelength against the oracle's adjoint propagation of
    2 u dL/dI computed from the GPU's own field (the fused inverse row pass
    runs the row schedule forwards and backwards)."""
    from paper_2506_08350_amd import _lib, api
    from scenegen import make_gaussians, make_targets
    from tests.gpu_helpers import to_device

    announce(f"radix schedules {plans} at 1080x1920")
    H, W = 1080, 1920
    lams, zs = (639e-9, 515e-9, 473e-9), (0.5e-3, 1e-3, 1.5e-3, 2e-3)
    opt = Optics(lams, zs, 8e-6, 2, 2)
    cam = identity_camera(W, H)
    r = make_renderer([cam], opt, 2000, fft_plans=plans)
    rng = np.random.default_rng(5)
    U = rng.uniform(0, 1, (1, 3, H, W)) * np.exp(2j * np.pi * rng.uniform(0, 1, (1, 3, H, W)))
    prop, _ = r.propagate(_to_gpu(U), want_intensity=False)
    torch.cuda.synchronize()
    assert rel_l2(cplx(prop[0, 2, 1]), oracle.propagate(U[0, 2], lams[2], zs[1], 8e-6, 2, 2)) < TOL
    del prop
    sc = make_gaussians(2000, 3, 77, x_range=(-0.3, 0.3), y_range=(-0.2, 0.2), log_scale_mean=-3.5)
    tg = make_targets((1, 3, 4, H, W), 78)
    r.train_step(to_device(sc), api.pack_cameras([cam]), torch.from_numpy(tg).cuda())
    torch.cuda.synchronize()
    Uf = cplx(r.region(_lib.REGION_FIELD, torch.float32).view(1, 3, H, W, 2))
    GU = cplx(r.region(_lib.REGION_GRAD_FIELD, torch.float32).view(1, 3, H, W, 2))
    li, numel = 1, tg.size
    ref = np.zeros((H, W), np.complex128)
    for k, z in enumerate(zs):
        u = oracle.propagate(Uf[0, li], lams[li], z, 8e-6, 2, 2)
        I = np.abs(u) ** 2
        ref += oracle.propagate_adjoint(2.0 * u * (2.0 * (I - tg[0, li, k]) / numel), lams[li], z, 8e-6, 2, 2)
    assert rel_l2(GU[0, li], ref) < TOL


@pytest.mark.parametrize("H,mode,cols", [(1080, 2, 2), (1080, 1, 4), (2160, 2, 2), (2160, 2, 1), (2160, 1, 2),
                                         (2160, 0, 0)])
def test_tuned_columns_with_band_masks(H, mode, cols):
    """Columns of 2160 and of 4320 (tuned transforms; 4320 as two of 2160,
    one or two columns per workgroup) where the band limits mask bins: a
    pitch of 0.2 um puts evanescent bins on the grid, band mode 1 cuts them,
    mode 2 also applies the sampling limit, and mode 0 keeps their decaying
    continuation (which the generic transforms form).  Narrow rows keep the
    oracle cheap; two planes of two wavelengths and the adjoint."""
    announce(f"masked columns H={H} mode={mode} cols={cols}")
    W, pitch = 64, 0.2e-6
    lams, zs = (515e-9, 639e-9), (4e-6, 1e-5)
    opt = Optics(lams, zs, pitch, 2, mode)
    r = make_renderer([identity_camera(W, H)], opt, 1, cols_per_block=cols)
    U = _field((1, 2, H, W), 31)
    prop, _ = r.propagate(_to_gpu(U), want_intensity=False)
    torch.cuda.synchronize()
    for li, ki in ((0, 0), (1, 1)):
        ref = oracle.propagate(U[0, li], lams[li], zs[ki], pitch, 2, mode)
        assert rel_l2(cplx(prop[0, li, ki]), ref) < TOL, (li, ki)
    G = _field((1, 2, 2, H, W), 32)
    back = r.propagate_adjoint(_to_gpu(G))
    torch.cuda.synchronize()
    ref = sum(oracle.propagate_adjoint(G[0, 1, k], lams[1], zs[k], pitch, 2, mode) for k in range(2))
    assert rel_l2(cplx(back[0, 1]), ref) < TOL


_LAMS_2160P, _ZS_2160P = (515e-9,), (0.8e-3, 1.6e-3)


@pytest.fixture(scope="module")
def field_2160p():
    """A 2160 x 3840 field (padded 4320 x 7680), the adjoint inputs of two
    planes, and the oracle's propagated second plane and summed adjoint,
    computed once for every radix schedule below."""
    H, W = 2160, 3840
    rng = np.random.default_rng(21)
    U = rng.uniform(0, 1, (1, 1, H, W)) * np.exp(2j * np.pi * rng.uniform(0, 1, (1, 1, H, W)))
    G = (rng.normal(size=(1, 1, 2, H, W)) + 1j * rng.normal(size=(1, 1, 2, H, W))).astype(np.complex64)
    lam = _LAMS_2160P[0]
    prop_ref = oracle.propagate(U[0, 0], lam, _ZS_2160P[1], 8e-6, 2, 2)
    adj_ref = sum(oracle.propagate_adjoint(G[0, 0, k].astype(np.complex128), lam, z, 8e-6, 2, 2)
                  for k, z in enumerate(_ZS_2160P))
    return U, G, prop_ref, adj_ref


@pytest.mark.parametrize("plans,cols", [((0, 0), 2), ((1, 0), 2), ((2, 0), 2), ((0, 1), 2), ((0, 2), 2), ((0, 3), 2),
                                        ((0, 0), 1), ((0, 3), 1)])
def test_radix_schedules_at_2160p(field_2160p, plans, cols):
    """The tuned transforms of the 2160 x 3840 geometry (rows of 7680 with
    512 threads; columns of 4320 as two transforms of 2160, even and odd
    bins, combined with w^-n, one or two columns per workgroup), every radix
    schedule: one propagated plane and the adjoint summed over two planes
    against the oracle."""
    announce(f"radix schedules {plans}, {cols} columns per workgroup at 2160x3840")
    U, G, prop_ref, adj_ref = field_2160p
    H, W = U.shape[2:]
    opt = Optics(_LAMS_2160P, _ZS_2160P, 8e-6, 2, 2)
    r = make_renderer([identity_camera(W, H)], opt, 1, fft_plans=plans, cols_per_block=cols)
    prop, _ = r.propagate(_to_gpu(U), want_intensity=False)
    torch.cuda.synchronize()
    assert rel_l2(cplx(prop[0, 0, 1]), prop_ref) < TOL
    del prop
    back = r.propagate_adjoint(torch.from_numpy(np.stack([G.real, G.imag], -1)).cuda())
    torch.cuda.synchronize()
    assert rel_l2(cplx(back[0, 0]), adj_ref) < TOL


@pytest.mark.parametrize("row_plan", [0, 1, 2])
def test_fused_training_rows_at_2160p(row_plan):
    """The fused inverse row pass of 7680 (inverse transform, |u|^2, MSE, then
    G = 2 u dL/dI transformed forward again with the reversed schedule) in a
    training step at 2160 x 3840, one plane: dL/dU against the oracle's
    adjoint propagation of 2 u dL/dI computed from the GPU's own field."""
    from paper_2506_08350_amd import _lib, api
    from scenegen import make_gaussians, make_targets
    from tests.gpu_helpers import to_device

    announce(f"fused training rows, row plan {row_plan}, 2160x3840")
    H, W = 2160, 3840
    lam, z = 515e-9, 1.2e-3
    opt = Optics((lam,), (z,), 8e-6, 2, 2)
    cam = identity_camera(W, H)
    r = make_renderer([cam], opt, 3000, fft_plans=(row_plan, 0))
    sc = make_gaussians(3000, 1, 91, x_range=(-0.3, 0.3), y_range=(-0.2, 0.2), log_scale_mean=-3.0)
    tg = make_targets((1, 1, 1, H, W), 92)
    r.train_step(to_device(sc), api.pack_cameras([cam]), torch.from_numpy(tg).cuda())
    torch.cuda.synchronize()
    Uf = cplx(r.region(_lib.REGION_FIELD, torch.float32).view(1, 1, H, W, 2))
    GU = cplx(r.region(_lib.REGION_GRAD_FIELD, torch.float32).view(1, 1, H, W, 2))
    u = oracle.propagate(Uf[0, 0], lam, z, 8e-6, 2, 2)
    ref = oracle.propagate_adjoint(2.0 * u * (2.0 * (np.abs(u) ** 2 - tg[0, 0, 0]) / tg.size), lam, z, 8e-6, 2, 2)
    assert rel_l2(GU[0, 0], ref) < TOL
