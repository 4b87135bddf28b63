"""Full-size workloads in the launch configuration the benchmark times.

At these sizes the oracle cannot render whole frames in test time, so the
checks are
* the rendered field on sampled windows of every view against the FP64 oracle
  restricted to those windows (relative L2 <= 1e-4);
* the tile lists against the oracle's single-precision binning, bit for bit:
  every tile of the 1080p frame and of two views of the 16-view ring, and
  sampled tiles of the 2160p views;
* the fused loss against the intensities the same call returned;
* the gradient against a central difference of the loss along the gradient
  direction with the means held fixed (a property that holds at any size).
The propagation at the full padded size is checked in test_gpu_asm.py.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import binning, projection, raster
from paper_2506_08350_amd import _lib, api
from scenegen import make_workload
from tests.gpu_helpers import announce, cplx, rel_l2

pytestmark = pytest.mark.gpu

WINDOWS = ((0.25, 0.3), (0.5, 0.5), (0.7, 0.8))   # fractional (row, column) of sampled windows
WIN = (40, 64)


def _renderer(w, cap_factor=1.25, want_cap=None):
    cams = w.cameras
    o = api.Optics(w.optics.wavelengths, w.optics.distances, w.optics.pitch, w.optics.pad, w.optics.band_limit)
    H, W = cams[0].height, cams[0].width
    params = {k: torch.from_numpy(a).cuda() for k, a in zip(api.PARAM_NAMES, w.scene.arrays())}
    cam_t = api.pack_cameras(cams)
    r = api.Renderer(H, W, o, n_views=len(cams), max_gaussians=w.scene.n, max_pairs=want_cap or (1 << 26))
    r.forward(params, cam_t, want_field=False, want_intensity=False)
    st, need = r.read_status()
    if st != 0 or want_cap is None:
        del r
        r = api.Renderer(H, W, o, n_views=len(cams), max_gaussians=w.scene.n, max_pairs=int(need * cap_factor) + 4096)
    return r, params, cam_t


def _window_checks(w, field, r):
    sc = w.scene
    H, W = w.cameras[0].height, w.cameras[0].width
    U = field
    for b, cam in enumerate(w.cameras):
        p = projection.project(sc.means, sc.log_scales, sc.quats, sc.amp, sc.phase, cam)
        fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam)
        for fr, fc in WINDOWS[: (3 if len(w.cameras) <= 4 else 1)]:
            r0, c0 = int(fr * H), int(fc * W)
            win = (r0, r0 + WIN[0], c0, c0 + WIN[1])
            res = raster.render_field(p, sc.opacity, fp, W, H, oracle.DEFAULT, window=win)
            got = cplx(U[b, :, win[0]:win[1], win[2]:win[3]])
            ref = res.U[:, win[0]:win[1], win[2]:win[3]]
            assert rel_l2(got, ref) < 1e-4, (b, win)


def _tile_checks(w, r):
    """Sampled tiles: the sorted Gaussian list of the tile equals the oracle's."""
    sc = w.scene
    H, W = w.cameras[0].height, w.cameras[0].width
    tx, ty = (W + 15) // 16, (H + 15) // 16
    n_tiles = tx * ty
    ranges = r.region(_lib.REGION_TILE_RANGES, torch.int32).cpu().numpy().view(np.uint32).reshape(-1, 2)
    vals = r.region(_lib.REGION_PAIR_VALUES, torch.int32)
    for b, cam in enumerate(w.cameras[:4]):
        fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam, 16, 16, oracle.DEFAULT.k_sigma,
                                    sc.opacity, oracle.DEFAULT.alpha_min)
        for (fr, fc) in WINDOWS:
            t_r, t_c = int(fr * ty), int(fc * tx)
            t = b * n_tiles + t_r * tx + t_c
            ref = binning.tile_members(fp, t_c, t_r)
            s, e = ranges[t]
            got = vals[int(s):int(e)].cpu().numpy().view(np.uint32).astype(np.int64) - b * sc.n
            assert np.array_equal(got, ref), (b, t)


def _full_list_check(w, r, views):
    """Every (view, tile) run of the listed views, and its range, against the
    oracle's binning of that view (bit-exact; pairs are selected on the
    device, so only one view's list is copied back)."""
    sc = w.scene
    thr = oracle.DEFAULT
    H, W = w.cameras[0].height, w.cameras[0].width
    tx, ty = (W + 15) // 16, (H + 15) // 16
    T = tx * ty
    b = int(T - 1).bit_length()
    n = r.read_status()[1]
    keys = r.region(_lib.REGION_PAIR_KEYS, torch.int32)[:n]
    vals = r.region(_lib.REGION_PAIR_VALUES, torch.int32)[:n]
    ranges = r.region(_lib.REGION_TILE_RANGES, torch.int32).view(-1, 2)
    for v in views:
        fp = binning.fp32_footprint(sc.means, sc.log_scales, sc.quats, w.cameras[v], 16, 16, thr.k_sigma,
                                    sc.opacity, thr.alpha_min)
        ref = binning.bin_pairs([fp], W, H)
        sel = torch.nonzero((keys >> b) == v).squeeze(1)
        tiles, order = torch.sort(keys[sel] & ((1 << b) - 1), stable=True)
        gauss = (vals[sel][order] - v * sc.n).cpu().numpy()
        assert np.array_equal(tiles.cpu().numpy(), ref["tile_key"].astype(np.int64)), v
        assert np.array_equal(gauss, ref["gauss"].astype(np.int64)), v
        # the ranges delimit each run inside the whole list
        rg = ranges[v * T:(v + 1) * T].cpu().numpy().view(np.uint32).astype(np.int64)
        ref_len = ref["ranges"][:, 1] - ref["ranges"][:, 0]
        assert np.array_equal(np.where(ref_len > 0, rg[:, 1] - rg[:, 0], 0), ref_len), v
        live = np.nonzero(ref_len)[0]
        idx = np.repeat(rg[live, 0] - np.cumsum(ref_len[live]) + ref_len[live], ref_len[live]) + np.arange(
            int(ref_len.sum()))
        run_vals = vals[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.int64) - v * sc.n
        assert np.array_equal(run_vals, ref["gauss"].astype(np.int64)), v


def _directional_check(r, params, cam_t, target, loss0, grads):
    gnorm2 = sum(float((grads[k].double() ** 2).sum()) for k in api.PARAM_NAMES)
    d = {k: grads[k] / np.sqrt(gnorm2) for k in api.PARAM_NAMES}
    h = 2e-3
    losses = []
    for sgn in (1.0, -1.0):
        pp = {k: (params[k] + sgn * h * d[k]).contiguous() for k in api.PARAM_NAMES}
        out = r.forward(pp, cam_t, want_field=False, want_intensity=False, target=target)
        losses.append(float(out["loss"]))
    fd = (losses[0] - losses[1]) / (2 * h)
    an = np.sqrt(gnorm2)
    assert abs(fd - an) < 0.1 * an, (fd, an)


def test_forward_backward_1080p_100k():
    w = make_workload("c3")
    announce("workload 1080p 100k fwd+bwd")
    r, params, cam_t = _renderer(w)
    target = torch.from_numpy(w.targets).cuda()
    out = r.forward(params, cam_t, want_field=True, want_intensity=True, target=target)
    grads = r.backward(params, cam_t)
    torch.cuda.synchronize()
    assert r.read_status()[0] == 0
    I = out["intensity"].double()
    ref_loss = float(((I - target.double()) ** 2).mean())
    assert abs(float(out["loss"]) - ref_loss) < 1e-5 * ref_loss
    _window_checks(w, out["field"], r)
    _full_list_check(w, r, [0])
    for k in api.PARAM_NAMES:
        assert torch.isfinite(grads[k]).all(), k


def test_gradient_direction_1080p_100k():
    """Directional derivative at full size along the gradient with the means
    held fixed.  Moving means reorders depths, and at 100,000 Gaussians the
    jumps from depth swaps outweigh the derivative; every other parameter
    leaves the sort order alone, and the remaining support/termination jumps
    are orders of magnitude smaller than the signal."""
    w = make_workload("c3")
    announce("workload 1080p 100k directional derivative")
    r, params, cam_t = _renderer(w)
    target = torch.from_numpy(w.targets).cuda()
    out = r.forward(params, cam_t, want_field=False, want_intensity=False, target=target)
    grads = r.backward(params, cam_t)
    torch.cuda.synchronize()
    grads["means"] = torch.zeros_like(grads["means"])
    _directional_check(r, params, cam_t, target, float(out["loss"]), grads)


def test_batched_16_views_ring_500k():
    w = make_workload("c4")
    announce("workload 16 views 500k")
    r, params, cam_t = _renderer(w)
    target = torch.from_numpy(w.targets).cuda()
    out = r.forward(params, cam_t, want_field=True, want_intensity=False, target=target)
    grads = r.backward(params, cam_t)
    torch.cuda.synchronize()
    st, need = r.read_status()
    assert st == 0
    counts = [int(np.count_nonzero(binning.fp32_footprint(w.scene.means, w.scene.log_scales, w.scene.quats,
                                                          c)["visible"])) for c in w.cameras[:3]]
    assert len(set(counts)) > 1      # uneven post-culling counts per view
    _window_checks(w, out["field"], r)
    _tile_checks(w, r)
    _full_list_check(w, r, [0, 9])
    for k in api.PARAM_NAMES:
        assert torch.isfinite(grads[k]).all(), k


def test_four_views_2160p_2m_16_planes():
    """The largest configuration: 2,000,000 Gaussians, four yawed views of
    2160 x 3840, pitch 4 um, 16 planes (padded 4320 x 7680: rows of 7680,
    columns of 4320 as two transforms of 2160)."""
    w = make_workload("c5")
    announce("workload 4 views 2160p 2m 16 planes")
    r, params, cam_t = _renderer(w, cap_factor=1.05)
    B, L, K, H, W = r.B, r.L, r.K, r.H, r.W
    gen = torch.Generator(device="cuda").manual_seed(1005 + 10_000)
    target = torch.rand((B, L, K, H, W), generator=gen, device="cuda")
    target_sum = float(target.double().sum())
    out = r.forward(params, cam_t, want_field=True, want_intensity=True, target=target)
    torch.cuda.synchronize()
    assert float(target.double().sum()) == target_sum
    assert r.read_status()[0] == 0
    I = out["intensity"]
    assert torch.isfinite(out["field"]).all() and torch.isfinite(I).all()
    # the fused loss: per-row sums first, then the reduction
    rows = ((I - target) ** 2).sum(dim=-1).double().reshape(-1)
    part = r.region(_lib.REGION_LOSS_PARTIAL, torch.float32)[:rows.numel()].double()
    bad = torch.nonzero(~torch.isclose(part, rows, rtol=1e-4, atol=1e-3)).reshape(-1)
    assert bad.numel() == 0, (bad.numel(), bad[:8].tolist(), part[bad[:4]].tolist(), rows[bad[:4]].tolist())
    ref_loss = float(rows.sum()) / I.numel()
    loss_before = float(out["loss"])
    assert abs(loss_before - ref_loss) < 1e-5 * ref_loss
    sums_before = [float(t.double().sum()) for t in (I, target)]
    grads = r.backward(params, cam_t)
    torch.cuda.synchronize()
    # the backward leaves every caller buffer it does not own untouched
    assert float(out["loss"]) == loss_before
    assert [float(t.double().sum()) for t in (I, target)] == sums_before
    _window_checks(w, out["field"], r)
    _tile_checks(w, r)
    for k in api.PARAM_NAMES:
        assert torch.isfinite(grads[k]).all(), k
    # one (wavelength, plane) pair of one view through the full padded propagation
    U = cplx(out["field"][1, 2])
    del out, I
    ref = oracle.propagate(U, w.optics.wavelengths[2], w.optics.distances[11], w.optics.pitch, w.optics.pad,
                           w.optics.band_limit)
    prop, _ = r.propagate(r.forward(params, cam_t, want_field=True, want_intensity=False)["field"],
                          want_intensity=False)
    assert rel_l2(cplx(prop[1, 2, 11]), ref) < 1e-4
