#!/usr/bin/env python
"""Throughput of the complex-hologram hot path on one MI355X.

A step is one pass of the whole path over one batch: projection and culling,
tile binning and sort, complex compositing, band-limited ASM propagation to
every plane, |u|^2, the MSE against seeded targets, and the full backward to
the Gaussian parameters.  The headline workload is 100,000 Gaussians rendered
at 1080 x 1920 for three wavelengths and propagated to four planes (one view
per step).  Inputs are synthetic and resident in HBM before timing starts.
The timed steps replay the whole training step captured once in a HIP graph
(``--eager`` times eager launches instead); per-kernel times come from a
separate eager pass with HIP events on the launch stream.

Besides the headline line's own keys, the default run adds:
  cpu_baseline     the FP64 oracle on the host's cores (up to 16 worker
                   processes), full frame: compositing forward and backward
                   over a 4 x 4 grid of windows, then the 12 (wavelength,
                   plane) propagations and their adjoints
  copy_bandwidth   a plain 1 GiB device-to-device copy, next to the 8 TB/s
                   vendor figure
  raster_work      (pixel, pair) tests and included pairs per frame, the
                   algorithmic work the raster roofline is priced on
  ring_16_views    16 views of a 500,000-Gaussian ring scene, 8 planes: the
                   batched step (autotuned, captured in a HIP graph) against
                   the same views one at a time
  views_2160p      4 views of 2,000,000 Gaussians at 2160 x 3840, 16 planes
  torch_fft_asm    the forward propagation of the headline frame written
                   with torch.fft (rocFFT), an external reference point

Prints one JSON line.  ``--gpus N`` with N > 1 is not supported: this build
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
# FP32 vector peak of MI355X, 157.3 TFLOP/s, in lane-operations per second
# (a fused multiply-add is one operation, two flops): 256 CUs x 2.4 GHz x
# 2 wave64 VALU instructions per CU-cycle x 64 lanes.
VALU_PEAK_GOPS = 256 * 2.4 * 2 * 64

# Arithmetic of the method per (pixel, pair), single-plane compositing with
# three wavelengths (operations of the formulas, an FMA counted once):
#   test of one pair at one pixel: d = p - mu (2), power = (A dx^2 + C dy^2)/2
#     + B dx dy (7), exp (1), o e^-power (1), clamp (1), three support
#     comparisons (3)                                                  = 15
#   forward, included pair: a T (1), U_l += v_l a T (2 per wavelength),
#     T *= 1 - a (2), last index (1)                                   = 10
#   backward, included pair: T / (1 - a) (3), a T (1); per wavelength
#     D = sum Re(conj(G) v) (2) and dL/dv (2) (12); dL/da = D - K and the
#     update K += a (D - K) of K = sum Re(conj(G) B) (2); dL/da T,
#     dL/dpower, dL/do (3), dL/dconic (5), dL/dmu (6), twelve gradient
#     sums (12)                                                        = 44
OPS_TEST, OPS_FWD_INC, OPS_BWD_INC = 15, 10, 44


def kernel_bytes(name, B, L, K, H, W, pH, pW, train, fused=True):
    """Algorithmic HBM bytes of one launch of each propagation kernel.  train:
    the inverse row pass reads the targets; fused: it also writes the
    adjoint's row spectra (MSE), else it stores u and I for the loss."""
    c = 8  # complex64
    if train and fused:
        inv_row = pW * c + pW * c + W * 4
    elif train:
        inv_row = pW * c + W * c + W * 4
    else:
        inv_row = pW * c + W * 4
    table = {
        "rows_forward": B * L * H * (W + pW) * c,
        "cols_forward": B * L * (H * pW + K * H * pW) * c,
        "rows_inverse": B * L * K * H * inv_row,
        "cols_adjoint": B * L * (K * H * pW + H * pW) * c,
        "rows_adjoint_out": B * L * H * (pW + W) * c,
    }
    return table.get(name)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_step_c3_1080p_100k.md")
VALU_PROFILE = os.path.join(ROOT, "profiles", "valu_step_c3_1080p_100k.md")

# HIP sources each timed kernel is built from (a change invalidates its counters)
KERNEL_SOURCES = {
    "rows_forward": ("asm.hip", "asm_tuned.hip", "fft.h", "internal.h"),
    "cols_forward": ("asm.hip", "asm_tuned.hip", "fft.h", "internal.h"),
    "rows_inverse": ("asm.hip", "asm_tuned.hip", "fft.h", "internal.h"),
    "cols_adjoint": ("asm.hip", "asm_tuned.hip", "fft.h", "internal.h"),
    "rows_adjoint_out": ("asm.hip", "asm_tuned.hip", "fft.h", "internal.h"),
    "raster_forward": ("raster.hip", "raster_common.h", "internal.h"),
    "raster_backward": ("raster.hip", "raster_common.h", "internal.h"),
}
VALU_NAMES = {"cols_adjoint": "k_cols_adjoint_t", "cols_forward": "k_cols_forward_t",
              "raster_backward": "k_raster_bwd", "raster_forward": "k_raster_fwd"}


def source_sha256(name):
    import hashlib
    with open(os.path.join(ROOT, "paper_2506_08350_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _profile_rows(path):
    try:
        text = open(path).read()
    except OSError:
        return {}, []
    shas, rows = {}, []
    for line in text.splitlines():
        if line.startswith("source-sha256 "):
            _, name, sha = line.split()
            shas[name] = sha
        rows.append([c.strip(" `") for c in line.strip().strip("|").split("|")])
    return shas, rows


def _sources_unchanged(kernel, shas):
    files = KERNEL_SOURCES.get(kernel)
    return bool(files) and all(shas.get(f) == source_sha256(f) for f in files)


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or
    None when that summary is missing, does not cover the kernel, or any of the
    kernel's sources changed since the counters were taken."""
    shas, rows = _profile_rows(TRAFFIC_PROFILE)
    table = {r[0]: int(r[4]) for r in rows if len(r) == 5 and r[0] and r[4].isdigit()}
    if kernel not in table or not _sources_unchanged(kernel, shas):
        return None
    return table[kernel]


def measured_valu_instructions(kernel):
    """VALU instructions per launch of ``kernel`` (SQ_INSTS_VALU) from the
    committed counter summary, or None when it is missing, does not cover the
    kernel, or any of the kernel's sources changed since."""
    shas, rows = _profile_rows(VALU_PROFILE)
    count = None
    for r in rows:
        if len(r) == 7 and kernel in VALU_NAMES and r[0].startswith(VALU_NAMES[kernel] + "<") and r[2].isdigit():
            count = int(r[2])
    if count is None or not _sources_unchanged(kernel, shas):
        return None
    return count


# ------------------------------------------------------------ CPU baseline --
def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_init(scene, cam, thr, seed):
    global _ORACLE_JOB
    _ORACLE_JOB = (scene, cam, thr, seed)


def _oracle_warm(_):
    import numpy  # noqa: F401
    import oracle  # noqa: F401
    return 0


def _oracle_window(window):
    """Compositing forward and backward of every Gaussian over one window of
    the frame (gradient of the field: seeded normal draws), with the
    projection and its backward.  Returns (seconds, included pairs)."""
    import numpy as np
    import oracle
    from oracle.projection import project_backward
    scene, cam, thr, seed = _ORACLE_JOB
    t0 = time.perf_counter()
    p = oracle.project(scene.means, scene.log_scales, scene.quats, scene.amp, scene.phase, cam)
    fp = oracle.fp32_footprint(scene.means, scene.log_scales, scene.quats, cam, k_sigma=thr.k_sigma)
    res = oracle.render_field(p, scene.opacity, fp, cam.width, cam.height, thr, window=window)
    r0, r1, c0, c1 = window
    rng = np.random.default_rng(seed + r0 * 7919 + c0)
    G = np.zeros_like(res.U)
    G[:, r0:r1, c0:c1] = rng.normal(size=(scene.n_lambda, r1 - r0, c1 - c0))
    d = oracle.render_field_backward(p, scene.opacity, fp, res, G, thr, window=window)
    project_backward(p, scene.quats, scene.amp, scene.phase, cam, *d)
    return time.perf_counter() - t0, int(res.n_contrib[r0:r1, c0:c1].sum())


def _oracle_propagation(job):
    """One (wavelength, plane) propagation of a full field and its adjoint."""
    import numpy as np
    import oracle
    lam, z, pitch, pad, band, shape, seed = job
    rng = np.random.default_rng(seed)
    U = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    t0 = time.perf_counter()
    u = oracle.propagate(U, lam, z, pitch, pad, band)
    oracle.propagate_adjoint(u, lam, z, pitch, pad, band)
    return time.perf_counter() - t0


def cpu_baseline(w, seed=0):
    """The FP64 oracle on the host cores, one full frame of the headline
    workload: its work (the compositing of every pixel, forward and backward,
    and every propagation with its adjoint) is split into independent jobs
    run by a pool of worker processes, one per core up to 16: 16 windows of a
    4 x 4 grid over the frame, then the 12 (wavelength, plane) propagations.
    The frame time is the wall time of the two phases."""
    import multiprocessing as mp

    import oracle

    sc, cam, opt = w.scene, w.cameras[0], w.optics
    H, W = cam.height, cam.width
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    rows = [H * i // 4 for i in range(5)]
    cols = [W * i // 4 for i in range(5)]
    windows = [(rows[i], rows[i + 1], cols[j], cols[j + 1]) for i in range(4) for j in range(4)]
    props = [(lam, z, opt.pitch, opt.pad, opt.band_limit, (H, W), seed + 31 * k)
             for k, (lam, z) in enumerate((l, z) for l in opt.wavelengths for z in opt.distances)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_oracle_init, initargs=(sc, cam, oracle.DEFAULT, seed)) as pool:
        pool.map(_oracle_warm, range(cores))   # workers up and imported before the clock starts
        t0 = time.perf_counter()
        win = pool.map(_oracle_window, windows, chunksize=1)
        t1 = time.perf_counter()
        prop = pool.map(_oracle_propagation, props, chunksize=1)
        t2 = time.perf_counter()
    frame = t2 - t0
    return {
        "value": 1.0 / frame, "unit": "frames/s", "cores": cores, "kind": "oracle",
        "sample": (f"one full frame: FP64 NumPy oracle, {cores} worker processes on {os.cpu_count()} logical CPUs "
                   f"({_cpu_model()}); compositing fwd+bwd of all {sc.n} Gaussians x {sc.n_lambda} wavelengths "
                   f"over a 4x4 grid of windows ({t1 - t0:.1f} s wall, {sum(t for t, _ in win):.1f} s of worker "
                   f"time) + {len(props)} full-size propagations and adjoints ({t2 - t1:.1f} s wall); "
                   f"{frame:.1f} s per frame"),
        "included_pairs": sum(n for _, n in win),
    }


# ------------------------------------------------------------ GPU helpers --
def _events_ms(fn, reps, stream=None):
    """Per-call times (ms) of fn() from HIP events on the current stream."""
    import torch
    stream = stream or torch.cuda.current_stream()
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        out.append(a.elapsed_time(b))
    return out


def copy_bandwidth(mib=1024, reps=10):
    """Read + write bytes per second of a plain device-to-device copy."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ms = statistics.median(_events_ms(lambda: dst.copy_(src), reps))
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2 * (mib << 20) / (ms * 1e-3) / 1e9
    return {"bytes_moved": 2 * (mib << 20), "ms": round(ms, 4), "achieved_gbs": round(gbs, 1),
            "vendor_peak_gbs": HBM_PEAK_GBS, "frac_of_vendor_peak": round(gbs / HBM_PEAK_GBS, 4)}


def raster_walks(r, B, H, W, tile, t_min):
    """(pixel, pair) tests of the forward and of the backward over the last
    forward's frame, from its tile ranges, last-included indices and
    transmittances: a pixel's forward walks its tile list up to its last
    included pair if it terminated, else to the end; its backward replays from
    its last included pair to the start."""
    import torch
    from paper_2506_08350_amd import _lib
    tw, th = tile
    tx, ty = (W + tw - 1) // tw, (H + th - 1) // th
    ranges = r.region(_lib.REGION_TILE_RANGES, torch.int32)[: 2 * B * tx * ty].view(B, ty, tx, 2).long()
    last = r.region(_lib.REGION_LAST, torch.int32)[: B * H * W].view(B, H, W).long()
    tfin = r.region(_lib.REGION_T_FINAL, torch.float32)[: B * H * W].view(B, H, W)
    rows = torch.arange(H, device=last.device) // th
    cols = torch.arange(W, device=last.device) // tw
    rg = ranges[:, rows][:, :, cols]                      # [B, H, W, 2]
    start, end = rg[..., 0], rg[..., 1]
    used = last > 0
    bwd = torch.where(used, last - start, torch.zeros_like(last))
    fwd = torch.where(used & (tfin < t_min), last - start, end - start)
    return int(fwd.sum()), int(bwd.sum())


def _kernel_table(per_launch, B, L, K, H, W, pH, pW, train, fused):
    tot = sum(c * m for c, m in per_launch.values())
    for n, (c, m) in sorted(per_launch.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        b = kernel_bytes(n, B, L, K, H, W, pH, pW, train, fused)
        bw = f"{b / (m * 1e-3) / 1e9:8.1f} GB/s" if b else ""
        print(f"{n:18s} {c:4d} x {m:8.4f} ms  {100 * c * m / tot:5.1f}%  {bw}", file=sys.stderr)


# -------------------------------------------------------- extra workloads --
def bench_ring(steps, warmup, log):
    """16 views of the 500,000-Gaussian ring scene (8 planes): the batched
    training step with the autotuner's configuration, captured in a HIP
    graph, against the same 16 views as 16 single-view training steps with
    the default configuration (eager launches)."""
    import torch

    import scenegen
    from paper_2506_08350_amd import api, autotune

    w = scenegen.make_workload("c4")
    sc, cams, opt = w.scene, w.cameras, w.optics
    B, H, W = len(cams), cams[0].height, cams[0].width
    o = api.Optics(opt.wavelengths, opt.distances, opt.pitch, opt.pad, opt.band_limit)
    params = {k: torch.from_numpy(a).cuda() for k, a in zip(api.PARAM_NAMES, sc.arrays())}
    cam_t = api.pack_cameras(cams)
    target = torch.from_numpy(w.targets).cuda()
    probe = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=1 << 30, tile=(8, 8))
    probe.forward(params, cam_t, want_field=False, want_intensity=False)
    st, need8 = probe.read_status()
    del probe
    torch.cuda.empty_cache()
    cap = int(need8 * 1.05) + 4096   # 8 x 8 tiles need the most pairs
    t0 = time.perf_counter()
    best, entry = autotune.autotune(H, W, o, params, cam_t, target, cap, cache=None)
    tune_s = time.perf_counter() - t0
    log(f"ring: autotuned {best} in {tune_s:.1f} s")
    rb = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=cap, **best)
    rb.train_step(params, cam_t, target)
    st, need = rb.read_status()
    if st != 0:
        raise RuntimeError(f"ring: pair list overflow ({need} > {cap})")
    cap_graph = api.CapturedTrainStep(rb, params, cam_t, target)
    for _ in range(warmup):
        cap_graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cap_graph.replay()
    torch.cuda.synchronize()
    batched_ms = (time.perf_counter() - t0) * 1000.0 / steps
    loss_b = float(cap_graph.loss)
    rb.timing(True)
    rb.train_step(params, cam_t, target)
    torch.cuda.synchronize()
    rb.timing(False)
    kt_b = rb.timing_report()
    del cap_graph, rb
    torch.cuda.empty_cache()

    # the single-view path sized for its largest view (16 x 16 tiles)
    probe = api.Renderer(H, W, o, n_views=1, max_gaussians=sc.n, max_pairs=need + 4096)
    need1 = 0
    for v in range(B):
        probe.forward(params, cam_t[v:v + 1], want_field=False, want_intensity=False)
        need1 = max(need1, probe.read_status()[1])
    del probe
    torch.cuda.empty_cache()
    r1 = api.Renderer(H, W, o, n_views=1, max_gaussians=sc.n, max_pairs=int(need1 * 1.05) + 4096)
    tv = [target[v:v + 1].contiguous() for v in range(B)]

    def sequential():
        for v in range(B):
            r1.train_step(params, cam_t[v:v + 1], tv[v])

    for _ in range(max(1, warmup // 2)):
        sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sequential()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1000.0 / steps
    r1.timing(True)
    sequential()
    torch.cuda.synchronize()
    r1.timing(False)
    kt_s = r1.timing_report()
    for name in sorted(set(kt_b) | set(kt_s), key=lambda n: -kt_b.get(n, (0, 0.0))[1]):
        log(f"ring kernel {name:18s} batched {kt_b.get(name, (0, 0.0))[1]:9.3f} ms   "
            f"16 single views {kt_s.get(name, (0, 0.0))[1]:9.3f} ms")
    del r1
    torch.cuda.empty_cache()
    return {
        "workload": w.name, "gaussians": sc.n, "views_per_step": B, "height": H, "width": W,
        "wavelengths": sc.n_lambda, "planes": len(opt.distances), "pairs": int(need),
        "batched": {"graph": True, "config": {k: list(v) if isinstance(v, tuple) else v for k, v in best.items()},
                    "ms_per_step": round(batched_ms, 3), "frames_per_s": round(B * 1000.0 / batched_ms, 2),
                    "loss": loss_b},
        "sequential_single_view": {"graph": False, "config": "default", "max_view_pairs": int(need1),
                                   "ms_per_16_views": round(seq_ms, 3),
                                   "frames_per_s": round(B * 1000.0 / seq_ms, 2)},
        "speedup_batched_vs_sequential": round(seq_ms / batched_ms, 3),
        "autotune_seconds": round(tune_s, 1), "autotune_candidates": len(entry.get("candidates", [])),
        "steps": steps, "warmup": warmup,
    }


def bench_2160p(steps, warmup, log=None):
    """4 views of 2,000,000 Gaussians at 2160 x 3840, 3 wavelengths, 16
    planes: eager training steps (gradients summed over the views by the
    wave-reduced atomics)."""
    import torch

    import scenegen
    from paper_2506_08350_amd import api

    w = scenegen.make_workload("c5")
    sc, cams, opt = w.scene, w.cameras, w.optics
    B, H, W = len(cams), cams[0].height, cams[0].width
    o = api.Optics(opt.wavelengths, opt.distances, opt.pitch, opt.pad, opt.band_limit)
    params = {k: torch.from_numpy(a).cuda() for k, a in zip(api.PARAM_NAMES, sc.arrays())}
    cam_t = api.pack_cameras(cams)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w.notes["target_seed"])
    target = torch.rand(w.notes["target_shape"], generator=gen, device="cuda")
    probe = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=1 << 30)
    probe.forward(params, cam_t, want_field=False, want_intensity=False)
    st, need = probe.read_status()
    del probe
    torch.cuda.empty_cache()
    r = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=int(need * 1.05) + 4096)
    for _ in range(warmup):
        r.train_step(params, cam_t, target)
    st, need = r.read_status()
    if st != 0:
        raise RuntimeError(f"2160p: pair list overflow ({need})")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        loss, grads, _ = r.train_step(params, cam_t, target)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    finite = all(bool(torch.isfinite(g).all()) for g in grads.values())
    if log:
        r.timing(True)
        r.train_step(params, cam_t, target)
        torch.cuda.synchronize()
        r.timing(False)
        kt = r.timing_report()
        for name, (c, t) in sorted(kt.items(), key=lambda kv: -kv[1][1])[:12]:
            log(f"2160p kernel {name:18s} {c:3d} x {t / c:9.3f} ms")
    del r, target, grads
    torch.cuda.empty_cache()
    return {"workload": w.name, "gaussians": sc.n, "views_per_step": B, "height": H, "width": W,
            "wavelengths": sc.n_lambda, "planes": len(opt.distances), "pad": opt.pad, "pairs": int(need),
            "graph": False, "ms_per_step": round(ms, 3), "frames_per_s": round(B * 1000.0 / ms, 3),
            "loss": float(loss), "gradients_finite": finite, "steps": steps, "warmup": warmup}


def bench_next_rows(steps, log):
    """Step times of the rows beyond the single-plane path, on the 1080p
    scene: the four-layer hologram (record + inverse propagation with
    straight-through plane assignment), the paper's training loss (masked
    reconstruction + SSIM), one phase-only conversion step of the rendered
    frame's hologram, and one step of the optimisation loop (render, Adan on
    every tensor, gradient statistics) plus one densification.  Each is timed
    over ``steps`` steps after two warm-up steps, with a synchronisation on
    both sides."""
    import torch

    import scenegen
    from paper_2506_08350_amd import api

    def timed(fn, n):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000.0 / n

    def renderer(w, params, cam_t, **kw):
        sc, cams, opt = w.scene, w.cameras, w.optics
        o = api.Optics(opt.wavelengths, opt.distances, opt.pitch, opt.pad, opt.band_limit)
        H, W = cams[0].height, cams[0].width
        probe = api.Renderer(H, W, o, n_views=len(cams), max_gaussians=sc.n, max_pairs=1 << 27,
                             layered=kw.get("layered", False))
        probe.forward(params, cam_t, want_field=False, want_intensity=False)
        need = probe.read_status()[1]
        del probe
        return api.Renderer(H, W, o, n_views=len(cams), max_gaussians=sc.n, max_pairs=int(need * 1.25) + 4096,
                            **kw)

    out = {}
    # four-layer hologram, the training step captured in a HIP graph
    w = scenegen.make_workload("c3_layers")
    cam_t = api.pack_cameras(w.cameras)
    params = {k: torch.from_numpy(a).cuda() for k, a in zip(api.PARAM_NAMES, w.scene.arrays())}
    params[api.LAYER_LOGITS] = torch.from_numpy(w.notes["logits"]).cuda()
    target = torch.from_numpy(w.targets).cuda()
    r = renderer(w, params, cam_t, layered=True)
    cap = api.CapturedTrainStep(r, params, cam_t, target)
    ms = timed(cap.replay, steps)
    out["layers_4_fwd_bwd"] = {"workload": w.name, "graph": True, "ms_per_step": round(ms, 4),
                               "frames_per_s": round(1000.0 / ms, 3)}
    log(f"four-layer step {ms:.3f} ms")
    del cap, r
    torch.cuda.empty_cache()
    # the paper's training loss
    w = scenegen.make_workload("c3")
    B, K, H, W = len(w.cameras), len(w.optics.distances), w.cameras[0].height, w.cameras[0].width
    cam_t = api.pack_cameras(w.cameras)
    params = {k: torch.from_numpy(a).cuda() for k, a in zip(api.PARAM_NAMES, w.scene.arrays())}
    target = torch.from_numpy(w.targets).cuda()
    masks = torch.from_numpy(scenegen.make_plane_masks(B, K, H, W, w.notes["masks_seed"])).cuda()
    r = renderer(w, params, cam_t, loss="paper")
    cap = api.CapturedTrainStep(r, params, cam_t, target, masks=masks)
    ms = timed(cap.replay, steps)
    out["paper_loss_fwd_bwd"] = {"workload": "c3_fwd_bwd_1080p_3l_4z_100k, masked reconstruction + SSIM",
                                 "graph": True, "ms_per_step": round(ms, 4), "frames_per_s": round(1000.0 / ms, 3)}
    log(f"paper-loss step {ms:.3f} ms")
    del cap, r, masks
    torch.cuda.empty_cache()
    # phase-only conversion of the rendered frame's hologram (3 wavelengths x 4 planes)
    r = renderer(w, params, cam_t, phase_only=True)
    field = r.forward(params, cam_t, want_field=True, want_intensity=False)["field"]
    targets, _ = r.propagate(field, want_intensity=False)
    phi = torch.atan2(field[..., 1], field[..., 0]).contiguous()
    ms = timed(lambda: r.phase_only_step(targets, phi), steps)
    out["phase_only_step"] = {"what": "loss and dL/dphi of exp(j phi) against the propagated planes, 1080p x 3 "
                                      "wavelengths x 4 planes", "ms_per_step": round(ms, 4)}
    log(f"phase-only step {ms:.3f} ms")
    del r, field, targets, phi
    torch.cuda.empty_cache()
    # the optimisation loop: render + Adan + statistics, then one densification
    raw = dict(params)
    o = raw["opacity"].clamp(1e-6, 1 - 1e-6)
    raw["opacity"] = torch.log(o / (1.0 - o)).contiguous()
    r = renderer(w, params, cam_t)
    tr = api.Trainer(r, raw, cam_t, target, total_steps=10 ** 6, densify_every=10 ** 6)
    ms = timed(tr.step, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr.densify()
    torch.cuda.synchronize()
    dms = (time.perf_counter() - t0) * 1000.0
    out["training_step"] = {"what": "render fwd+bwd (eager), Adan on every tensor, view-space gradient statistics",
                            "ms_per_step": round(ms, 4), "densify_ms": round(dms, 3), "gaussians_after": tr.n}
    log(f"training step {ms:.3f} ms, densification {dms:.2f} ms")
    del tr, r
    torch.cuda.empty_cache()
    return out


def torch_fft_reference(r, o, field, reps=10):
    """Forward propagation of one frame (zero pad, FFT2, transfer function,
    inverse FFT2, crop, |u|^2 for every wavelength and plane) written with
    torch.fft, against this library's propagation of the same field."""
    import math

    import torch
    B, L, H, W = field.shape[:4]
    pH, pW = o.pad * H, o.pad * W
    fy = torch.fft.fftfreq(pH, d=o.pitch, dtype=torch.float64, device="cuda")
    fx = torch.fft.fftfreq(pW, d=o.pitch, dtype=torch.float64, device="cuda")
    f2 = fy[:, None] ** 2 + fx[None, :] ** 2
    Hs = []
    for lam in o.wavelengths:
        root = torch.sqrt(torch.clamp(1.0 / lam ** 2 - f2, min=0.0))
        Hs.append(torch.stack([torch.exp(1j * 2 * math.pi * z * root) for z in o.distances]))
    Hz = torch.stack(Hs).to(torch.complex64)                    # [L, K, pH, pW]
    U = torch.view_as_complex(field[0].contiguous())             # [L, H, W]

    def run():
        Up = torch.zeros((L, pH, pW), dtype=torch.complex64, device="cuda")
        Up[:, :H, :W] = U
        S = torch.fft.fft2(Up)
        u = torch.fft.ifft2(S[:, None] * Hz)[..., :H, :W]
        return u.real ** 2 + u.imag ** 2

    for _ in range(2):
        run()
    t_torch = statistics.median(_events_ms(run, reps))
    for _ in range(2):
        r.propagate(field, want_prop=False, want_intensity=True)
    t_lib = statistics.median(_events_ms(lambda: r.propagate(field, want_prop=False, want_intensity=True), reps))
    del Hz
    torch.cuda.empty_cache()
    return {"what": "pad + FFT2 + transfer + IFFT2 + crop + |u|^2, 3 wavelengths x 4 planes, 2160x3840 padded",
            "torch_fft_ms": round(t_torch, 4), "library_propagate_ms": round(t_lib, 4),
            "library_speedup": round(t_torch / t_lib, 2)}


# ------------------------------------------------------------------ main --
def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c3_layers"],
                    help="c3: 1080p fwd+bwd (default); c2: same, forward only; c4: only the 16-view ring batch; "
                         "c3_layers: the c3 scene as a four-layer hologram (record + inverse propagation)")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches (with per-kernel events) instead of replays of the step captured "
                         "in a HIP graph (the default for the training step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the ring, 2160p, copy and torch.fft measurements (for profiler runs)")
    ap.add_argument("--kernel-table", action="store_true", help="also print the per-kernel table to stderr")
    ap.add_argument("--cols-per-block", type=int, default=0, help="column FFT pass: 1, 2 or 4 columns per workgroup")
    ap.add_argument("--tile", default=None, help="raster tile, e.g. 16x16, 16x8, 8x8 (default 16x16)")
    ap.add_argument("--loss", default="mse", choices=["mse", "paper"],
                    help="training loss: the MSE (default) or the paper's masked reconstruction + SSIM loss")
    ap.add_argument("--no-fwd-rate", action="store_true",
                    help="skip the separate forward-only timing (keeps every launch a training-step launch)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (reference for HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build measures one GPU "
              "(the path shards by views across GPUs, see the design notes)", file=sys.stderr)
        return 2

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    import scenegen
    layered = args.workload == "c3_layers"
    w = scenegen.make_workload("c3_layers" if layered else "c3")   # c2: the c3 scene and optics without the loss
    # the CPU baseline runs first, before this process initialises the GPU
    cpu = None
    if not args.no_cpu_baseline and not layered and args.workload != "c4":
        log("cpu baseline (oracle, full frame)")
        cpu = cpu_baseline(w)
        log(cpu["sample"])

    import torch

    from paper_2506_08350_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"calibration copy: {n} bytes read, {n} bytes written", file=sys.stderr)
        del src, dst
    if args.workload == "c4":
        print(json.dumps(bench_ring(args.steps, args.warmup, log)), flush=True)
        return 0

    sc, cams, opt = w.scene, w.cameras, w.optics
    B, L, K = len(cams), sc.n_lambda, len(opt.distances)
    H, W = cams[0].height, cams[0].width
    pH, pW = opt.pad * H, opt.pad * W
    train = args.workload in ("c3", "c3_layers")
    o = api.Optics(opt.wavelengths, opt.distances, opt.pitch, opt.pad, opt.band_limit)
    params = {k: torch.from_numpy(a).cuda() for k, a in zip(api.PARAM_NAMES, sc.arrays())}
    if layered:
        params[api.LAYER_LOGITS] = torch.from_numpy(w.notes["logits"]).cuda()
    tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else (16, 16)
    masks = None
    if args.loss == "paper":
        masks = torch.from_numpy(scenegen.make_plane_masks(B, K, H, W, w.notes["masks_seed"])).cuda()
    cam_t = api.pack_cameras(cams)
    target = torch.from_numpy(w.targets).cuda()

    # size the pair list from one eager forward
    r = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=1 << 27, tile=tile, layered=layered)
    r.forward(params, cam_t, want_field=False, want_intensity=False)
    st, need = r.read_status()
    cap = int(need * 1.25) + 4096
    del r
    r = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=cap, tile=tile,
                     cols_per_block=args.cols_per_block, layered=layered, loss=args.loss)

    def step():
        if train:
            r.train_step(params, cam_t, target, masks=masks)
        else:
            r.forward(params, cam_t, want_field=False, want_intensity=True)

    for _ in range(args.warmup):
        step()
    st, need = r.read_status()
    if st != 0:
        raise RuntimeError(f"pair list overflow: {need} > {cap}")
    torch.cuda.synchronize()
    graph = train and not args.eager
    captured = None
    if graph:
        captured = api.CapturedTrainStep(r, params, cam_t, target, masks=masks)
        step = captured.replay
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
    # the timed region: exactly `steps` steps between two synchronisations
    r.timing(not graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r.timing(False)
    ms = (t1 - t0) * 1000.0 / args.steps
    value = B * 1000.0 / ms
    # per-step HIP-event times of the same step (median of 50 after the warm-up)
    step_ms = _events_ms(step, 50)
    if graph:       # per-kernel events cannot live inside a graph: time them eagerly
        r.timing(True)
        for _ in range(args.steps):
            r.train_step(params, cam_t, target, masks=masks) if train else r.forward(params, cam_t, want_field=False)
        torch.cuda.synchronize()
        r.timing(False)
    kt = r.timing_report()

    # forward-only rate (intensities out), same scene and optics
    fwd_ms = None
    if train and not args.no_fwd_rate:
        fstep = lambda: r.forward(params, cam_t, want_field=False, want_intensity=True)  # noqa: E731
        for _ in range(2):
            fstep()
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(args.steps):
            fstep()
        torch.cuda.synchronize()
        fwd_ms = (time.perf_counter() - f0) * 1000.0 / args.steps

    # raster work of the frame (the last forward's tile ranges and indices)
    walk_fwd, walk_bwd = (None, None) if layered else raster_walks(r, B, H, W, tile, 1e-4)
    inc = cpu["included_pairs"] if cpu else None
    work = None
    if walk_bwd is not None:
        work = {"tests_forward": walk_fwd, "tests_backward": walk_bwd, "included_pairs": inc,
                "included_pairs_from": "FP64 oracle, full frame" if inc else None,
                "ops_per_test": OPS_TEST, "ops_per_included_forward": OPS_FWD_INC,
                "ops_per_included_backward": OPS_BWD_INC,
                "lane_ops_forward": OPS_TEST * walk_fwd + OPS_FWD_INC * inc if inc else None,
                "lane_ops_backward": OPS_TEST * walk_bwd + OPS_BWD_INC * inc if inc else None}

    per_launch = {n: (c, tot / c) for n, (c, tot) in kt.items()}
    fused = args.loss == "mse"
    asm = {n: v for n, v in per_launch.items() if kernel_bytes(n, B, L, K, H, W, pH, pW, train, fused) is not None}

    def hbm_entry(n):
        b = kernel_bytes(n, B, L, K, H, W, pH, pW, train, fused)
        a = b / (per_launch[n][1] * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": n, "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(a / HBM_PEAK_GBS, 4), "traffic": measured_traffic(n),
                "avg_ms": round(per_launch[n][1], 4), "algorithmic_bytes": b}

    def alu_entry(n):
        ops = (work or {}).get("lane_ops_backward" if n == "raster_backward" else "lane_ops_forward")
        t = per_launch[n][1]
        instr = measured_valu_instructions(n)
        a = ops / (t * 1e-3) / 1e9 if ops else None
        return {"bound": "alu", "kernel": n, "achieved": round(a, 1) if a else None, "peak": VALU_PEAK_GOPS,
                "unit": "G lane-ops/s", "frac": round(a / VALU_PEAK_GOPS, 4) if a else None,
                "traffic": measured_traffic(n), "avg_ms": round(t, 4), "algorithmic_lane_ops": ops,
                "valu_instructions": instr,
                "issued_frac": round(instr * 64 / (t * 1e-3) / 1e9 / VALU_PEAK_GOPS, 4) if instr else None,
                "algorithmic_over_issued": round(ops / (instr * 64), 4) if ops and instr else None}

    dom = max(per_launch, key=lambda n: per_launch[n][0] * per_launch[n][1])
    if dom in ("raster_backward", "raster_forward") and not layered:
        roofline = alu_entry(dom)
    elif dom in asm:
        roofline = hbm_entry(dom)
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": None, "traffic": measured_traffic(dom), "avg_ms": round(per_launch[dom][1], 4)}
    per_kernel = {n: hbm_entry(n) for n in asm}
    if not layered:
        for n in ("raster_forward", "raster_backward"):
            if n in per_launch:
                per_kernel[n] = alu_entry(n)
    if args.kernel_table:
        _kernel_table(per_launch, B, L, K, H, W, pH, pW, train, fused)

    metric = ("hologram frames/s (splat+ASM, fwd+bwd) 1080p x 3 wavelengths x 4 planes" if not layered else
              "hologram frames/s (4-layer splat + record + inverse ASM, fwd+bwd) 1080p x 3 wavelengths")
    workload = ("c3_fwd_bwd_1080p_3l_4z_100k" if train else "c2_fwd_1080p_3l_4z_100k") if not layered else w.name
    line = {
        "metric": metric,
        "value": round(value, 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "tile": f"{tile[0]}x{tile[1]}", "loss": args.loss,
                   "gaussians": sc.n, "height": H, "width": W, "wavelengths": L, "planes": K,
                   "views_per_step": B, "pad": opt.pad, "pairs": int(need), "parallelism": "single-gpu"},
        "step_ms_events": {"median": round(statistics.median(step_ms), 4), "min": round(min(step_ms), 4),
                           "n": len(step_ms)},
        "fwd_frames_per_s": round(1000.0 / fwd_ms * B, 3) if fwd_ms else None,
        "fwd_ms": round(fwd_ms, 4) if fwd_ms else None,
        "graph": bool(graph),
        "roofline": roofline,
        "roofline_per_kernel": per_kernel,
        "raster_work": work,
        "kernels_ms_per_step": {n: round(c * m / args.steps, 4) for n, (c, m) in per_launch.items()},
    }
    if cpu:
        line["cpu_baseline"] = {k: v for k, v in cpu.items() if k != "included_pairs"}
    if not args.headline_only and not layered:
        log("copy bandwidth")
        line["copy_bandwidth"] = copy_bandwidth()
        log("torch.fft reference")
        field = r.forward(params, cam_t, want_field=True, want_intensity=False)["field"]
        line["torch_fft_asm"] = torch_fft_reference(r, o, field)
        del field, r, captured
        torch.cuda.empty_cache()
        log("ring of 16 views")
        line["ring_16_views"] = bench_ring(max(2, args.steps // 4), 2, log)
        log("2160p, 4 views")
        line["views_2160p"] = bench_2160p(3, 1, log)
        log("rows beyond the single-plane path")
        line["next_rows"] = bench_next_rows(max(5, args.steps // 2), log)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
