#!/usr/bin/env python
"""Throughput of the complex-hologram hot path on one MI355X.

A step is one pass of the whole path over one batch: projection and culling,
tile binning and sort, complex compositing, band-limited ASM propagation to
every plane, |u|^2, the MSE against seeded targets, and the full backward to
the Gaussian parameters.  The default workload is 100,000 Gaussians rendered
at 1080 x 1920 for three wavelengths and propagated to four planes (one view
per step).  Inputs are synthetic and resident in HBM before timing starts.
The timed steps replay the whole training step captured once in a HIP graph
(``--eager`` times eager launches instead); per-kernel times come from a
separate eager pass with HIP events on the launch stream.

Prints one JSON line (see the keys below).  ``--gpus N`` with N > 1 is not
supported: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure


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


def source_sha256(name):
    import hashlib
    with open(os.path.join(ROOT, "paper_2506_08350_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or
    None when that summary is missing, does not cover the kernel, or any of the
    kernel's sources changed since the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    shas = {}
    table = {}
    for line in text.splitlines():
        if line.startswith("source-sha256 "):
            _, name, sha = line.split()
            shas[name] = sha
        cells = [c.strip(" `") for c in line.strip().strip("|").split("|")]
        if len(cells) == 5 and cells[0] and cells[4].isdigit():
            table[cells[0]] = int(cells[4])
    files = KERNEL_SOURCES.get(kernel)
    if kernel not in table or not files:
        return None
    for f in files:
        if shas.get(f) != source_sha256(f):
            return None
    return table[kernel]


VALU_PROFILE = os.path.join(ROOT, "profiles", "valu_step_c3_1080p_100k.md")
VALU_NAMES = {"cols_adjoint": "k_cols_adjoint_t", "cols_forward": "k_cols_forward_t",
              "raster_backward": "k_raster_bwd", "raster_forward": "k_raster_fwd"}
# Vector-ALU issue peak: 2 wave64 VALU instructions per CU per cycle (the FP32
# vector rate, 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 2 x 64 lanes x 2 flops), in
# lane-operations per second.
VALU_PEAK_GOPS = 256 * 2.4 * 2 * 64


def measured_valu_instructions(kernel):
    """VALU instructions per launch of ``kernel`` (SQ_INSTS_VALU) from the
    committed counter summary, or None when the summary is missing, does not
    cover the kernel, or any of the kernel's sources changed since."""
    try:
        text = open(VALU_PROFILE).read()
    except OSError:
        return None
    shas, count = {}, None
    for line in text.splitlines():
        if line.startswith("source-sha256 "):
            _, name, sha = line.split()
            shas[name] = sha
        cells = [c.strip(" `") for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and kernel in VALU_NAMES and cells[0].startswith(VALU_NAMES[kernel] + "<"):
            count = int(cells[2])
    files = KERNEL_SOURCES.get(kernel)
    if count is None or not files or any(shas.get(f) != source_sha256(f) for f in files):
        return None
    return count


def cpu_baseline(w, seed=0):
    """Time the CPU oracle on a bounded sample of the workload.

    Sample: the projection plus the compositing forward and backward of all
    Gaussians and all wavelengths restricted to the central 1/16 of the frame
    (a 270 x 480 window, the densest part of the image), plus one full-size
    propagation and its adjoint for one (wavelength, plane) pair.  The frame
    time is extrapolated as 16 x window + (L x K) x propagation pair.
    """
    import numpy as np
    import oracle
    from oracle.projection import project_backward

    sc, cam, opt = w.scene, w.cameras[0], w.optics
    H, W = cam.height, cam.width
    thr = oracle.DEFAULT
    win = (H * 3 // 8, H * 5 // 8, W * 3 // 8, W * 5 // 8)
    frac = ((win[1] - win[0]) * (win[3] - win[2])) / float(H * W)
    t0 = time.perf_counter()
    p = oracle.project(sc.means, sc.log_scales, sc.quats, sc.amp, sc.phase, cam)
    fp = oracle.fp32_footprint(sc.means, sc.log_scales, sc.quats, cam, k_sigma=thr.k_sigma)
    res = oracle.render_field(p, sc.opacity, fp, W, H, thr, window=win)
    rng = np.random.default_rng(seed)
    G = np.zeros_like(res.U)
    G[:, win[0]:win[1], win[2]:win[3]] = rng.normal(size=(sc.n_lambda, win[1] - win[0], win[3] - win[2]))
    d = oracle.render_field_backward(p, sc.opacity, fp, res, G, thr, window=win)
    project_backward(p, sc.quats, sc.amp, sc.phase, cam, *d)
    t_raster = time.perf_counter() - t0
    t0 = time.perf_counter()
    u = oracle.propagate(res.U[0], opt.wavelengths[0], opt.distances[0], opt.pitch, opt.pad, opt.band_limit)
    oracle.propagate_adjoint(u, opt.wavelengths[0], opt.distances[0], opt.pitch, opt.pad, opt.band_limit)
    t_asm = time.perf_counter() - t0
    n_pairs = len(opt.wavelengths) * len(opt.distances)
    t_frame = t_raster / frac + n_pairs * t_asm
    return {
        "value": 1.0 / t_frame, "unit": "frames/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 NumPy oracle, single thread: compositing fwd+bwd of all {sc.n} Gaussians x "
                   f"{sc.n_lambda} wavelengths on the central {win[1] - win[0]}x{win[3] - win[2]} window "
                   f"({t_raster:.1f} s, scaled x{1 / frac:.0f}) + one full-size propagation and adjoint "
                   f"({t_asm:.1f} s, scaled x{n_pairs}); estimated {t_frame:.0f} s per frame"),
    }


def bench_batched(args):
    """16 views of the 500,000-Gaussian ring scene in one batched step, against
    the same work done one view at a time with a single-view plan."""
    import torch

    import scenegen
    from paper_2506_08350_amd import api

    w = scenegen.make_workload("c4")
    sc, cams, opt = w.scene, w.cameras, w.optics
    B, H, W = len(cams), cams[0].height, cams[0].width
    o = api.Optics(opt.wavelengths, opt.distances, opt.pitch, opt.pad, opt.band_limit)
    params = {k: torch.from_numpy(a).cuda() for k, a in zip(api.PARAM_NAMES, sc.arrays())}
    cam_t = api.pack_cameras(cams)
    target = torch.from_numpy(w.targets).cuda()
    probe = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=1 << 28)
    probe.forward(params, cam_t, want_field=False, want_intensity=False)
    st, need = probe.read_status()
    del probe
    rb = api.Renderer(H, W, o, n_views=B, max_gaussians=sc.n, max_pairs=int(need * 1.1) + 4096)
    r1 = api.Renderer(H, W, o, n_views=1, max_gaussians=sc.n, max_pairs=int(need * 1.1) + 4096)
    tv = [target[v:v + 1].contiguous() for v in range(B)]

    def batched():
        return rb.train_step(params, cam_t, target)

    def sequential():
        for v in range(B):
            r1.train_step(params, cam_t[v:v + 1], tv[v])

    res = {}
    for name, fn in (("batched", batched), ("sequential", sequential)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) * 1000.0 / args.steps
    line = {
        "metric": "hologram frames/s (splat+ASM, fwd+bwd) 1080p x 3 wavelengths x 8 planes, 16-view batch",
        "value": round(B * 1000.0 / res["batched"], 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(res["batched"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4_batched_16view_ring_500k", "gaussians": sc.n, "views_per_step": B,
                   "height": H, "width": W, "wavelengths": sc.n_lambda, "planes": len(opt.distances),
                   "pairs": int(need), "parallelism": "single-gpu"},
        "sequential_ms_per_step": round(res["sequential"], 4),
        "sequential_frames_per_s": round(B * 1000.0 / res["sequential"], 3),
        "speedup_vs_sequential": round(res["sequential"] / res["batched"], 3),
    }
    print(json.dumps(line), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c3_layers"],
                    help="c3: 1080p fwd+bwd (default); c2: same, forward only; c4: 16-view batch vs sequential; "
                         "c3_layers: the c3 scene as a four-layer hologram (record + inverse propagation)")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches (with per-kernel events) instead of replays of the step captured "
                         "in a HIP graph (the default for the training step)")
    ap.add_argument("--graph", action="store_true", help=argparse.SUPPRESS)   # the default; kept for old scripts
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-table", action="store_true", help="also print the per-kernel table to stderr")
    ap.add_argument("--cols-per-block", type=int, default=0, help="column FFT pass: 2 or 4 columns per workgroup")
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

    import numpy as np
    import torch

    import scenegen
    from paper_2506_08350_amd import _lib, api

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
        return bench_batched(args)
    layered = args.workload == "c3_layers"
    w = scenegen.make_workload("c3_layers" if layered else "c3")   # c2: the c3 scene and optics without the loss
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
    if graph:
        captured = api.CapturedTrainStep(r, params, cam_t, target, masks=masks)
        step = captured.replay
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
    r.timing(not graph)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r.timing(False)
    if graph:       # per-kernel events cannot live inside a graph: time them eagerly
        r.timing(True)
        for _ in range(args.steps):
            r.train_step(params, cam_t, target, masks=masks) if train else r.forward(params, cam_t, want_field=False)
        torch.cuda.synchronize()
        r.timing(False)
    kt = r.timing_report()
    ms = (t1 - t0) * 1000.0 / args.steps
    value = B * 1000.0 / ms

    # forward-only rate (intensities out), same scene and optics
    fwd_ms = None
    if train and not args.no_fwd_rate:
        for _ in range(2):
            r.forward(params, cam_t, want_field=False, want_intensity=True)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(args.steps):
            r.forward(params, cam_t, want_field=False, want_intensity=True)
        torch.cuda.synchronize()
        fwd_ms = (time.perf_counter() - f0) * 1000.0 / args.steps

    # The dominant kernel of the step (the raster backward, or a column FFT
    # pass) issues more vector-ALU lane-operations per HBM byte than the
    # chip's ratio (78.6 T/s over 8 TB/s, about 10 per byte), so it is
    # reported against the VALU issue peak (lane-operations issued per
    # second, from its counted VALU instructions and the live launch time).
    # The dominant propagation kernel is also reported against HBM.
    per_launch = {n: (c, tot / c) for n, (c, tot) in kt.items()}
    fused = args.loss == "mse"
    asm = {n: v for n, v in per_launch.items() if kernel_bytes(n, B, L, K, H, W, pH, pW, train, fused) is not None}
    pdom = max(asm, key=lambda n: asm[n][0] * asm[n][1])
    pdom_ms = asm[pdom][1]
    pdom_bytes = kernel_bytes(pdom, B, L, K, H, W, pH, pW, train, fused)
    p_achieved = pdom_bytes / (pdom_ms * 1e-3) / 1e9
    hbm = {"bound": "hbm", "kernel": pdom, "achieved": round(p_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(p_achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(pdom),
           "avg_ms": round(pdom_ms, 4), "algorithmic_bytes": pdom_bytes}
    dom = max(per_launch, key=lambda n: per_launch[n][0] * per_launch[n][1])
    if dom in VALU_NAMES and not layered:
        dom_ms = per_launch[dom][1]
        instr = measured_valu_instructions(dom)
        achieved = instr * 64 / (dom_ms * 1e-3) / 1e9 if instr else None
        roofline = {"bound": "alu", "kernel": dom,
                    "achieved": round(achieved, 1) if achieved else None, "peak": VALU_PEAK_GOPS,
                    "unit": "G VALU lane-ops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4) if achieved else None,
                    "traffic": measured_traffic(dom), "avg_ms": round(dom_ms, 4), "valu_instructions": instr,
                    "hbm_dominant_propagation": hbm}
    else:
        roofline = hbm
    if args.kernel_table:
        tot = sum(c * m for c, m in per_launch.values())
        for n, (c, m) in sorted(per_launch.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            b = kernel_bytes(n, B, L, K, H, W, pH, pW, train, fused)
            bw = f"{b / (m * 1e-3) / 1e9:8.1f} GB/s" if b else ""
            print(f"{n:18s} {c:4d} x {m:8.4f} ms  {100 * c * m / tot:5.1f}%  {bw}", file=sys.stderr)

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
        "fwd_frames_per_s": round(1000.0 / fwd_ms * B, 3) if fwd_ms else None,
        "fwd_ms": round(fwd_ms, 4) if fwd_ms else None,
        "graph": bool(graph),
        "roofline": roofline,
        "kernels_ms_per_step": {n: round(c * m / args.steps, 4) for n, (c, m) in per_launch.items()},
    }
    if not args.no_cpu_baseline and not layered:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
