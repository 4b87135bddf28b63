"""Autotuner for the launch configuration of one workload shape.

Candidates are (raster tile shape, columns per workgroup of the column FFT
pass).  Each candidate builds a plan, runs the fused training step a few
times and is timed with HIP events on the launch stream (median of the
timed repetitions); the fastest is kept.  Results persist in a JSON cache
keyed by the device architecture and the workload shape, so a later process
reuses them without timing again.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "chrf_autotune.json")

TILES = ((16, 16), (16, 8), (8, 16), (32, 8), (8, 8))
COLS = (4, 2, 1)


def shape_key(height, width, n_lambda, n_planes, n_views, n_gaussians, pad):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    bucket = 1 << max(0, int(n_gaussians - 1).bit_length())
    return f"{arch}|{height}x{width}|L{n_lambda}|K{n_planes}|B{n_views}|N{bucket}|p{pad}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_config(height, width, optics, params, cams, target, tile, cols, max_pairs, reps=5, warmup=2, **plan_kw):
    """Median milliseconds of one fused training step for one configuration."""
    r = api.Renderer(height, width, optics, n_views=cams.shape[0], max_gaussians=params["means"].shape[0],
                     max_pairs=max_pairs, tile=tile, cols_per_block=cols, **plan_kw)
    for _ in range(warmup):
        r.train_step(params, cams, target)
    st, need = r.read_status()
    if st != 0:
        raise RuntimeError(f"pair capacity {max_pairs} too small (needs {need})")
    times = []
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r.train_step(params, cams, target)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def autotune(height, width, optics, params, cams, target, max_pairs, cache=DEFAULT_CACHE, tiles=TILES, cols=COLS,
             force=False, **plan_kw):
    """Best (tile, cols_per_block) for this shape; cached across processes."""
    key = shape_key(height, width, len(optics.wavelengths), len(optics.distances), cams.shape[0],
                    params["means"].shape[0], optics.pad)
    data = _load(cache) if cache else {}
    if not force and key in data:
        d = data[key]
        return tuple(d["tile"]), int(d["cols_per_block"]), d
    results = []
    for t in tiles:
        for c in cols:
            try:
                ms = time_config(height, width, optics, params, cams, target, t, c, max_pairs, **plan_kw)
            except Exception as exc:   # unsupported candidate for this shape
                results.append({"tile": list(t), "cols_per_block": c, "error": str(exc)})
                continue
            results.append({"tile": list(t), "cols_per_block": c, "ms": ms})
    ok = [r for r in results if "ms" in r]
    if not ok:
        raise RuntimeError("no candidate configuration ran")
    best = min(ok, key=lambda r: r["ms"])
    entry = {"tile": best["tile"], "cols_per_block": best["cols_per_block"], "ms": best["ms"], "candidates": results}
    if cache:
        data[key] = entry
        _store(cache, data)
    return tuple(best["tile"]), int(best["cols_per_block"]), entry
