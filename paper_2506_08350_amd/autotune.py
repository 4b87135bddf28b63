"""Autotuner for the launch configuration of one workload shape.

The searched configuration is the raster tile shape, the columns per
workgroup of the column FFT pass and, where the padded grid has tuned
transforms (widths 3840 and 7680, heights 2160 and 4320), the radix schedules
of the row and of the column transforms.  Each candidate builds a plan, runs the fused training
step a few times and is timed with HIP events on the launch stream (median of
the timed repetitions).  The search is coordinate-wise: the tile with the
default transforms first, then the columns per workgroup, then the row
schedule, then the column schedule, each keeping the best of the earlier
steps.  Results persist in a JSON cache keyed by the device architecture and
the workload shape, so a later process reuses them without timing again.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "chrf_autotune.json")

TILES = ((16, 16), (16, 8), (8, 16), (32, 8), (8, 8))
COLS = (0, 4, 1)            # 0: the library's choice for the padded height (2 at 2160 and at 4320)
ROW_PLANS = (0, 1, 2)       # 3840: 16*16*15, 16*15*16, 15*16*16; 7680: 16*20*24, 16*24*20, 24*20*16
COL_PLANS = (0, 1, 2, 3)    # 2160 (and 4320 as two of 2160): 16*15*9, 16*9*15, 15*16*9, 12*12*15


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


def time_config(height, width, optics, params, cams, target, max_pairs, reps=5, warmup=2, **plan_kw):
    """Median milliseconds of one fused training step for one configuration
    (plan_kw: Renderer keyword arguments, e.g. tile, cols_per_block, fft_plans)."""
    r = api.Renderer(height, width, optics, n_views=cams.shape[0], max_gaussians=params["means"].shape[0],
                     max_pairs=max_pairs, **plan_kw)
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
    del r
    return statistics.median(times)


def _jsonable(cfg):
    return {k: list(v) if isinstance(v, tuple) else v for k, v in cfg.items()}


def _from_json(d):
    return {"tile": tuple(d["tile"]), "cols_per_block": int(d["cols_per_block"]),
            "fft_plans": tuple(d.get("fft_plans", (0, 0)))}


def autotune(height, width, optics, params, cams, target, max_pairs, cache=DEFAULT_CACHE, tiles=TILES, cols=COLS,
             row_plans=ROW_PLANS, col_plans=COL_PLANS, force=False, **plan_kw):
    """Best configuration for this shape, as Renderer keyword arguments
    {tile, cols_per_block, fft_plans}, and the cache entry with every timed
    candidate; cached across processes unless cache is None."""
    key = shape_key(height, width, len(optics.wavelengths), len(optics.distances), cams.shape[0],
                    params["means"].shape[0], optics.pad)
    data = _load(cache) if cache else {}
    if not force and key in data:
        return _from_json(data[key]), data[key]
    results = []

    def trial(cfg):
        for r in results:
            if r["config"] == _jsonable(cfg):
                return r.get("ms")
        try:
            ms = time_config(height, width, optics, params, cams, target, max_pairs, **cfg, **plan_kw)
        except Exception as exc:   # a candidate this shape or build does not support
            results.append({"config": _jsonable(cfg), "error": str(exc)})
            return None
        results.append({"config": _jsonable(cfg), "ms": ms})
        return ms

    best = {"tile": tuple(tiles[0]), "cols_per_block": cols[0], "fft_plans": (0, 0)}

    def with_value(axis, v):
        cfg = dict(best)
        if axis == "row_plan":
            cfg["fft_plans"] = (v, best["fft_plans"][1])
        elif axis == "col_plan":
            cfg["fft_plans"] = (best["fft_plans"][0], v)
        else:
            cfg[axis] = v
        return cfg

    for axis, values in (("tile", [tuple(t) for t in tiles]), ("cols_per_block", list(cols)),
                         ("row_plan", list(row_plans)), ("col_plan", list(col_plans))):
        scored = []
        for v in values:
            cfg = with_value(axis, v)
            ms = trial(cfg)
            if ms is not None:
                scored.append((ms, cfg))
        if scored:
            best = min(scored, key=lambda t: t[0])[1]
    ok = [r for r in results if "ms" in r]
    if not ok:
        raise RuntimeError("no candidate configuration ran")
    best_ms = min(r["ms"] for r in ok if r["config"] == _jsonable(best))
    entry = dict(_jsonable(best), ms=best_ms, candidates=results)
    if cache:
        data[key] = entry
        _store(cache, data)
    return best, entry
