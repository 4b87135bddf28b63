"""Shared helpers for the GPU parity tests (inputs to device, error metrics)."""
import numpy as np
import torch

import oracle
from paper_2506_08350_amd import api


def to_device(scene):
    return {k: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
            for k, a in zip(api.PARAM_NAMES, scene.arrays())}


def make_renderer(cams, optics, n, thr=oracle.DEFAULT, tile=(16, 16), **kw):
    o = api.Optics(tuple(optics.wavelengths), tuple(optics.distances), optics.pitch, optics.pad, optics.band_limit)
    return api.Renderer(cams[0].height, cams[0].width, o, n_views=len(cams), max_gaussians=n,
                        k_sigma=thr.k_sigma, alpha_min=thr.alpha_min, alpha_max=thr.alpha_max, t_min=thr.t_min,
                        tile=tile, **kw)


def cplx(t):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
