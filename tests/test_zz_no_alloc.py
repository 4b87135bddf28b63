"""chrf_densify_noalloc (scratch from the library's per-GPU device array)
against chrf_densify (scratch from a caller buffer): identical outputs on two
calls in a row, the second with fewer Gaussians, so that the second call runs
on the array the first one left behind; sizes above the array's maximum are
refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2506_08350_amd import _lib, api
from tests.gpu_helpers import announce

pytestmark = pytest.mark.gpu

MAX_N = 4194304   # CHRF_NOALLOC_MAX_GAUSSIANS


def _inputs(n, n_lam, seed):
    rng = np.random.default_rng(seed)
    count = rng.integers(0, 4, size=n).astype(np.float32)
    a = dict(means=rng.normal(size=(n, 3)), log_scales=rng.normal(np.log(0.03), 1.0, size=(n, 3)),
             quats=rng.normal(size=(n, 4)), opacity=rng.uniform(0.0, 0.05, size=n),
             phase=rng.uniform(0, 2 * np.pi, size=(n, n_lam)), count=count,
             accum=count * rng.uniform(0.0, 2.0, size=n) * 2e-4, xi=rng.normal(size=(n, 2, 3)),
             zeta=rng.normal(size=(n, 2, n_lam)))
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).cuda() for k, v in a.items()}


def _run(dev, cfg, noalloc):
    params = {k: dev[k] for k in ("means", "log_scales", "quats", "phase")}
    m, src, kind, means, ls, ph, _ = api.densify(params, dev["opacity"], dev["accum"], dev["count"], dev["xi"],
                                                 dev["zeta"], cfg, noalloc=noalloc)
    return m, [t.cpu().numpy() for t in (src, kind, means, ls, ph)]


def test_noalloc_densify_matches_the_scratch_entry_point():
    cfg = api.DensifyConfig(tau_grad=2e-4, split_scale=0.05, prune_scale=0.5, min_opacity=0.005, phase_sigma=0.02)
    for n, seed in ((300000, 11), (4099, 12)):   # second call smaller than the first
        announce(f"densify_noalloc n={n}")
        dev = _inputs(n, 3, seed)
        m_ref, ref = _run(dev, cfg, noalloc=False)
        m, out = _run(dev, cfg, noalloc=True)
        assert m == m_ref and m > 0
        for a, b in zip(out, ref):
            assert np.array_equal(a, b)
        assert {0, 1, 2} <= set(ref[1].tolist())   # clones, splits and kept Gaussians all occur


def test_noalloc_densify_refuses_more_than_its_maximum():
    lib = _lib.load()
    d = _lib.DensifyDesc()
    d.n, d.n_lambda = MAX_N + 1, 3
    n_out = torch.zeros((), dtype=torch.int64, device="cuda")
    st = lib.chrf_densify_noalloc(C.byref(d), 0, None, None, None, None, None, C.c_void_p(n_out.data_ptr()),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.CHRF_EINVAL
    assert b"exceeds the maximum" in lib.chrf_last_error()
