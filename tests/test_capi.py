"""Host-side checks of the C ABI (no GPU calls): the library loads, exports every
function include/chrf.h declares, and the ctypes structures match the C layout."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2506_08350_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chrf.h")


def _ensure_built():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2506_08350_amd import build
        build.build()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chrf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_bound_functions():
    assert set(_declared()) == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (chrf_\w+)", out))
    assert set(_declared()) <= exported


def test_struct_layout_matches_c():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "chrf.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(chrf_plan_desc), sizeof(chrf_camera), sizeof(chrf_gaussians),
         sizeof(chrf_grads), offsetof(chrf_plan_desc, k_sigma));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(chrf_plan_desc, pitch), offsetof(chrf_plan_desc, distances),
         offsetof(chrf_plan_desc, cols_per_block), offsetof(chrf_plan_desc, layered),
         offsetof(chrf_gaussians, logits), offsetof(chrf_grads, logits));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(chrf_plan_desc, loss_kind), offsetof(chrf_plan_desc, ssim_weight),
         offsetof(chrf_plan_desc, phase_only), offsetof(chrf_plan_desc, deterministic),
         offsetof(chrf_plan_desc, fft_rows_plan), offsetof(chrf_plan_desc, fft_cols_plan));
  printf("%zu %zu %zu %zu\n", sizeof(chrf_densify_desc), offsetof(chrf_densify_desc, zeta),
         offsetof(chrf_densify_desc, tau_grad), offsetof(chrf_densify_desc, shrink));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    P = _lib.PlanDesc
    D = _lib.DensifyDesc
    assert vals == [ctypes.sizeof(P), ctypes.sizeof(_lib.Camera), ctypes.sizeof(_lib.Gaussians),
                    ctypes.sizeof(_lib.Grads), P.k_sigma.offset, P.pitch.offset, P.distances.offset,
                    P.cols_per_block.offset, P.layered.offset, _lib.Gaussians.logits.offset,
                    _lib.Grads.logits.offset, P.loss_kind.offset, P.ssim_weight.offset, P.phase_only.offset,
                    P.deterministic.offset, P.fft_rows_plan.offset, P.fft_cols_plan.offset,
                    ctypes.sizeof(D), D.zeta.offset, D.tau_grad.offset, D.shrink.offset]


def test_camera_record_packing_matches_struct():
    from scenegen import identity_camera
    cam = identity_camera(64, 32)
    assert cam.as_array().nbytes == ctypes.sizeof(_lib.Camera)


def test_last_error_and_version_callable_without_gpu():
    _ensure_built()
    lib = _lib.load()
    assert lib.chrf_version().startswith(b"chrf")
    assert isinstance(lib.chrf_last_error(), bytes)
