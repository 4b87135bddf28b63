"""ctypes binding of the C ABI declared in include/chrf.h (argument marshalling only).

The shared library is built in-tree (``python -m paper_2506_08350_amd.build``)
as ``paper_2506_08350_amd/libchrf.so``.  Loading fails loudly when it is
missing: there is no CPU or PyTorch fallback for any step of the path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchrf.so")

CHRF_OK = 0
CHRF_EINVAL = -1
CHRF_ENOMEM = -2
CHRF_EHIP = -3
CHRF_ECAPACITY = -4
CHRF_EUNSUPPORTED = -5

REGION_PAIR_KEYS = 0
REGION_PAIR_VALUES = 1
REGION_TILE_RANGES = 2
REGION_STATUS = 3
REGION_T_FINAL = 4
REGION_LAST = 5
REGION_FIELD = 6
REGION_GRAD_FIELD = 7
REGION_LAYER_FIELDS = 8
REGION_LAYER_T_FINAL = 9
REGION_LAYER_STOP = 10
REGION_LAYER_GRAD = 11
REGION_LOSS_PARTIAL = 12

EXPORTED = [
    "chrf_create", "chrf_destroy", "chrf_last_error", "chrf_version", "chrf_plan_create",
    "chrf_plan_destroy", "chrf_plan_workspace_bytes", "chrf_plan_region", "chrf_forward",
    "chrf_backward", "chrf_propagate", "chrf_propagate_adjoint", "chrf_read_status",
    "chrf_timing_enable", "chrf_timing_report", "chrf_phase_only_step", "chrf_adam_step",
    "chrf_adan_step", "chrf_densify_stats", "chrf_densify_workspace_bytes", "chrf_densify", "chrf_gather_rows",
    "chrf_densify_noalloc",
]


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("z_near", C.c_float), ("reserved", C.c_float * 3)]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("amp", C.c_void_p), ("phase", C.c_void_p), ("logits", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("amp", C.c_void_p), ("phase", C.c_void_p), ("logits", C.c_void_p)]


class PlanDesc(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("n_views", C.c_int32), ("n_lambda", C.c_int32),
                ("n_planes", C.c_int32), ("max_gaussians", C.c_int32), ("max_pairs", C.c_int64),
                ("pad_factor", C.c_int32), ("band_limit", C.c_int32), ("pitch", C.c_double),
                ("wavelengths", C.c_double * 4), ("distances", C.c_double * 64), ("k_sigma", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("cols_per_block", C.c_int32),
                ("layered", C.c_int32), ("loss_kind", C.c_int32), ("ssim_weight", C.c_float),
                ("phase_only", C.c_int32), ("deterministic", C.c_int32), ("fft_rows_plan", C.c_int32),
                ("fft_cols_plan", C.c_int32)]


class DensifyDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_lambda", C.c_int32), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity", C.c_void_p), ("phase", C.c_void_p),
                ("grad_accum", C.c_void_p), ("grad_count", C.c_void_p), ("xi", C.c_void_p), ("zeta", C.c_void_p),
                ("tau_grad", C.c_float), ("sigma_split", C.c_float), ("sigma_prune", C.c_float),
                ("min_opacity", C.c_float), ("phase_sigma", C.c_float), ("shrink", C.c_float)]


class ChrfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"chrf status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str | None = None):
    """Load libchrf.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (loads the HIP runtime torch uses first)
    except ImportError:
        pass
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing "
                           "(run `python -m paper_2506_08350_amd.build`)")
    lib = C.CDLL(p)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "chrf_create": (i32, [C.c_int, C.POINTER(vp)]),
        "chrf_destroy": (None, [vp]),
        "chrf_last_error": (C.c_char_p, []),
        "chrf_version": (C.c_char_p, []),
        "chrf_plan_create": (i32, [vp, C.POINTER(PlanDesc), C.POINTER(vp)]),
        "chrf_plan_destroy": (None, [vp]),
        "chrf_plan_workspace_bytes": (sz, [vp]),
        "chrf_plan_region": (i32, [vp, C.c_int, C.POINTER(sz), C.POINTER(sz)]),
        "chrf_forward": (i32, [vp, C.POINTER(Gaussians), vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "chrf_backward": (i32, [vp, C.POINTER(Gaussians), vp, vp, vp, vp, vp, vp, vp, C.POINTER(Grads), vp]),
        "chrf_propagate": (i32, [vp, vp, vp, vp, vp, vp]),
        "chrf_propagate_adjoint": (i32, [vp, vp, vp, vp, vp]),
        "chrf_read_status": (i32, [vp, vp, C.POINTER(i64), vp]),
        "chrf_phase_only_step": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "chrf_adam_step": (i32, [vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp]),
        "chrf_adan_step": (i32, [vp, vp, vp, vp, vp, vp, i64] + [C.c_float] * 6 + [i32, vp]),
        "chrf_densify_stats": (i32, [vp, vp, i32, vp, vp, vp]),
        "chrf_densify_workspace_bytes": (sz, [i64]),
        "chrf_densify": (i32, [C.POINTER(DensifyDesc), vp, i64, vp, vp, vp, vp, vp, vp, vp]),
        "chrf_gather_rows": (i32, [vp, i64, vp, vp, vp, i64, i32, vp, vp]),
        "chrf_densify_noalloc": (i32, [C.POINTER(DensifyDesc), i64, vp, vp, vp, vp, vp, vp, vp]),
        "chrf_timing_enable": (i32, [vp, C.c_int]),
        "chrf_timing_report": (i32, [vp, C.c_char_p, sz]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != CHRF_OK:
        raise ChrfError(status, load().chrf_last_error().decode())
    return status
