"""PyTorch-facing wrapper of the C ABI: device memory, streams and autograd.

Every step of the hot path runs in the HIP library; this module only
allocates tensors, passes their pointers and the current HIP stream, and
wires chrf_backward into torch.autograd.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check

PARAM_NAMES = ("means", "log_scales", "quats", "opacity", "amp", "phase")
LAYER_LOGITS = "logits"   # [N, layers] plane-assignment logits of a layered renderer


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def pack_cameras(cameras, device="cuda") -> torch.Tensor:
    """Device tensor [n_views, 20] of chrf_camera records from objects with
    attributes R (3x3), t (3), fx, fy, cx, cy and optionally z_near."""
    rows = []
    for c in cameras:
        r = torch.zeros(20, dtype=torch.float32)
        r[0:9] = torch.as_tensor(c.R, dtype=torch.float32).reshape(9)
        r[9:12] = torch.as_tensor(c.t, dtype=torch.float32).reshape(3)
        r[12:17] = torch.tensor([c.fx, c.fy, c.cx, c.cy, getattr(c, "z_near", 0.01)], dtype=torch.float32)
        rows.append(r)
    return torch.stack(rows).to(device)


@dataclass
class Optics:
    wavelengths: tuple
    distances: tuple
    pitch: float
    pad: int = 2
    band_limit: int = 2


class Context:
    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        h = C.c_void_p()
        check(self.lib.chrf_create(device, C.byref(h)))
        self.handle = h
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.chrf_destroy(self.handle)
            self.handle = C.c_void_p()


_default_ctx = {}


def context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


class Renderer:
    """One plan (shapes, optics, thresholds) plus its device workspace."""

    def __init__(self, height, width, optics: Optics, n_views=1, max_gaussians=1, n_lambda=None,
                 max_pairs=0, k_sigma=3.0, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4,
                 tile=None, cols_per_block=0, layered=False, loss="mse", ssim_weight=0.005, phase_only=False,
                 device=0):
        """layered=True: multi-layer hologram with one layer per entry of
        optics.distances (the layer-to-hologram distances Z_l); the Gaussians
        then carry "logits" [N, layers] and the forward's "field" is the
        recorded hologram P.  loss: "mse" (Eq. 17) or "paper" (the masked
        three-term reconstruction loss plus ssim_weight * (1 - SSIM))."""
        self.ctx = context(device)
        self.lib = self.ctx.lib
        d = _lib.PlanDesc()
        d.height, d.width = int(height), int(width)
        d.n_views = int(n_views)
        d.n_lambda = int(n_lambda if n_lambda is not None else len(optics.wavelengths))
        d.n_planes = len(optics.distances)
        d.max_gaussians = int(max_gaussians)
        d.max_pairs = int(max_pairs)
        d.pad_factor = int(optics.pad)
        d.band_limit = int(optics.band_limit)
        d.pitch = float(optics.pitch)
        for i, lam in enumerate(optics.wavelengths):
            d.wavelengths[i] = float(lam)
        for i, z in enumerate(optics.distances):
            d.distances[i] = float(z)
        d.k_sigma, d.alpha_min, d.alpha_max, d.t_min = k_sigma, alpha_min, alpha_max, t_min
        if tile is None:
            tile = (16, 16)
        d.tile_w, d.tile_h = int(tile[0]), int(tile[1])
        d.cols_per_block = int(cols_per_block)
        d.layered = 1 if layered else 0
        self.layered = bool(layered)
        if loss not in ("mse", "paper"):
            raise ValueError(f"unknown loss {loss!r}")
        d.loss_kind = 1 if loss == "paper" else 0
        d.ssim_weight = float(ssim_weight)
        d.phase_only = 1 if phase_only else 0
        self.loss = loss
        self.desc = d
        h = C.c_void_p()
        check(self.lib.chrf_plan_create(self.ctx.handle, C.byref(d), C.byref(h)))
        self.plan = h
        self.optics = optics
        self.H, self.W, self.B = d.height, d.width, d.n_views
        self.L, self.K = d.n_lambda, d.n_planes
        self.max_gaussians = d.max_gaussians
        nbytes = int(self.lib.chrf_plan_workspace_bytes(self.plan))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")
        self.device = torch.device(f"cuda:{device}")

    def __del__(self):
        if getattr(self, "plan", None) is not None and self.plan.value:
            self.lib.chrf_plan_destroy(self.plan)
            self.plan = C.c_void_p()

    # ---- inspection ----
    def region(self, region: int, dtype=torch.uint8):
        off, nb = C.c_size_t(), C.c_size_t()
        check(self.lib.chrf_plan_region(self.plan, region, C.byref(off), C.byref(nb)))
        raw = self.workspace[off.value: off.value + nb.value]
        return raw.view(dtype)

    def read_status(self):
        need = C.c_int64()
        st = self.lib.chrf_read_status(self.plan, _ptr(self.workspace), C.byref(need), _stream())
        return st, need.value

    def timing(self, enable: bool):
        check(self.lib.chrf_timing_enable(self.plan, 1 if enable else 0))

    def timing_report(self) -> dict:
        buf = C.create_string_buffer(1 << 16)
        check(self.lib.chrf_timing_report(self.plan, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, count, ms = line.split()
            out[name] = (int(count), float(ms))
        return out

    # ---- calls ----
    def _gauss(self, p):
        g = _lib.Gaussians()
        g.n = int(p["means"].shape[0])
        for k in PARAM_NAMES:
            t = p[k]
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), k
            setattr(g, k, t.data_ptr())
        if self.layered:
            t = p[LAYER_LOGITS]
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape == (g.n, self.K)
            g.logits = t.data_ptr()
        return g

    def param_names(self):
        return PARAM_NAMES + ((LAYER_LOGITS,) if self.layered else ())

    def forward(self, params: dict, cams: torch.Tensor, want_field=True, want_prop=False, want_intensity=True,
                target=None, masks=None):
        """masks: uint8 [views, planes, H, W] plane masks of the "paper" loss
        (kept alive until the backward, like target)."""
        B, L, K, H, W = self.B, self.L, self.K, self.H, self.W
        dev = self.device
        field = torch.empty((B, L, H, W, 2), dtype=torch.float32, device=dev) if want_field else None
        prop = torch.empty((B, L, K, H, W, 2), dtype=torch.float32, device=dev) if want_prop else None
        inten = torch.empty((B, L, K, H, W), dtype=torch.float32, device=dev) if want_intensity else None
        loss = torch.empty((), dtype=torch.float32, device=dev) if target is not None else None
        if target is not None:
            assert target.shape == (B, L, K, H, W) and target.is_contiguous()
        if masks is not None:
            assert masks.shape == (B, K, H, W) and masks.dtype == torch.uint8 and masks.is_contiguous()
        g = self._gauss(params)
        check(self.lib.chrf_forward(self.plan, C.byref(g), _ptr(cams), _ptr(self.workspace), _ptr(field),
                                    _ptr(prop), _ptr(inten), _ptr(target), _ptr(masks), _ptr(loss), _stream()))
        self._saved = (target, masks, prop, inten)   # read again by a backward of the "paper" loss
        return {"field": field, "prop": prop, "intensity": inten, "loss": loss}

    def backward(self, params: dict, cams: torch.Tensor, dL_dI=None, prop=None, dL_dprop=None, dL_dfield=None,
                 grad_scale=None):
        grads = {k: torch.empty_like(params[k]) for k in self.param_names()}
        gr = _lib.Grads(*[grads[k].data_ptr() for k in PARAM_NAMES])
        if self.layered:
            gr.logits = grads[LAYER_LOGITS].data_ptr()
        g = self._gauss(params)
        check(self.lib.chrf_backward(self.plan, C.byref(g), _ptr(cams), _ptr(self.workspace), _ptr(dL_dI),
                                     _ptr(prop), _ptr(dL_dprop), _ptr(dL_dfield), _ptr(grad_scale),
                                     C.byref(gr), _stream()))
        return grads

    def train_step(self, params: dict, cams: torch.Tensor, target: torch.Tensor, want_intensity=False, masks=None):
        """Forward with the plan's loss, then the backward: (loss, grads)."""
        out = self.forward(params, cams, want_field=False, want_prop=False, want_intensity=want_intensity,
                           target=target, masks=masks)
        grads = self.backward(params, cams)
        return out["loss"], grads, out

    def propagate(self, field: torch.Tensor, want_prop=True, want_intensity=True):
        B, L, K, H, W = self.B, self.L, self.K, self.H, self.W
        prop = torch.empty((B, L, K, H, W, 2), dtype=torch.float32, device=self.device) if want_prop else None
        inten = torch.empty((B, L, K, H, W), dtype=torch.float32, device=self.device) if want_intensity else None
        check(self.lib.chrf_propagate(self.plan, _ptr(field), _ptr(self.workspace), _ptr(prop), _ptr(inten),
                                      _stream()))
        return prop, inten

    def phase_only_step(self, targets: torch.Tensor, phi: torch.Tensor):
        """Loss and dL/dphi of the phase-only hologram exp(j phi) against the
        propagated target fields (plan created with phase_only=True)."""
        assert targets.shape == (self.B, self.L, self.K, self.H, self.W, 2) and targets.is_contiguous()
        assert phi.shape == (self.B, self.L, self.H, self.W) and phi.is_contiguous()
        loss = torch.empty((), dtype=torch.float32, device=self.device)
        dphi = torch.empty_like(phi)
        check(self.lib.chrf_phase_only_step(self.plan, _ptr(targets), _ptr(phi), _ptr(self.workspace), _ptr(loss),
                                            _ptr(dphi), _stream()))
        return loss, dphi

    def convert_phase_only(self, hologram: torch.Tensor, steps=200, lr=0.05, phi0=None):
        """Phase-only conversion of a complex hologram [B, L, H, W, 2]: Adam on
        phi (library kernels for the loss, gradient and update), starting from
        the hologram's own phase.  Returns (phi, losses)."""
        targets, _ = self.propagate(hologram, want_intensity=False)
        phi = (torch.atan2(hologram[..., 1], hologram[..., 0]) if phi0 is None else phi0).contiguous().clone()
        m = torch.zeros_like(phi)
        v = torch.zeros_like(phi)
        losses = []
        for t in range(1, steps + 1):
            loss, dphi = self.phase_only_step(targets, phi)
            adam_step(phi, dphi, m, v, lr, step=t)
            losses.append(loss)
        return phi, torch.stack(losses)

    def propagate_adjoint(self, grad_prop: torch.Tensor):
        out = torch.empty((self.B, self.L, self.H, self.W, 2), dtype=torch.float32, device=self.device)
        check(self.lib.chrf_propagate_adjoint(self.plan, _ptr(grad_prop), _ptr(self.workspace), _ptr(out),
                                              _stream()))
        return out


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float, step: int,
              beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of a float32 device tensor by the library kernel."""
    lib = _lib.load()
    for t in (param, grad, m, v):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == param.numel()
    check(lib.chrf_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), lr, beta1, beta2, eps,
                             int(step), _stream()))


class CapturedTrainStep:
    """The fused training step (forward with the plan's loss, then the
    backward) captured once in a HIP graph and replayed.

    The graph holds the pointers of ``params``, ``cams``, ``target`` and
    ``masks``: update those tensors in place (``copy_``) between replays.  ``loss`` and ``grads``
    are overwritten by every replay.  The library's forward and backward
    enqueue no synchronisation, allocation or memset, so the whole sequence
    (projection, sorts, raster, propagation, backward) is capturable.
    """

    def __init__(self, renderer: Renderer, params: dict, cams: torch.Tensor, target: torch.Tensor, warmup: int = 2,
                 masks=None):
        self.renderer = renderer
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                renderer.train_step(params, cams, target, masks=masks)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.loss, self.grads, _ = renderer.train_step(params, cams, target, masks=masks)

    def replay(self):
        self.graph.replay()
        return self.loss, self.grads


class HologramFunction(torch.autograd.Function):
    """Intensities [B, L, K, H, W] of the propagated complex field, differentiable
    w.r.t. all six Gaussian parameter tensors (and the layer logits of a
    layered renderer, through the straight-through estimator) by the
    library's backward."""

    @staticmethod
    def forward(ctx, renderer: Renderer, cams, means, log_scales, quats, opacity, amp, phase, logits=None):
        params = dict(zip(PARAM_NAMES, (means, log_scales, quats, opacity, amp, phase)))
        if renderer.layered:
            params[LAYER_LOGITS] = logits
        params = {k: v.detach().contiguous() for k, v in params.items()}
        out = renderer.forward(params, cams, want_field=False, want_prop=True, want_intensity=True)
        ctx.renderer = renderer
        ctx.cams = cams
        ctx.params = params
        ctx.save_for_backward(out["prop"])
        return out["intensity"]

    @staticmethod
    def backward(ctx, dI):
        (prop,) = ctx.saved_tensors
        grads = ctx.renderer.backward(ctx.params, ctx.cams, dL_dI=dI.contiguous(), prop=prop)
        g_logits = grads.get(LAYER_LOGITS)
        return (None, None) + tuple(grads[k] for k in PARAM_NAMES) + (g_logits,)


def render_intensity(renderer: Renderer, cams, means, log_scales, quats, opacity, amp, phase, logits=None):
    return HologramFunction.apply(renderer, cams, means, log_scales, quats, opacity, amp, phase, logits)
