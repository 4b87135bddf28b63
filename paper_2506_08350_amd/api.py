"""PyTorch-facing wrapper of the C ABI: device memory, streams and autograd.

Every step of the hot path runs in the HIP library; this module only
allocates tensors, passes their pointers and the current HIP stream, and
wires chrf_backward into torch.autograd.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check

PARAM_NAMES = ("means", "log_scales", "quats", "opacity", "amp", "phase")
LAYER_LOGITS = "logits"   # [N, layers] plane-assignment logits of a layered renderer


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_tensor(t, name, shape=None, dtype=torch.float32):
    """The library reads raw pointers, so every tensor handed to it must be a
    contiguous device tensor of the expected element type and shape."""
    if t is None:
        return
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name}: expected a contiguous {dtype} device tensor, got "
                        f"{getattr(t, 'dtype', type(t))} on {getattr(t, 'device', '?')}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


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
                 deterministic=False, fft_plans=(0, 0), device=0):
        """layered=True: multi-layer hologram with one layer per entry of
        optics.distances (the layer-to-hologram distances Z_l); the Gaussians
        then carry "logits" [N, layers] and the forward's "field" is the
        recorded hologram P.  loss: "mse" (Eq. 17) or "paper" (the masked
        three-term reconstruction loss plus ssim_weight * (1 - SSIM)).
        deterministic=True: gradients reproducible bit for bit (per-pair rows
        summed in a fixed order instead of float atomics; single-plane only).
        fft_plans: (row, column) radix schedules of the tuned transforms
        (chrf_plan_desc.fft_rows_plan / fft_cols_plan; 0 = default)."""
        self._config = dict(height=height, width=width, optics=optics, n_views=n_views, max_gaussians=max_gaussians,
                            n_lambda=n_lambda, max_pairs=max_pairs, k_sigma=k_sigma, alpha_min=alpha_min,
                            alpha_max=alpha_max, t_min=t_min, tile=tile, cols_per_block=cols_per_block,
                            layered=layered, loss=loss, ssim_weight=ssim_weight, phase_only=phase_only,
                            deterministic=deterministic, fft_plans=tuple(fft_plans), device=device)
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
        d.deterministic = 1 if deterministic else 0
        d.fft_rows_plan, d.fft_cols_plan = int(fft_plans[0]), int(fft_plans[1])
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
        # Counts the calls that rewrite the state a backward reads from the
        # workspace (forward, propagate, phase-only step); the autograd path
        # checks it so that a backward never runs against a later forward.
        self.generation = 0

    def __del__(self):
        if getattr(self, "plan", None) is not None and self.plan.value:
            self.lib.chrf_plan_destroy(self.plan)
            self.plan = C.c_void_p()

    def resized(self, max_gaussians=None, max_pairs=None):
        """A new renderer with the same configuration and other capacities."""
        cfg = dict(self._config)
        if max_gaussians is not None:
            cfg["max_gaussians"] = int(max_gaussians)
        if max_pairs is not None:
            cfg["max_pairs"] = int(max_pairs)
        return Renderer(**cfg)

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
        n = int(p["means"].shape[0])
        g.n = n
        shapes = dict(means=(n, 3), log_scales=(n, 3), quats=(n, 4), opacity=(n,), amp=(n, self.L),
                      phase=(n, self.L))
        for k in PARAM_NAMES:
            _check_tensor(p[k], k, shapes[k])
            setattr(g, k, p[k].data_ptr())
        if self.layered:
            _check_tensor(p[LAYER_LOGITS], LAYER_LOGITS, (n, self.K))
            g.logits = p[LAYER_LOGITS].data_ptr()
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
        _check_tensor(cams, "cams", (B, 20))
        _check_tensor(target, "target", (B, L, K, H, W))
        _check_tensor(masks, "masks", (B, K, H, W), torch.uint8)
        g = self._gauss(params)
        self.generation += 1
        check(self.lib.chrf_forward(self.plan, C.byref(g), _ptr(cams), _ptr(self.workspace), _ptr(field),
                                    _ptr(prop), _ptr(inten), _ptr(target), _ptr(masks), _ptr(loss), _stream()))
        self._saved = (target, masks, prop, inten)   # read again by a backward of the "paper" loss
        return {"field": field, "prop": prop, "intensity": inten, "loss": loss}

    def backward(self, params: dict, cams: torch.Tensor, dL_dI=None, prop=None, dL_dprop=None, dL_dfield=None,
                 grad_scale=None):
        B, L, K, H, W = self.B, self.L, self.K, self.H, self.W
        _check_tensor(cams, "cams", (B, 20))
        _check_tensor(dL_dI, "dL_dI", (B, L, K, H, W))
        _check_tensor(prop, "prop", (B, L, K, H, W, 2))
        _check_tensor(dL_dprop, "dL_dprop", (B, L, K, H, W, 2))
        _check_tensor(dL_dfield, "dL_dfield", (B, L, H, W, 2))
        _check_tensor(grad_scale, "grad_scale", ())
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
        _check_tensor(field, "field", (B, L, H, W, 2))
        prop = torch.empty((B, L, K, H, W, 2), dtype=torch.float32, device=self.device) if want_prop else None
        inten = torch.empty((B, L, K, H, W), dtype=torch.float32, device=self.device) if want_intensity else None
        self.generation += 1
        check(self.lib.chrf_propagate(self.plan, _ptr(field), _ptr(self.workspace), _ptr(prop), _ptr(inten),
                                      _stream()))
        return prop, inten

    def phase_only_step(self, targets: torch.Tensor, phi: torch.Tensor):
        """Loss and dL/dphi of the phase-only hologram exp(j phi) against the
        propagated target fields (plan created with phase_only=True)."""
        _check_tensor(targets, "targets", (self.B, self.L, self.K, self.H, self.W, 2))
        _check_tensor(phi, "phi", (self.B, self.L, self.H, self.W))
        loss = torch.empty((), dtype=torch.float32, device=self.device)
        dphi = torch.empty_like(phi)
        self.generation += 1
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

    def densify_stats(self, n: int, accum: torch.Tensor, count: torch.Tensor):
        """After a backward: add ||dL/d mu_2D|| of every view that binned each of
        the first n Gaussians to accum and the number of such views to count."""
        for t in (accum, count):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() >= n
        check(self.lib.chrf_densify_stats(self.plan, _ptr(self.workspace), int(n), _ptr(accum), _ptr(count),
                                          _stream()))

    def propagate_adjoint(self, grad_prop: torch.Tensor):
        _check_tensor(grad_prop, "grad_prop", (self.B, self.L, self.K, self.H, self.W, 2))
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


ADAN_BETAS = (0.9, 0.92, 0.99)


def adan_step(param: torch.Tensor, grad: torch.Tensor, state: dict, lr: float, step: int, betas=ADAN_BETAS,
              eps=1e-8, weight_decay=0.0):
    """In-place Adan update of a float32 device tensor by the library kernel;
    ``state`` holds grad_prev, m, v, n (created zeroed on first use)."""
    lib = _lib.load()
    for k in ("grad_prev", "m", "v", "n"):
        if k not in state:
            state[k] = torch.zeros_like(param)
    for t in (param, grad, *(state[k] for k in ("grad_prev", "m", "v", "n"))):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == param.numel()
    check(lib.chrf_adan_step(_ptr(param), _ptr(grad), _ptr(state["grad_prev"]), _ptr(state["m"]), _ptr(state["v"]),
                             _ptr(state["n"]), param.numel(), lr, betas[0], betas[1], betas[2], eps, weight_decay,
                             int(step), _stream()))


@dataclass
class DensifyConfig:
    """Thresholds of the densification (the 3DGS values; the phase perturbation
    size is not given by the paper)."""
    tau_grad: float = 2e-4 * 1080          # mean ||dL/d mu_2D|| in pixels
    split_scale: float = 0.05              # world-space scale above which a growing Gaussian splits
    prune_scale: float = 1.0               # world-space scale above which a Gaussian is pruned
    min_opacity: float = 0.005
    phase_sigma: float = 0.01              # radians
    shrink: float = float(math.log(1.6))


def densify(params: dict, opacity: torch.Tensor, accum: torch.Tensor, count: torch.Tensor, xi: torch.Tensor,
            zeta: torch.Tensor, cfg: DensifyConfig = DensifyConfig(), capacity=None, noalloc: bool = False):
    """Runs the library's densification.  params holds at least means,
    log_scales, quats and phase (float32 device tensors of n rows); opacity is
    the activated opacity used by the pruning test.  Returns (n_out, src, kind,
    means, log_scales, phase) with the new arrays cut to n_out rows; xi
    [n, 2, 3] and zeta [n, 2, n_lambda] are standard normal draws.  noalloc:
    call the library's allocation-free variant (its scratch is a device array
    the library holds) instead of passing a scratch buffer."""
    lib = _lib.load()
    n = int(params["means"].shape[0])
    n_lam = int(params["phase"].shape[1])
    cap = 2 * n if capacity is None else int(capacity)
    dev = params["means"].device
    d = _lib.DensifyDesc()
    d.n, d.n_lambda = n, n_lam
    arrays = dict(means=params["means"], log_scales=params["log_scales"], quats=params["quats"], opacity=opacity,
                  phase=params["phase"], grad_accum=accum, grad_count=count, xi=xi, zeta=zeta)
    for k, t in arrays.items():
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == n, k
        setattr(d, k, t.data_ptr())
    d.tau_grad = cfg.tau_grad
    d.sigma_split = math.log(cfg.split_scale)
    d.sigma_prune = math.log(cfg.prune_scale)
    d.min_opacity = cfg.min_opacity
    d.phase_sigma = cfg.phase_sigma
    d.shrink = cfg.shrink
    scratch = None if noalloc else torch.empty(int(lib.chrf_densify_workspace_bytes(n)), dtype=torch.uint8,
                                               device=dev)
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    kind = torch.empty(cap, dtype=torch.int32, device=dev)
    means = torch.empty((cap, 3), dtype=torch.float32, device=dev)
    log_scales = torch.empty((cap, 3), dtype=torch.float32, device=dev)
    phase = torch.empty((cap, n_lam), dtype=torch.float32, device=dev)
    n_out = torch.empty((), dtype=torch.int64, device=dev)
    if noalloc:
        check(lib.chrf_densify_noalloc(C.byref(d), cap, _ptr(src), _ptr(kind), _ptr(means), _ptr(log_scales),
                                       _ptr(phase), _ptr(n_out), _stream()))
    else:
        check(lib.chrf_densify(C.byref(d), _ptr(scratch), cap, _ptr(src), _ptr(kind), _ptr(means),
                               _ptr(log_scales), _ptr(phase), _ptr(n_out), _stream()))
    m = int(n_out)   # synchronises
    if m > cap:
        raise RuntimeError(f"densify: {m} outputs exceed the capacity {cap}")
    return m, src[:m], kind[:m], means[:m], log_scales[:m], phase[:m], n_out


def gather_rows(values: torch.Tensor, src: torch.Tensor, kind: torch.Tensor, n_out: torch.Tensor, zero_new: bool):
    """values [n, ...] carried through a densification: row j is values[src[j]]
    (zero for new Gaussians when zero_new)."""
    lib = _lib.load()
    m = int(src.shape[0])
    row = int(math.prod(values.shape[1:]))
    out = torch.empty((m,) + tuple(values.shape[1:]), dtype=torch.float32, device=values.device)
    assert values.dtype == torch.float32 and values.is_contiguous()
    check(lib.chrf_gather_rows(_ptr(values), row, _ptr(src), _ptr(kind), _ptr(n_out), m, 1 if zero_new else 0,
                               _ptr(out), _stream()))
    return out


def cosine_lr(step, total, lr0, lr_min):
    """Cosine annealing from lr0 at step 0 to lr_min at step ``total``."""
    t = min(max(step, 0), total) / float(total)
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * t))


class Trainer:
    """The optimisation loop of the paper's training algorithm on given target
    intensities.  Each step renders and differentiates with the library (the
    plan's loss; straight-through plane assignment on a layered renderer),
    applies Adan to every parameter tensor with the paper's per-parameter
    learning rates (cosine annealing to lr_min for means and plane logits),
    and accumulates the view-space gradient statistics; every
    ``densify_every`` steps up to ``densify_until`` the Gaussians are pruned,
    cloned and split by the library.

    Parameters are kept raw: opacity as a logit (the library takes the
    activated value, so the sigmoid and its derivative are applied here).
    A renderer whose Gaussian or pair capacity becomes too small is replaced
    by a larger one of the same configuration."""

    LR = dict(means=0.01, log_scales=0.005, quats=0.001, opacity=0.025, amp=0.0025, phase=0.0025, logits=0.01)
    ANNEALED = ("means", LAYER_LOGITS)

    def __init__(self, renderer: Renderer, params: dict, cams: torch.Tensor, target: torch.Tensor, masks=None,
                 total_steps=20000, densify_every=300, densify_until=None, densify_cfg: DensifyConfig = None,
                 lr_min=1e-5, seed=0, pair_headroom=1.25):
        self.r = renderer
        self.cams, self.target, self.masks = cams, target, masks
        self.p = {k: params[k].detach().clone().contiguous() for k in renderer.param_names()}
        self.state = {k: {} for k in self.p}
        self.total_steps = int(total_steps)
        self.densify_every = int(densify_every)
        self.densify_until = int(densify_until if densify_until is not None else total_steps // 2)
        self.cfg = densify_cfg or DensifyConfig()
        self.lr_min = lr_min
        self.headroom = pair_headroom
        self.gen = torch.Generator(device=self.p["means"].device).manual_seed(seed)
        self.step_count = 0
        self.overflows = 0
        self._status_pending = None
        self._reset_stats()
        self._ensure_capacity()

    @property
    def n(self) -> int:
        return int(self.p["means"].shape[0])

    def _reset_stats(self):
        dev = self.p["means"].device
        self.accum = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.count = torch.zeros(self.n, dtype=torch.float32, device=dev)

    def render_params(self) -> dict:
        d = dict(self.p)
        d["opacity"] = torch.sigmoid(self.p["opacity"]).contiguous()
        return d

    def _ensure_capacity(self):
        if self.n > self.r.max_gaussians:
            self.r = self.r.resized(max_gaussians=int(math.ceil(1.5 * self.n)))
        self.r.forward(self.render_params(), self.cams, want_field=False, want_intensity=False)
        st, need = self.r.read_status()
        if st != 0:
            self.r = self.r.resized(max_pairs=int(need * self.headroom) + 4096)

    def _check_status(self):
        """Reads the pair-list status the previous step copied to host memory
        (its copy has long completed, so this does not stall the stream).  A
        step whose pairs overflowed had incomplete gradients: the renderer is
        replaced by one with room for the pairs it needed."""
        if self._status_pending is None:
            return
        host, done = self._status_pending
        self._status_pending = None
        done.synchronize()
        total = (int(host[0]) & 0xFFFFFFFF) | ((int(host[1]) & 0xFFFFFFFF) << 32)
        if int(host[3]) != 0:
            raise RuntimeError("radix sort: a look-back wait gave up; the step's pair lists were not valid")
        if int(host[2]) != 0:
            self.overflows += 1
            self.r = self.r.resized(max_pairs=int(total * self.headroom) + 4096)

    def _queue_status(self):
        """Copies the status words of the step just enqueued to pinned host
        memory, to be read at the next step."""
        host = torch.empty(4, dtype=torch.int32, pin_memory=True)
        status = self.r.region(_lib.REGION_STATUS, torch.int32)[:4]
        host.copy_(status, non_blocking=True)
        done = torch.cuda.Event()
        done.record(torch.cuda.current_stream())
        self._status_pending = (host, done)

    def step(self):
        """One training step; returns the loss (device scalar) before the update."""
        self._check_status()
        self.step_count += 1
        rp = self.render_params()
        loss, grads, _ = self.r.train_step(rp, self.cams, self.target, masks=self.masks)
        self._queue_status()
        o = rp["opacity"]
        grads["opacity"] = (grads["opacity"] * o * (1.0 - o)).contiguous()
        self.r.densify_stats(self.n, self.accum, self.count)
        for k, t in self.p.items():
            lr = self.LR[k]
            if k in self.ANNEALED:
                lr = cosine_lr(self.step_count, self.total_steps, lr, self.lr_min)
            adan_step(t, grads[k], self.state[k], lr, self.step_count)
        if self.step_count % self.densify_every == 0 and self.step_count <= self.densify_until:
            self.densify()
        return loss

    def densify(self):
        """Prune, clone and split by the accumulated statistics; parameters and
        optimiser state follow the library's index map (fresh state for new
        Gaussians)."""
        n = self.n
        dev = self.p["means"].device
        n_lam = int(self.p["phase"].shape[1])
        xi = torch.randn((n, 2, 3), generator=self.gen, device=dev, dtype=torch.float32)
        zeta = torch.randn((n, 2, n_lam), generator=self.gen, device=dev, dtype=torch.float32)
        opacity = torch.sigmoid(self.p["opacity"]).contiguous()
        m, src, kind, means, log_scales, phase, n_out = densify(self.p, opacity, self.accum, self.count, xi, zeta,
                                                                self.cfg)
        changed = {"means": means, "log_scales": log_scales, "phase": phase}
        new_p = {}
        for k, t in self.p.items():
            new_p[k] = changed[k].contiguous() if k in changed else gather_rows(t, src, kind, n_out, False)
        self.state = {k: {s: gather_rows(v, src, kind, n_out, True) for s, v in st.items()}
                      for k, st in self.state.items()}
        self.p = new_p
        self._reset_stats()
        self._ensure_capacity()
        return m


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
        ctx.generation = renderer.generation
        ctx.cams = cams
        ctx.params = params
        ctx.save_for_backward(out["prop"])
        return out["intensity"]

    @staticmethod
    def backward(ctx, dI):
        (prop,) = ctx.saved_tensors
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("render_intensity: the renderer ran another forward after this one; its workspace "
                               "(pair lists, transmittance) no longer belongs to this graph.  Use one renderer per "
                               "outstanding autograd forward.")
        st, need = r.read_status()
        if st == _lib.CHRF_ECAPACITY:
            raise _lib.ChrfError(st, f"pair list overflow in the forward ({need} pairs needed, capacity "
                                     f"{r.desc.max_pairs}); the gradient would be incomplete")
        check(st)
        grads = r.backward(ctx.params, ctx.cams, dL_dI=dI.contiguous(), prop=prop)
        g_logits = grads.get(LAYER_LOGITS)
        return (None, None) + tuple(grads[k] for k in PARAM_NAMES) + (g_logits,)


def render_intensity(renderer: Renderer, cams, means, log_scales, quats, opacity, amp, phase, logits=None):
    return HologramFunction.apply(renderer, cams, means, log_scales, quats, opacity, amp, phase, logits)
