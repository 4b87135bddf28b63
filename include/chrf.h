/*
 * chrf.h -- C ABI of the MI355X (gfx950) complex-hologram renderer.
 *
 * The library renders complex-valued 3D Gaussians into a complex field and
 * propagates it to several planes with the band-limited angular spectrum
 * method, then returns |u|^2 per plane; it also runs the analytic backward of
 * that map.  The calls follow the problem statement of the paper
 * (Complex-Valued Holographic Radiance Fields, Sec. 3 "Hologram Plane, Camera
 * and Problem Definition"): Gaussians k = (c, x, R, S, alpha, phi) (Sec. 4.1,
 * Eq. 9), a camera with pitch and resolution, wavelengths and propagation
 * distances in; the complex field U and the intensities I_l = |u_l|^2
 * (Eq. 16) out.
 *
 * Conventions shared by every call
 * - All array arguments are device pointers to caller-owned memory (for
 *   example torch tensors), FP32, C-contiguous, unless a comment says "host".
 *   Complex arrays are interleaved (re, im) float pairs.
 * - Every call is asynchronous on the given HIP stream (NULL = the null
 *   stream) and does not synchronise, except chrf_read_status.
 * - Argument checks happen before anything is enqueued; a failing check
 *   returns a negative status and enqueues nothing.  chrf_last_error() then
 *   describes the failure.  No C++ exception crosses this interface.
 * - A plan is not thread-safe; use one plan per stream.  Workspace contents
 *   written by chrf_forward stay valid for chrf_backward until the next
 *   chrf_forward on the same plan and workspace.
 */
#ifndef CHRF_H_
#define CHRF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum chrf_status {
  CHRF_OK = 0,
  CHRF_EINVAL = -1,        /* bad argument (null pointer, size, option) */
  CHRF_ENOMEM = -2,        /* host or device allocation failed */
  CHRF_EHIP = -3,          /* a HIP runtime call failed */
  CHRF_ECAPACITY = -4,     /* the tile-pair list overflowed its capacity */
  CHRF_EUNSUPPORTED = -5   /* shape or option this build does not handle */
} chrf_status;

typedef struct chrf_ctx chrf_ctx;   /* one per device: twiddle tables */
typedef struct chrf_plan chrf_plan; /* shapes, optics, options, workspace layout */

/*
 * Pinhole camera (Sec. 3: pose r and the hologram plane it carries; the
 * Euler-angle pose is converted to R, t by the caller).  x_cam = R x + t with
 * camera axes x right, y down, z forward; the projection of Eq. 8 is
 * mu = (fx x_cam/z_cam + cx, fy y_cam/z_cam + cy) in pixels, the centre of
 * pixel (row r, column c) being (c + 0.5, r + 0.5).  Gaussians with
 * z_cam <= z_near are culled.  80 bytes; passed as a device array [n_views].
 */
typedef struct chrf_camera {
  float R[9]; /* row-major */
  float t[3];
  float fx, fy, cx, cy;
  float z_near;
  float reserved[3];
} chrf_camera;

/*
 * Complex Gaussians k = (c, x, R, S, alpha, phi, rho') of Eq. 9.  Device arrays:
 *   means [n,3]; log_scales [n,3] (S = diag(exp(s))); quats [n,4] as
 *   (w, x, y, z) of any nonzero norm (normalised inside); opacity [n] already
 *   activated, in (0,1); amp [n, n_lambda] (c, the wave amplitude); phase
 *   [n, n_lambda] in radians (phi); logits [n, n_planes], the raw plane
 *   assignment logits rho' of a layered plan (Eq. 12; NULL for a
 *   single-plane plan, where rho = 1).
 */
typedef struct chrf_gaussians {
  int32_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity;
  const float* amp;
  const float* phase;
  const float* logits;
} chrf_gaussians;

/* Gradients, same shapes as chrf_gaussians; every non-NULL array is
 * overwritten.  logits (layered plans only, may be NULL) receives the
 * straight-through gradient dL/drho' = dL/drho * softmax(rho' / 0.001)
 * (Eq. 12, backward). */
typedef struct chrf_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity;
  float* amp;
  float* phase;
  float* logits;
} chrf_grads;

/*
 * Plan description (host struct).
 *   height x width     field size (n_y x n_x of Sec. 3), both <= 4096
 *   n_views            cameras rendered per call (batch)
 *   n_lambda           wavelengths, 1..4
 *   n_planes           propagation distances K, 1..64
 *   max_gaussians      largest n accepted by this plan
 *   max_pairs          capacity of the (tile, Gaussian) list over all views;
 *                      0 selects 128 * n_views * max_gaussians, capped at 2^28
 *   pad_factor         1 or 2: the propagation grid is pad_factor times the
 *                      field in each dimension (zero padding, top-left)
 *   band_limit         0: none: every bin is kept, a bin with f^2 > 1/lambda^2
 *                      taking the decaying continuation of Eq. 7,
 *                      exp(-2 pi |z| sqrt(f^2 - 1/lambda^2));
 *                      1: cut f^2 > 1/lambda^2 (Eq. 7); 2: also the sampling
 *                      band limit |f_x| <= 1/(lambda sqrt((2 df_x z)^2 + 1)),
 *                      likewise in y, with df = 1/(padded size * pitch)
 *   pitch              pixel pitch in metres (Delta x of Sec. 3)
 *   wavelengths        metres, n_lambda entries
 *   distances          metres, signed, n_planes entries (Eqs. 14 and 16)
 *   k_sigma            support half-width in standard deviations (3)
 *   alpha_min, alpha_max, t_min   compositing thresholds (1/255, 0.99, 1e-4):
 *                      a Gaussian contributes where a >= alpha_min; a is
 *                      clamped at alpha_max, which must be below 1 (the
 *                      backward recovers the transmittance in front of a
 *                      Gaussian by dividing by 1 - a, Sec. 4.2); a pixel
 *                      stops after T < t_min
 *   tile_w, tile_h     raster tile, multiples of 8 with tile_w*tile_h in {64,128,256}
 *                      (0, 0 selects 16 x 16, the tile of Sec. 4.2)
 *   cols_per_block     columns per workgroup in the column FFT passes
 *                      (0 = choose from the LDS size)
 *   layered            0: single plane (rho = 1): the rendered field U is
 *                      propagated to every distance z_k.
 *                      1: multi-layer hologram (Sec. 4.1, Eqs. 12-16) with
 *                      n_planes layers, 1..4, at distances Z_l (metres,
 *                      layer to hologram plane): every Gaussian joins the
 *                      layer of its largest logit and composites only with
 *                      that layer (per-layer transmittance and early
 *                      termination); the hologram is recorded as
 *                      P = sum_l ASM(U_l; +Z_l) and propagated back to every
 *                      layer, u_k = ASM(P; -Z_k), I_k = |u_k|^2.
 *   loss_kind          loss computed by chrf_forward when a target is given:
 *                      0: MSE, the mean of (I - T)^2 over all elements (Eq. 17);
 *                      1: the paper's training loss (Sec. 4.1): the
 *                      three-term reconstruction loss with plane masks M,
 *                      mean of (I - T)^2 (1 + M + T^2), plus
 *                      ssim_weight * (1 - mean SSIM(I, T)) (11 x 11 Gaussian
 *                      window, sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, zero
 *                      padding; one SSIM per view, wavelength and plane)
 *   ssim_weight        lambda_1 of the SSIM term (0.005 in the paper)
 *   phase_only         1: reserve the workspace of chrf_phase_only_step
 *   deterministic      1: gradients reproducible bit for bit from run to run
 *                      (single-plane plans): instead of adding per-pair
 *                      gradient sums to the per-(view, Gaussian) rows with
 *                      float atomics, the backward stores one row per
 *                      (tile, Gaussian) pair and a second kernel sums each
 *                      Gaussian's rows in the fixed order of its tiles (the
 *                      per-view rows are then summed over views in view
 *                      order, as always).  Costs workspace of about
 *                      4 (2 + per-Gaussian row length) bytes per pair and
 *                      two extra passes over it.
 *   fft_rows_plan      radix schedule of the row transforms when the padded
 *                      width is 3840 (0: 16*16*15, 1: 16*15*16, 2: 15*16*16)
 *                      or 7680 (0: 16*20*24, 1: 16*24*20, 2: 24*20*16);
 *                      must be 0 for other widths
 *   fft_cols_plan      radix schedule of the column transforms when the
 *                      padded height is 2160 and cols_per_block is 2 (0:
 *                      16*15*9, 1: 16*9*15, 2: 15*16*9, 3: 12*12*15, in
 *                      forward stage order), or 4320 with height = 2160
 *                      (cols_per_block 0, 1 or 2; each column runs as two
 *                      transforms of 2160 with the same four schedules);
 *                      must be 0 otherwise.  Schedules change
 *                      rounding only (CHRF_EUNSUPPORTED for a value out of
 *                      range); the autotuner picks them.
 */
typedef struct chrf_plan_desc {
  int32_t height, width;
  int32_t n_views, n_lambda, n_planes;
  int32_t max_gaussians;
  int64_t max_pairs;
  int32_t pad_factor;
  int32_t band_limit;
  double pitch;
  double wavelengths[4];
  double distances[64];
  float k_sigma, alpha_min, alpha_max, t_min;
  int32_t tile_w, tile_h;
  int32_t cols_per_block;
  int32_t layered;
  int32_t loss_kind;
  float ssim_weight;
  int32_t phase_only;
  int32_t deterministic;
  int32_t fft_rows_plan, fft_cols_plan;
} chrf_plan_desc;

/* Named regions of the workspace, for inspection by tests and tools. */
typedef enum chrf_region {
  CHRF_REGION_PAIR_KEYS = 0,   /* uint32 [max_pairs]: view << b | tile, b = bits of n_tiles - 1, stably
                                  sorted by the b tile bits (or by the low 8 ceil(b / 8) bits when the
                                  capacity takes single-sweep passes); each (view, tile) run is
                                  contiguous and front to back (runs sharing the sorted bits follow in
                                  view order) */
  CHRF_REGION_PAIR_VALUES = 1, /* uint32 [max_pairs]: view * max_gaussians + gaussian */
  CHRF_REGION_TILE_RANGES = 2, /* uint32 [n_views * n_tiles][2]: [start, end) of (view, tile) view * n_tiles + tile */
  CHRF_REGION_STATUS = 3,      /* uint64 [0] pairs needed, uint32 [2] overflow flag */
  CHRF_REGION_T_FINAL = 4,     /* float [n_views][H][W] transmittance after compositing */
  CHRF_REGION_LAST = 5,        /* uint32 [n_views][H][W] last included pair + 1 */
  CHRF_REGION_FIELD = 6,       /* complex [n_views][n_lambda][H][W] rendered field */
  CHRF_REGION_GRAD_FIELD = 7,  /* complex [n_views][n_lambda][H][W] dL/dU after backward */
  /* layered plans only (zero bytes otherwise) */
  CHRF_REGION_LAYER_FIELDS = 8,  /* complex [n_views][n_lambda][n_planes][H][W] layer fields U_l */
  CHRF_REGION_LAYER_T_FINAL = 9, /* float [n_views][n_planes][H][W] transmittance of each layer */
  CHRF_REGION_LAYER_STOP = 10,   /* uint32 [n_views][n_planes][H][W] pair + 1 that ended the layer, ~0 if none */
  CHRF_REGION_LAYER_GRAD = 11,   /* complex [n_views][n_lambda][n_planes][H][W] dL/dU_l after backward */
  CHRF_REGION_LOSS_PARTIAL = 12, /* float [n_views][n_lambda][n_planes][H]: MSE row sums of the last forward */
  CHRF_REGION_COUNT
} chrf_region;

/* Create a context on HIP device `device`; *out receives it.  Errors:
 * CHRF_EINVAL (null out), CHRF_EHIP (device unusable), CHRF_ENOMEM. */
chrf_status chrf_create(int device, chrf_ctx** out);
/* Release a context and its device tables; plans made from it must be destroyed first. */
void chrf_destroy(chrf_ctx* ctx);
/* Text of the last failure on this thread (static storage; never NULL). */
const char* chrf_last_error(void);
/* Library version string. */
const char* chrf_version(void);

/* Validate desc and build a plan (host object + small device tables).
 * Errors: CHRF_EINVAL, CHRF_EUNSUPPORTED (size/radix/LDS limits), CHRF_EHIP, CHRF_ENOMEM. */
chrf_status chrf_plan_create(chrf_ctx* ctx, const chrf_plan_desc* desc, chrf_plan** out);
/* Destroy a plan.  It frees no device memory itself (its small tables are
 * released by the next chrf_plan_create or by chrf_destroy), so it may be
 * called while another stream is being captured into a HIP graph. */
void chrf_plan_destroy(chrf_plan* plan);
/* Bytes of device workspace the caller must allocate (256-byte aligned start). */
size_t chrf_plan_workspace_bytes(const chrf_plan* plan);
/* Offset and size in bytes of a region inside the workspace. */
chrf_status chrf_plan_region(const chrf_plan* plan, int region, size_t* offset, size_t* bytes);

/*
 * Forward pass: project and cull (Eqs. 2-4, 8), bin into tiles and sort by
 * depth (Algorithm 2), composite front to back (Eqs. 10, 13 with one plane),
 * propagate every wavelength to every distance (Eqs. 7, 14, 16).  A layered
 * plan composites every layer (Eq. 13), records the hologram P (Eqs. 14-15)
 * and propagates it back to the layers (Eq. 16).
 *   cams            device [n_views] chrf_camera
 *   workspace       device, chrf_plan_workspace_bytes() bytes
 *   field_out       complex [n_views][n_lambda][H][W] or NULL: the rendered
 *                   field U, or for a layered plan the hologram P
 *   prop_out        complex [n_views][n_lambda][n_planes][H][W] or NULL (u)
 *   intensity_out   float   [n_views][n_lambda][n_planes][H][W] or NULL (|u|^2)
 *   target          float   same shape as intensity, or NULL; when given,
 *                   loss_out (device float scalar) receives the plan's loss
 *                   (loss_kind) and the workspace is prepared for
 *                   chrf_backward with dL_dI = NULL.  With loss_kind 1 the
 *                   target, masks, prop_out and intensity_out buffers are read
 *                   again by that chrf_backward and must stay unchanged.
 *   masks           uint8 [n_views][n_planes][H][W] (0/1) plane masks of
 *                   loss_kind 1, or NULL (all zero); ignored otherwise
 * A pair-list overflow is not reported here (no synchronisation); outputs are
 * then incomplete but every access stays in bounds, and chrf_read_status
 * reports CHRF_ECAPACITY.
 */
chrf_status chrf_forward(chrf_plan* plan, const chrf_gaussians* g, const chrf_camera* cams, void* workspace,
                         float* field_out, float* prop_out, float* intensity_out, const float* target,
                         const uint8_t* masks, float* loss_out, void* hip_stream);

/*
 * Backward pass (Supplementary D): gradients of the loss w.r.t. every
 * Gaussian parameter, summed over views.
 *   dL_dI      float [n_views][n_lambda][n_planes][H][W] or NULL.  NULL means:
 *              use the loss of the last chrf_forward that had a target.
 *   prop       complex u saved from chrf_forward (prop_out); required when
 *              dL_dI is given
 *   dL_dprop   complex, same shape as prop, or NULL
 *   dL_dfield  complex [n_views][n_lambda][H][W] or NULL (dL/dP for a layered plan)
 *   grad_scale device float scalar multiplying all of the above, or NULL (1)
 *   out        gradients (overwritten)
 */
chrf_status chrf_backward(chrf_plan* plan, const chrf_gaussians* g, const chrf_camera* cams, void* workspace,
                          const float* dL_dI, const float* prop, const float* dL_dprop, const float* dL_dfield,
                          const float* grad_scale, const chrf_grads* out, void* hip_stream);

/*
 * Propagation only (Eqs. 14/16 on a given field): field [n_views][n_lambda][H][W]
 * complex -> prop_out (complex, may be NULL) and intensity_out (may be NULL).
 * For a layered plan this is the inverse propagation of a hologram P to the
 * layers (distances -Z_k), and chrf_propagate_adjoint, its adjoint, is the
 * forward recording of layer fields into P (Eqs. 14-15).
 */
chrf_status chrf_propagate(chrf_plan* plan, const float* field, void* workspace, float* prop_out,
                           float* intensity_out, void* hip_stream);
/*
 * Adjoint of chrf_propagate's field -> prop map:
 * grad_prop [n_views][n_lambda][n_planes][H][W] complex -> grad_field
 * [n_views][n_lambda][H][W] complex (sum over planes of the conjugate-transfer
 * propagation).
 */
chrf_status chrf_propagate_adjoint(chrf_plan* plan, const float* grad_prop, void* workspace, float* grad_field,
                                   void* hip_stream);

/*
 * Phase-only hologram conversion, one loss/gradient evaluation (the paper's
 * phase-only conversion: a phase-only hologram P_phi = exp(j phi) and the
 * complex hologram P are propagated to the same depth layers and compared).
 * The plan's propagation (chrf_propagate) maps P_phi to
 * V [n_views][n_lambda][n_planes][H][W]; the loss is
 *   mean |V - U|^2 + ssim_weight * (1 - mean SSIM over the real and the
 *   imaginary parts of every (view, wavelength, plane) image),
 * and dphi = Im(G exp(-j phi)) with G the adjoint propagation of dL/dV.
 *   targets   complex [n_views][n_lambda][n_planes][H][W]: U, e.g. chrf_propagate of P
 *   phi       float [n_views][n_lambda][H][W]
 *   loss_out  device float scalar;  dphi  float, same shape as phi
 * Needs a plan created with phase_only = 1.  Overwrites the workspace state a
 * chrf_forward left for chrf_backward.
 */
chrf_status chrf_phase_only_step(chrf_plan* plan, const float* targets, const float* phi, void* workspace,
                                 float* loss_out, float* dphi, void* hip_stream);

/*
 * One Adam step (Kingma and Ba, 2015) on n device floats, in place:
 * m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 * x -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), step t >= 1.
 */
chrf_status chrf_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                           float beta2, float eps, int32_t step, void* hip_stream);

/*
 * One Adan step (Xie et al., adaptive Nesterov momentum; the optimiser of
 * Sec. 5) on n device floats, in place, in the decay-coefficient form:
 *   d = g - g_prev (0 at step 1);  m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) d;
 *   n = b3 n + (1 - b3) (g + b2 d)^2;  g_prev = g;
 *   x = (x - lr (m / c1 + b2 v / c2) / (sqrt(n / c3) + eps)) / (1 + lr weight_decay)
 * with c_i = 1 - b_i^step.  The paper's (0.9, 0.99) are b1 and b3; Adan's
 * default b2 = 0.92 is the gradient-difference moment.  All five state
 * arrays have n floats; m, v and nm start at zero; g_prev is overwritten at
 * step 1.  Errors: CHRF_EINVAL for NULL arrays, step < 1, betas outside
 * [0, 1) or eps <= 0.
 */
chrf_status chrf_adan_step(float* param, const float* grad, float* grad_prev, float* m, float* v, float* nm,
                           int64_t n, float lr, float beta1, float beta2, float beta3, float eps, float weight_decay,
                           int32_t step, void* hip_stream);

/*
 * Densification statistics (the 3DGS strategy the paper adopts): after a
 * chrf_backward on a single-plane or layered plan, for each of the first n
 * Gaussians, add to grad_accum[g] the norm of dL/d mu_2D (pixels) of every
 * view that binned it and to grad_count[g] the number of such views.  Both
 * are device float arrays of n entries, caller-owned, accumulated in place.
 */
chrf_status chrf_densify_stats(chrf_plan* plan, void* workspace, int32_t n, float* grad_accum, float* grad_count,
                               void* hip_stream);

/*
 * Densification (the optimisation algorithm of the Supplementary: prune,
 * clone and split with phase perturbation), all arrays device memory.
 * Input Gaussian i grows if grad_count[i] > 0 and grad_accum[i] >= fl(tau_grad
 * * grad_count[i]); it splits if it grows and its largest log-scale exceeds
 * sigma_split, else it is kept and, if it grows, cloned.  Outputs, in input
 * order: a kept Gaussian (kind 0) followed by its clone (kind 1, phases +
 * phase_sigma zeta[i][0]); or, for a split, two children (kind 2) with means
 * mu + R(q) (exp(s) * xi[i][c]), log-scales s - shrink and phases
 * + phase_sigma zeta[i][c].  Any output with opacity < min_opacity or largest
 * log-scale > sigma_prune is dropped.  Decisions are taken in single
 * precision exactly as written (grow: one rounded product; a child's largest
 * log-scale: fl(max s - shrink)).
 */
typedef struct {
  int32_t n, n_lambda;
  const float* means;       /* [n][3] */
  const float* log_scales;  /* [n][3] */
  const float* quats;       /* [n][4] (w, x, y, z), any norm */
  const float* opacity;     /* [n] activated, for the pruning test only */
  const float* phase;       /* [n][n_lambda] */
  const float* grad_accum;  /* [n], from chrf_densify_stats */
  const float* grad_count;  /* [n] */
  const float* xi;          /* [n][2][3] standard normal draws (split offsets) */
  const float* zeta;        /* [n][2][n_lambda] standard normal draws (phase perturbation) */
  float tau_grad;           /* mean view-space gradient threshold */
  float sigma_split;        /* log of the scale above which a growing Gaussian splits */
  float sigma_prune;        /* log of the scale above which a Gaussian is pruned */
  float min_opacity;        /* opacity below which a Gaussian is pruned */
  float phase_sigma;        /* size of the phase perturbation of new Gaussians */
  float shrink;             /* log-scale decrease of split children (log 1.6) */
} chrf_densify_desc;

/* Scratch bytes chrf_densify needs for n input Gaussians. */
size_t chrf_densify_workspace_bytes(int64_t n);

/*
 * Runs the densification of desc into outputs of `capacity` rows:
 *   src [capacity] int32 (input index of each output), kind [capacity] int32,
 *   means_out [capacity][3], log_scales_out [capacity][3],
 *   phase_out [capacity][n_lambda];
 *   n_out: device int64, the number of outputs (written even when it exceeds
 *   capacity, in which case rows past capacity are not written; capacity
 *   2 n always suffices).
 * scratch: chrf_densify_workspace_bytes(n) bytes of device memory.
 */
chrf_status chrf_densify(const chrf_densify_desc* desc, void* scratch, int64_t capacity, int32_t* src, int32_t* kind,
                         float* means_out, float* log_scales_out, float* phase_out, int64_t* n_out,
                         void* hip_stream);

/*
 * chrf_densify for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, outputs and errors as chrf_densify, without the scratch
 * argument: the scratch comes from a device array that the library holds
 * per GPU (CHRF_NOALLOC_MAX_GAUSSIANS inputs' worth, about 48 MiB, resident
 * from the first use on that GPU until the process ends).  The call itself
 * allocates nothing; chrf_create resolves the array of its device, otherwise
 * the first call on a device does.  The device is that of hip_stream (the
 * current device for the null stream).
 *   CHRF_EINVAL  desc->n > CHRF_NOALLOC_MAX_GAUSSIANS, or as chrf_densify.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from several threads) race and must be
 * ordered by the caller.  Nothing in the array has to start at zero.
 */
#define CHRF_NOALLOC_MAX_GAUSSIANS 4194304
chrf_status chrf_densify_noalloc(const chrf_densify_desc* desc, int64_t capacity, int32_t* src, int32_t* kind,
                                 float* means_out, float* log_scales_out, float* phase_out, int64_t* n_out,
                                 void* hip_stream);

/*
 * Carries a per-Gaussian array [n][row] through a densification: output row j
 * < min(*n_out, capacity) is in[src[j]], or zero when zero_new != 0 and
 * kind[j] != 0 (fresh optimiser state for new Gaussians).  out has
 * capacity rows; rows past *n_out are left untouched.
 */
chrf_status chrf_gather_rows(const float* in, int64_t row, const int32_t* src, const int32_t* kind,
                             const int64_t* n_out, int64_t capacity, int32_t zero_new, float* out,
                             void* hip_stream);

/* Synchronise the stream and report the last forward's pair-list status:
 * CHRF_OK, CHRF_ECAPACITY with *pairs_needed set, or CHRF_EHIP if a wait of
 * the radix sort's look-back gave up (its output is then not valid; the
 * wait is bounded so that no kernel can run forever). */
chrf_status chrf_read_status(chrf_plan* plan, void* workspace, int64_t* pairs_needed, void* hip_stream);

/*
 * Per-kernel timing with HIP events recorded on the launch stream.  While
 * enabled, every launch is bracketed by events; chrf_timing_report
 * synchronises, writes "name count total_ms" lines into buf (NUL-terminated,
 * truncated to size) and clears the records.
 */
chrf_status chrf_timing_enable(chrf_plan* plan, int enable);
chrf_status chrf_timing_report(chrf_plan* plan, char* buf, size_t size);

#ifdef __cplusplus
}
#endif
#endif /* CHRF_H_ */
