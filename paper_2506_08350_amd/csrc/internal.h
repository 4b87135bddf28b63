// Internal declarations shared by the kernel translation units and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.h"

namespace chrf {

constexpr int kMaxLambda = 4;     // wavelengths handled by the raster kernels
constexpr int kMaxPlanes = 64;
constexpr int kRasterThreads = 256;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per sort block
constexpr int kMaxSortPasses = 5;                       // 8-bit digits of up to 40-bit keys
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// Device copy of a camera: x_cam = R x + t; fx, fy, cx, cy in pixels.
struct Cam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy, z_near;
  float pad_[3];
};

// Per-(view, Gaussian) raster record.
//   g0 = (mu_x, mu_y, A, B), g1 = (C, opacity, -, -) with conic [[A, B], [B, C]]
//   rect = (c0, c1 - c0, r0, r1 - r0): inclusive pixel rectangle of the support
struct ProjArgs {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity;
  const Cam* cams;
  int n;          // Gaussians in this call
  int n_stride;   // record stride per view (plan's maximum)
  int n_views;
  int width, height;
  int tile_w, tile_h, tiles_x, tiles_y;
  float k_sigma;
  float alpha_min;      // support threshold on a (bounds the support ellipse stored in rec_g1.z)
  float4* rec_g0;
  float4* rec_g1;
  int4* rec_rect;
  uint64_t* sort_key;   // (view << 32) | depth bits; invisible -> depth bits 0xffffffff
  uint32_t* sort_val;   // view * n_stride + g
  uint32_t* count;      // tiles covered (0 if culled)
  float* grad2d;        // zeroed when not null
  int grad2d_stride;
  // folded into the same launch: v[g][l] = amp e^{j phase} for g < n (the
  // view-0 threads), and zeroing of two word buffers (status, tile ranges)
  const float* amp;
  const float* phase;
  float2* v;
  int n_lambda;
  uint32_t* clear_a;
  int64_t n_clear_a;
  uint32_t* clear_b;
  int64_t n_clear_b;
};

struct FftDesc {
  int n;
  int nstages;
  int radix[kMaxStages];
  const cpx* tw;       // exp(-2 pi i m / n), m < n
  const cpx* tw_half;  // exp(-2 pi i m / (n / 2)), m < n / 2 (n even; else null)
};

// Transfer-function parameters of one (wavelength, distance) pair.
struct HParam {
  float frac_rev;    // fractional part of z / lambda (carrier phase in revolutions)
  float z;           // metres
  float inv_lam;     // 1 / lambda
  float inv_lam2;    // 1 / lambda^2
  int kx_max, ky_max;          // sampling band limit in bins (mode 2), else large
  long long evan_bound;        // kx^2 pH^2 + ky^2 pW^2 <= bound  <=> f^2 <= 1/lambda^2
  float decay;                 // 2 pi |z|: band mode 0 keeps evanescent bins as exp(-decay sqrt(f^2 - 1/lambda^2))
  float pad_;
};

struct AsmGeom {
  int H, W, pH, pW;
  int n_bl;         // views * wavelengths
  int n_lambda, K;
  int band_mode;    // 0 none (evanescent bins decay), 1 Eq. 7, 2 Eq. 7 + sampling limit
  int evanescent;   // some bin of the padded grid lies beyond 1 / lambda for some wavelength
  float ax, ay;     // 1 / (pW pitch), 1 / (pH pitch)
  float norm;       // 1 / (pH pW)
  const HParam* hp; // [n_lambda][K]
  int mask_free;    // no bin of the padded grid is masked for any wavelength and plane
  int row_plan;     // radix schedule of the tuned row transforms (0 = default)
  int col_plan;     // radix schedule of the tuned column transforms (0 = default)
};

// ---- launchers (each returns hipGetLastError after the launch) ----
hipError_t launch_project(const ProjArgs& a, hipStream_t s);
hipError_t launch_project_backward(const float* means, const float* log_scales, const float* quats,
                                   const float* amp, const float* phase, const Cam* cams, int n, int n_stride,
                                   int n_views, int n_lambda, const uint32_t* count, const float* grad2d,
                                   int g2stride, float* d_means, float* d_log_scales, float* d_quats,
                                   float* d_opacity, float* d_amp, float* d_phase, hipStream_t s);

// exclusive scans; total (if not null) receives the sum
hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* block_tmp, hipStream_t s);
hipError_t launch_scan_u64_from_u32(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* block_tmp,
                                    uint64_t* total, hipStream_t s);
int64_t scan_tmp_elems(int64_t n);

// Stable LSD radix sort.  n_dev (device, may be null) caps the count at run time.
// error: device word set to 1 if a look-back wait of the single-sweep passes gave up
hipError_t radix_sort_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t n_max,
                          const uint64_t* n_dev, int begin_bit, int end_bit, uint32_t* hist, uint32_t* scan_tmp,
                          uint32_t* error, bool* result_in_alt, hipStream_t s);
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t n_max,
                          const uint64_t* n_dev, int begin_bit, int end_bit, uint32_t* hist, uint32_t* scan_tmp,
                          uint32_t* error, bool* result_in_alt, hipStream_t s);
int64_t radix_hist_elems(int64_t n_max);

// Pairs of every depth-sorted (view, Gaussian) entry: per tile row of its
// support rectangle, the tiles its ellipse's column span reaches.
hipError_t launch_count_pairs(const uint32_t* sorted_val, const uint32_t* count, const float4* rec_g0,
                              const float4* rec_g1, const int4* rect, int64_t n, int tile_w, int tile_h,
                              uint32_t* cnt_sorted, hipStream_t s);
hipError_t launch_emit_pairs(const uint32_t* sorted_val, const uint64_t* offsets, const uint32_t* cnt_sorted,
                             const float4* rec_g0, const float4* rec_g1, const int4* rect, int64_t n, int n_stride,
                             int tile_w, int tile_h, int tiles_x, int tile_bits, uint32_t* pair_key,
                             uint32_t* pair_val, int64_t capacity, const uint64_t* total, uint32_t* status,
                             uint32_t* det_rid, hipStream_t s);
// deterministic gradient mode: slot bookkeeping after the pair sort, and the
// fixed-order reduction of per-pair gradient rows into per-(view, Gaussian) rows
hipError_t launch_det_gather(uint32_t* pair_val, const uint32_t* det_rid, uint32_t* inv, const uint64_t* total,
                             int64_t capacity, hipStream_t s);
hipError_t launch_det_reduce(const uint32_t* sorted_val, const uint64_t* offsets, const uint32_t* cnt_sorted,
                             const uint32_t* inv, const float* pair_grad, int64_t n, int g2, int64_t capacity,
                             float* grad2d, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t* pair_key, int tile_bits, int n_tiles, const uint64_t* total,
                              int64_t capacity, uint2* ranges, hipStream_t s);

struct RasterArgs {
  const float4* rec_g0;
  const float4* rec_g1;
  const int4* rec_rect;
  const float2* v;          // [N][n_lambda]
  const uint32_t* pair_val;
  const uint2* ranges;
  const uint32_t* tile_order;   // workgroup -> (view, tile) index, longest lists first; null: identity
  int n_stride, n_lambda;
  int width, height, tile_w, tile_h, tiles_x, tiles_y, n_views;
  float k_sigma, alpha_min, alpha_max, t_min;
  float2* field;            // [B][L][H][W]
  float* t_final;           // [B][H][W]
  uint32_t* last;           // [B][H][W]: index of the last included pair + 1 (0 = none)
  // backward only
  const float2* grad_field; // [B][L][H][W]
  const float* grad_scale;  // device scalar or null
  float* grad2d;            // [B * n_stride][g2stride]
  int g2stride;
  float* pair_grad;         // deterministic mode: [pairs][g2stride] per-pair rows (plain stores), else null
  // multi-layer mode: field, grad_field [B][L][n_layers][H][W], t_final [B][n_layers][H][W]
  const uint8_t* layer_of;  // [n_stride] hard layer of each Gaussian
  int n_layers;
  uint32_t* layer_stop;     // [B][n_layers][H][W]: pair index + 1 that ended the layer, ~0u if none
};
// Order of the (view, tile) work items for the raster launches: descending
// list length in buckets of 1/8 octave (order within a bucket unspecified).
hipError_t launch_tile_order(const uint2* ranges, int n, uint32_t* order, hipStream_t s);
hipError_t launch_raster_forward(const RasterArgs& a, hipStream_t s);
hipError_t launch_raster_backward(const RasterArgs& a, hipStream_t s);

// The paper's training loss (masked reconstruction loss + SSIM term).
int64_t loss_partial_elems(int n_img, int H, int W);
hipError_t launch_paper_loss_forward(const float* I, const float* T, const uint8_t* masks, int n_img, int per_view,
                                     int planes, int H, int W, float ssim_weight, float* dmu, float* dexx,
                                     float* dexy, float* partial, float* loss_out, hipStream_t s);
hipError_t launch_paper_loss_backward(const float* I, const float* T, const uint8_t* masks, int n_img, int per_view,
                                      int planes, int H, int W, float ssim_weight, const float* dmu,
                                      const float* dexx, const float* dexy, const float* grad_scale, float* dL_dI,
                                      hipStream_t s);

// Phase-only conversion and the Adam update.
hipError_t launch_field_loss_forward(const float2* V, const float2* U, int n_img, int H, int W, float ssim_weight,
                                     float* dmaps, float* partial, float* loss_out, hipStream_t s);
hipError_t launch_field_loss_backward(const float2* V, const float2* U, int n_img, int H, int W, float ssim_weight,
                                      const float* dmaps, float2* dL_dV, hipStream_t s);
hipError_t launch_phase_field(const float* phi, int64_t n, float2* out, hipStream_t s);
hipError_t launch_phase_grad(const float2* G, const float* phi, int64_t n, float* dphi, hipStream_t s);
hipError_t launch_adam(float* x, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t s);

// Multi-layer mode (hard plane assignment).
constexpr int kMaxLayers = 4;
// temperature of the straight-through softmax over the layer logits (Sec. 4.1, Eq. 12)
constexpr float kSteTau = 1e-3f;
// layer_of[g]: bits 0-2 the argmax layer, bits 4-7 the layers of nonzero
// straight-through weight softmax(logits / tau) in single precision
hipError_t launch_assign_layers(const float* logits, int n, int n_layers, float tau, uint8_t* layer_of,
                                hipStream_t s);
hipError_t launch_raster_layers_forward(const RasterArgs& a, hipStream_t s);
hipError_t launch_raster_layers_backward(const RasterArgs& a, hipStream_t s);
hipError_t launch_logits_backward(const float* logits, const float* grad2d, int g2stride, int rho_offset,
                                  const uint32_t* count, int n, int n_stride, int n_views, int n_layers, float tau,
                                  float* d_logits, hipStream_t s);

// Angular-spectrum passes (layout: rows of [bl][r] are contiguous complex64)
hipError_t launch_rows_forward(const float2* in, float2* out, const AsmGeom& g, const FftDesc& fr, hipStream_t s);
hipError_t launch_cols_forward(const float2* x1, float2* y, const AsmGeom& g, const FftDesc& fc, int cols_per_block,
                               hipStream_t s);
// inverse row pass with epilogue: u (optional), I, loss partials and the fused adjoint row FFT (when target != null)
hipError_t launch_rows_inverse(float2* y, const AsmGeom& g, const FftDesc& fr, float2* prop_out, float* intensity,
                               const float* target, float* loss_partial, float grad_coef, bool fuse_adjoint,
                               hipStream_t s);
hipError_t launch_rows_adjoint_in(const float2* prop, const float* dL_dI, const float2* dL_dprop, float2* z,
                                  const AsmGeom& g, const FftDesc& fr, hipStream_t s);
hipError_t launch_cols_adjoint(const float2* z, float2* w1, const AsmGeom& g, const FftDesc& fc, int cols_per_block,
                               hipStream_t s);
hipError_t launch_rows_adjoint_out(const float2* w1, const float2* dL_dfield, float2* grad_field, const AsmGeom& g,
                                   const FftDesc& fr, hipStream_t s);
hipError_t launch_reduce_loss(const float* partial, int64_t n, float scale, float* out, hipStream_t s);
hipError_t launch_fill_f32(float* p, float value, int64_t n, hipStream_t s);
hipError_t asm_allow_lds(int bytes);
// tuned passes for padded rows of 3840 and columns of 2160 (asm_tuned.hip)
bool tuned_rows(const AsmGeom& g);
bool tuned_cols(const AsmGeom& g);
int tuned_row_plans(const AsmGeom& g);        // radix schedules of the tuned row transforms
int tuned_col_plans(const AsmGeom& g);        // radix schedules of the tuned column transforms
bool tuned_col_plan_fits(const AsmGeom& g, int C);   // those schedules exist for C columns per workgroup
hipError_t launch_rows_forward_t(const float2* in, float2* out, const AsmGeom& g, const FftDesc& fr, hipStream_t s);
hipError_t launch_rows_inverse_t(float2* y, const AsmGeom& g, const FftDesc& fr, float2* prop_out, float* intensity,
                                 const float* target, float* loss_partial, float grad_coef, bool fuse, hipStream_t s);
hipError_t launch_rows_adjoint_in_t(const float2* prop, const float* dL_dI, const float2* dL_dprop, float2* z,
                                    const AsmGeom& g, const FftDesc& fr, hipStream_t s);
hipError_t launch_rows_adjoint_out_t(const float2* w1, const float2* dL_dfield, float2* grad_field, const AsmGeom& g,
                                     const FftDesc& fr, hipStream_t s);
// C = 2 or 4 columns per workgroup
hipError_t launch_cols_forward_t(const float2* x1, float2* y, const AsmGeom& g, const FftDesc& fc, int C,
                                 hipStream_t s);
hipError_t launch_cols_adjoint_t(const float2* z, float2* w1, const AsmGeom& g, const FftDesc& fc, int C,
                                 hipStream_t s);
size_t col_lds_bytes(int pH, int C);
int fft_max_elems();

// ------------------------------------------------------------ training ---
hipError_t launch_adan(float* x, const float* g, float* g_prev, float* m, float* v, float* nn, int64_t n, float lr,
                       float b1, float b2, float b3, float eps, float weight_decay, int step, hipStream_t s);
hipError_t launch_densify_stats(const float* grad2d, int g2stride, const uint32_t* count, int n, int n_stride,
                                int n_views, float* accum, float* seen, hipStream_t s);

struct DensifyArgs {
  int n, n_lambda;
  const float *means, *log_scales, *quats, *opacity, *phase, *grad_accum, *grad_count, *xi, *zeta;
  float tau_grad, sigma_split, sigma_prune, min_opacity, phase_sigma, shrink;
  int64_t capacity;
  int32_t *src, *kind;
  float *means_out, *log_scales_out, *phase_out;
};
hipError_t launch_densify(const DensifyArgs& a, uint32_t* counts, uint64_t* offsets, uint64_t* scan_tmp,
                          uint64_t* total, hipStream_t s);
hipError_t launch_gather_rows(const float* in, int64_t row, const int32_t* src, const int32_t* kind,
                              const uint64_t* live, int64_t capacity, int zero_new, float* out, hipStream_t s);

}  // namespace chrf
