// The paper's training loss on the propagated intensities (Sec. 4.1):
//   L = mean over views, wavelengths, planes and pixels of
//       (I - T)^2 (1 + M + T^2)                       (three-term recon loss)
//     + w (1 - mean SSIM(I, T))                       (SSIM term, w = 0.005)
// with binary plane masks M.  SSIM uses 11 x 11 Gaussian window averages
// (sigma 1.5) with zero padding, C1 = 0.01^2, C2 = 0.03^2.
//
// Forward, per 32 x 32 output tile of one image: the tile and a 5-pixel halo
// of I and T are staged in LDS, the five window averages (mu_x, mu_y, E[x^2],
// E[y^2], E[xy]) are formed by a horizontal then a vertical 11-tap pass, and
// each pixel yields S and the three partial derivatives of S w.r.t. mu_x,
// E[x^2] and E[xy], which are stored for the backward, plus per-tile sums of
// S and of the reconstruction term.
//
// Backward: the same separable window average of the three stored maps (the
// window is symmetric, so the zero-padded filter is its own adjoint) gives
//   dL/dI = -w / (n_img N) [G*dS/dmu + 2 I G*dS/dE[x^2] + T G*dS/dE[xy]]
//         + 2 (I - T)(1 + M + T^2) / numel.
#include "internal.h"

namespace chrf {

constexpr int kLT = 32;                 // output tile edge
constexpr int kLR = 5;                  // window radius
constexpr int kLE = kLT + 2 * kLR;      // staged edge
constexpr int kLThreads = 256;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct LossGeom {
  int H, W, n_img;
  int per_view;          // images per view (wavelengths x planes)
  int planes;
  int tiles_x, tiles_y;
  float g[2 * kLR + 1];  // normalised 1-D Gaussian taps
};

__device__ inline float ld_or0(const float* img, int H, int W, int r, int c) {
  return (r >= 0 && r < H && c >= 0 && c < W) ? img[(size_t)r * W + c] : 0.f;
}

__global__ __launch_bounds__(kLThreads) void k_loss_fwd(const float* __restrict__ I, const float* __restrict__ T,
                                                        const uint8_t* __restrict__ masks, LossGeom lg,
                                                        float* __restrict__ dmu, float* __restrict__ dexx,
                                                        float* __restrict__ dexy, float* __restrict__ partial) {
  __shared__ float sx[kLE][kLE + 1], sy[kLE][kLE + 1];
  __shared__ float hs[5][kLE][kLT + 1];
  __shared__ float red[2][kLThreads / 64];
  const int img = blockIdx.y;
  const int ty = blockIdx.x / lg.tiles_x, tx = blockIdx.x % lg.tiles_x;
  const int r0 = ty * kLT - kLR, c0 = tx * kLT - kLR;
  const size_t base = (size_t)img * lg.H * lg.W;
  const float* x = I + base;
  const float* y = T + base;
  for (int i = threadIdx.x; i < kLE * kLE; i += kLThreads) {
    const int r = i / kLE, c = i % kLE;
    sx[r][c] = ld_or0(x, lg.H, lg.W, r0 + r, c0 + c);
    sy[r][c] = ld_or0(y, lg.H, lg.W, r0 + r, c0 + c);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kLE * kLT; i += kLThreads) {
    const int r = i / kLT, c = i % kLT;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kLR; ++k) {
      const float u = sx[r][c + k], v = sy[r][c + k], w = lg.g[k];
      a += w * u;
      b += w * v;
      aa += w * u * u;
      bb += w * v * v;
      ab += w * u * v;
    }
    hs[0][r][c] = a;
    hs[1][r][c] = b;
    hs[2][r][c] = aa;
    hs[3][r][c] = bb;
    hs[4][r][c] = ab;
  }
  __syncthreads();
  const uint8_t* mk = masks ? masks + ((size_t)(img / lg.per_view) * lg.planes + img % lg.planes) * lg.H * lg.W
                            : nullptr;
  float s_sum = 0.f, r_sum = 0.f;
  for (int i = threadIdx.x; i < kLT * kLT; i += kLThreads) {
    const int r = i / kLT, c = i % kLT;
    const int gr = ty * kLT + r, gc = tx * kLT + c;
    if (gr >= lg.H || gc >= lg.W) continue;
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k <= 2 * kLR; ++k) {
      const float w = lg.g[k];
#pragma unroll
      for (int q = 0; q < 5; ++q) m[q] += w * hs[q][r + k][c];
    }
    const float mx = m[0], my = m[1];
    const float a1 = 2.f * mx * my + kC1;
    const float a2 = 2.f * (m[4] - mx * my) + kC2;
    const float b1 = mx * mx + my * my + kC1;
    const float b2 = (m[2] - mx * mx) + (m[3] - my * my) + kC2;
    const float inv = 1.0f / (b1 * b2);
    const float S = a1 * a2 * inv;
    const size_t o = base + (size_t)gr * lg.W + gc;
    dmu[o] = (2.f * my * a2 - 2.f * my * a1) * inv - S * (2.f * mx / b1 - 2.f * mx / b2);
    dexx[o] = -S / b2;
    dexy[o] = 2.f * a1 * inv;
    s_sum += S;
    const float xv = sx[r + kLR][c + kLR], yv = sy[r + kLR][c + kLR];
    const float d = xv - yv;
    const float mval = mk ? (float)mk[(size_t)gr * lg.W + gc] : 0.f;
    r_sum += d * d * (1.f + mval + yv * yv);
  }
  for (int off = 32; off > 0; off >>= 1) {
    s_sum += __shfl_xor(s_sum, off, 64);
    r_sum += __shfl_xor(r_sum, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s_sum;
    red[1][threadIdx.x >> 6] = r_sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f, b = 0.f;
    for (int w = 0; w < kLThreads / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    const size_t blk = (size_t)img * gridDim.x + blockIdx.x;
    partial[2 * blk] = a;
    partial[2 * blk + 1] = b;
  }
}

__global__ __launch_bounds__(kLThreads) void k_loss_bwd(const float* __restrict__ I, const float* __restrict__ T,
                                                        const uint8_t* __restrict__ masks, LossGeom lg,
                                                        const float* __restrict__ dmu, const float* __restrict__ dexx,
                                                        const float* __restrict__ dexy, float ssim_coef,
                                                        float recon_coef, const float* __restrict__ grad_scale,
                                                        float* __restrict__ dL_dI) {
  __shared__ float sd[3][kLE][kLE + 1];
  __shared__ float hs[3][kLE][kLT + 1];
  const int img = blockIdx.y;
  const int ty = blockIdx.x / lg.tiles_x, tx = blockIdx.x % lg.tiles_x;
  const int r0 = ty * kLT - kLR, c0 = tx * kLT - kLR;
  const size_t base = (size_t)img * lg.H * lg.W;
  for (int i = threadIdx.x; i < kLE * kLE; i += kLThreads) {
    const int r = i / kLE, c = i % kLE;
    sd[0][r][c] = ld_or0(dmu + base, lg.H, lg.W, r0 + r, c0 + c);
    sd[1][r][c] = ld_or0(dexx + base, lg.H, lg.W, r0 + r, c0 + c);
    sd[2][r][c] = ld_or0(dexy + base, lg.H, lg.W, r0 + r, c0 + c);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kLE * kLT; i += kLThreads) {
    const int r = i / kLT, c = i % kLT;
    float a = 0.f, b = 0.f, e = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kLR; ++k) {
      const float w = lg.g[k];
      a += w * sd[0][r][c + k];
      b += w * sd[1][r][c + k];
      e += w * sd[2][r][c + k];
    }
    hs[0][r][c] = a;
    hs[1][r][c] = b;
    hs[2][r][c] = e;
  }
  __syncthreads();
  const float scale = grad_scale ? *grad_scale : 1.0f;
  const uint8_t* mk = masks ? masks + ((size_t)(img / lg.per_view) * lg.planes + img % lg.planes) * lg.H * lg.W
                            : nullptr;
  for (int i = threadIdx.x; i < kLT * kLT; i += kLThreads) {
    const int r = i / kLT, c = i % kLT;
    const int gr = ty * kLT + r, gc = tx * kLT + c;
    if (gr >= lg.H || gc >= lg.W) continue;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kLR; ++k) {
      const float w = lg.g[k];
      f0 += w * hs[0][r + k][c];
      f1 += w * hs[1][r + k][c];
      f2 += w * hs[2][r + k][c];
    }
    const size_t o = base + (size_t)gr * lg.W + gc;
    const float xv = I[o], yv = T[o];
    const float mval = mk ? (float)mk[(size_t)gr * lg.W + gc] : 0.f;
    const float g_ssim = ssim_coef * (f0 + 2.f * xv * f1 + yv * f2);
    const float g_rec = recon_coef * (xv - yv) * (1.f + mval + yv * yv);
    dL_dI[o] = scale * (g_ssim + g_rec);
  }
}

// loss = recon_sum / numel + w (1 - ssim_sum / (n_img N)); partial holds (S, recon) per tile
__global__ __launch_bounds__(1024) void k_loss_total(const float* __restrict__ partial, int64_t n_tiles,
                                                     double inv_numel, double ssim_w, double inv_img_px,
                                                     float* __restrict__ out) {
  __shared__ double red[2][1024 / 64];
  double s = 0.0, r = 0.0;
  for (int64_t i = threadIdx.x; i < n_tiles; i += blockDim.x) {
    s += partial[2 * i];
    r += partial[2 * i + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    r += __shfl_xor(r, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    *out = (float)(b * inv_numel + ssim_w * (1.0 - a * inv_img_px));
  }
}

static LossGeom loss_geom(int n_img, int per_view, int planes, int H, int W) {
  LossGeom lg{};
  lg.H = H;
  lg.W = W;
  lg.n_img = n_img;
  lg.per_view = per_view;
  lg.planes = planes;
  lg.tiles_x = (W + kLT - 1) / kLT;
  lg.tiles_y = (H + kLT - 1) / kLT;
  double g[2 * kLR + 1], sum = 0.0;
  for (int k = 0; k <= 2 * kLR; ++k) {
    const double d = k - kLR;
    g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k <= 2 * kLR; ++k) lg.g[k] = (float)(g[k] / sum);
  return lg;
}

int64_t loss_partial_elems(int n_img, int H, int W) {
  return (int64_t)2 * n_img * ((W + kLT - 1) / kLT) * ((H + kLT - 1) / kLT);
}

hipError_t launch_paper_loss_forward(const float* I, const float* T, const uint8_t* masks, int n_img, int per_view,
                                     int planes, int H, int W, float ssim_weight, float* dmu, float* dexx,
                                     float* dexy, float* partial, float* loss_out, hipStream_t s) {
  const LossGeom lg = loss_geom(n_img, per_view, planes, H, W);
  const dim3 grid((unsigned)(lg.tiles_x * lg.tiles_y), (unsigned)n_img);
  k_loss_fwd<<<grid, kLThreads, 0, s>>>(I, T, masks, lg, dmu, dexx, dexy, partial);
  const double numel = (double)n_img * H * W;
  k_loss_total<<<1, 1024, 0, s>>>(partial, (int64_t)grid.x * grid.y, 1.0 / numel, (double)ssim_weight,
                                  1.0 / numel, loss_out);
  return hipGetLastError();
}

hipError_t launch_paper_loss_backward(const float* I, const float* T, const uint8_t* masks, int n_img, int per_view,
                                      int planes, int H, int W, float ssim_weight, const float* dmu,
                                      const float* dexx, const float* dexy, const float* grad_scale, float* dL_dI,
                                      hipStream_t s) {
  const LossGeom lg = loss_geom(n_img, per_view, planes, H, W);
  const dim3 grid((unsigned)(lg.tiles_x * lg.tiles_y), (unsigned)n_img);
  const double numel = (double)n_img * H * W;
  k_loss_bwd<<<grid, kLThreads, 0, s>>>(I, T, masks, lg, dmu, dexx, dexy, (float)(-ssim_weight / numel),
                                        (float)(2.0 / numel), grad_scale, dL_dI);
  return hipGetLastError();
}

}  // namespace chrf
