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
constexpr int kLThreads = 512;
constexpr int kLB = 4;                  // outputs per item of the horizontal pass (register blocking)
constexpr int kLBV = 2;                 // output rows per thread of the vertical pass
static_assert(kLE * (kLT / kLB) <= kLThreads, "the horizontal pass takes one round");
static_assert(kLThreads == kLT * (kLT / kLBV), "one vertical-pass block of kLBV rows per thread");
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct LossGeom {
  int H, W, n_img;
  int per_view;          // images per view (wavelengths x planes)
  int planes;
  int tiles_x, tiles_y;
  int chan;              // 1: float images; 2: real and imaginary parts of complex images
  int recon;             // 1: the (1 + M + T^2) weighting of the reconstruction loss; 0: plain squares
  float g[2 * kLR + 1];  // normalised 1-D Gaussian taps
};

// Image i of the launch: element (r, c) sits at base(i) + (r W + c) chan.
__device__ inline size_t img_base(const LossGeom& lg, int i) {
  return ((size_t)(i / lg.chan) * lg.H * lg.W) * lg.chan + (size_t)(i % lg.chan);
}

// Staged element e = it * kLThreads + threadIdx.x of the (kLE x kLE) window
// whose top-left element is (r0, c0): its offset in the image, or -1 where it
// lies outside the window's element count or the image (zero padding).
constexpr int kLStageIters = (kLE * kLE + kLThreads - 1) / kLThreads;
__device__ inline long long stage_offset(int it, int r0, int c0, int H, int W, int chan) {
  const int e = it * kLThreads + (int)threadIdx.x;
  const int r = r0 + e / kLE, c = c0 + e % kLE;
  const bool in = e < kLE * kLE && r >= 0 && r < H && c >= 0 && c < W;
  return in ? ((long long)r * W + c) * chan : -1;
}

// Loads of every staged element of one image, all issued before any is
// used: each reads a valid address (the image's first element stands in for
// the padding) and the padding is zeroed afterwards.
__device__ inline void stage_load(const float* __restrict__ img, const long long (&off)[kLStageIters],
                                  float (&v)[kLStageIters]) {
#pragma unroll
  for (int it = 0; it < kLStageIters; ++it) v[it] = img[off[it] < 0 ? 0 : off[it]];
#pragma unroll
  for (int it = 0; it < kLStageIters; ++it) v[it] = off[it] < 0 ? 0.f : v[it];
}

__device__ inline void stage_store(float (*dst)[kLE + 1], const float (&v)[kLStageIters]) {
#pragma unroll
  for (int it = 0; it < kLStageIters; ++it) {
    const int e = it * kLThreads + (int)threadIdx.x;
    if (e < kLE * kLE) dst[e / kLE][e % kLE] = v[it];
  }
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
  const size_t base = img_base(lg, img);
  {
    long long off[kLStageIters];
#pragma unroll
    for (int it = 0; it < kLStageIters; ++it) off[it] = stage_offset(it, r0, c0, lg.H, lg.W, lg.chan);
    float vx[kLStageIters], vy[kLStageIters];
    stage_load(I + base, off, vx);
    stage_load(T + base, off, vy);
    stage_store(sx, vx);
    stage_store(sy, vy);
  }
  __syncthreads();
  // horizontal pass: item (row r, 4-column group) reads 14 staged values of
  // each image once for its 4 outputs of the five products
  for (int i = threadIdx.x; i < kLE * (kLT / kLB); i += kLThreads) {
    const int r = i / (kLT / kLB), cb = (i % (kLT / kLB)) * kLB;
    float acc[kLB][5] = {};
#pragma unroll
    for (int k = 0; k < kLB + 2 * kLR; ++k) {
      const float u = sx[r][cb + k], v = sy[r][cb + k];
      const float uu = u * u, vv = v * v, uv = u * v;
#pragma unroll
      for (int o = 0; o < kLB; ++o) {
        const int tap = k - o;
        if (tap < 0 || tap > 2 * kLR) continue;
        const float w = lg.g[tap];
        acc[o][0] += w * u;
        acc[o][1] += w * v;
        acc[o][2] += w * uu;
        acc[o][3] += w * vv;
        acc[o][4] += w * uv;
      }
    }
#pragma unroll
    for (int o = 0; o < kLB; ++o)
#pragma unroll
      for (int q = 0; q < 5; ++q) hs[q][r][cb + o] = acc[o][q];
  }
  __syncthreads();
  const uint8_t* mk = masks ? masks + ((size_t)(img / lg.per_view) * lg.planes + img % lg.planes) * lg.H * lg.W
                            : nullptr;
  float s_sum = 0.f, r_sum = 0.f;
  // vertical pass: thread (column c, row group) forms the window averages of
  // kLBV consecutive output rows from kLBV + 10 staged rows
  {
    const int c = threadIdx.x % kLT, r0o = (threadIdx.x / kLT) * kLBV;
    float mo[kLBV];   // plane-mask values of this thread's outputs, loaded during the pass
#pragma unroll
    for (int o = 0; o < kLBV; ++o) {
      const int gr = ty * kLT + r0o + o, gc = tx * kLT + c;
      mo[o] = mk ? (float)mk[(gr < lg.H && gc < lg.W) ? (size_t)gr * lg.W + gc : 0] : 0.f;
    }
    float m[kLBV][5] = {};
#pragma unroll
    for (int k = 0; k < kLBV + 2 * kLR; ++k) {
      float h[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) h[q] = hs[q][r0o + k][c];
#pragma unroll
      for (int o = 0; o < kLBV; ++o) {
        const int tap = k - o;
        if (tap < 0 || tap > 2 * kLR) continue;
        const float w = lg.g[tap];
#pragma unroll
        for (int q = 0; q < 5; ++q) m[o][q] += w * h[q];
      }
    }
#pragma unroll
    for (int o = 0; o < kLBV; ++o) {
      const int r = r0o + o;
      const int gr = ty * kLT + r, gc = tx * kLT + c;
      if (gr >= lg.H || gc >= lg.W) continue;
      const float mx = m[o][0], my = m[o][1];
      const float a1 = 2.f * mx * my + kC1;
      const float a2 = 2.f * (m[o][4] - mx * my) + kC2;
      const float b1 = mx * mx + my * my + kC1;
      const float b2 = (m[o][2] - mx * mx) + (m[o][3] - my * my) + kC2;
      // one division: 1/b1 = b2 inv, 1/b2 = b1 inv
      const float inv = 1.0f / (b1 * b2);
      const float S = a1 * a2 * inv;
      const size_t oi = (size_t)img * lg.H * lg.W + (size_t)gr * lg.W + gc;   // maps are dense per image
      dmu[oi] = (2.f * my * a2 - 2.f * my * a1) * inv - S * 2.f * mx * (b2 - b1) * inv;
      dexx[oi] = -S * b1 * inv;
      dexy[oi] = 2.f * a1 * inv;
      s_sum += S;
      const float xv = sx[r + kLR][c + kLR], yv = sy[r + kLR][c + kLR];
      const float d = xv - yv;
      const float mval = mo[o];
      r_sum += lg.recon ? d * d * (1.f + mval + yv * yv) : d * d;
    }
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
  const size_t mbase = (size_t)img * lg.H * lg.W;   // derivative maps: dense per image
  const size_t base = img_base(lg, img);
  {
    long long off[kLStageIters];
#pragma unroll
    for (int it = 0; it < kLStageIters; ++it) off[it] = stage_offset(it, r0, c0, lg.H, lg.W, 1);
    float v0[kLStageIters], v1[kLStageIters], v2[kLStageIters];
    stage_load(dmu + mbase, off, v0);
    stage_load(dexx + mbase, off, v1);
    stage_load(dexy + mbase, off, v2);
    stage_store(sd[0], v0);
    stage_store(sd[1], v1);
    stage_store(sd[2], v2);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kLE * (kLT / kLB); i += kLThreads) {
    const int r = i / (kLT / kLB), cb = (i % (kLT / kLB)) * kLB;
    float acc[kLB][3] = {};
#pragma unroll
    for (int k = 0; k < kLB + 2 * kLR; ++k) {
      float h[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) h[q] = sd[q][r][cb + k];
#pragma unroll
      for (int o = 0; o < kLB; ++o) {
        const int tap = k - o;
        if (tap < 0 || tap > 2 * kLR) continue;
        const float w = lg.g[tap];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[o][q] += w * h[q];
      }
    }
#pragma unroll
    for (int o = 0; o < kLB; ++o)
#pragma unroll
      for (int q = 0; q < 3; ++q) hs[q][r][cb + o] = acc[o][q];
  }
  __syncthreads();
  const float scale = grad_scale ? *grad_scale : 1.0f;
  const uint8_t* mk = masks ? masks + ((size_t)(img / lg.per_view) * lg.planes + img % lg.planes) * lg.H * lg.W
                            : nullptr;
  const int c = threadIdx.x % kLT, r0o = (threadIdx.x / kLT) * kLBV;
  // this thread's outputs' own values, loaded while the vertical pass runs
  float xo[kLBV], yo[kLBV], mo[kLBV];
#pragma unroll
  for (int o = 0; o < kLBV; ++o) {
    const int gr = ty * kLT + r0o + o, gc = tx * kLT + c;
    const bool in = gr < lg.H && gc < lg.W;
    const size_t px = in ? (size_t)gr * lg.W + gc : 0;
    xo[o] = I[base + px * lg.chan];
    yo[o] = T[base + px * lg.chan];
    mo[o] = mk ? (float)mk[px] : 0.f;
  }
  float f[kLBV][3] = {};
#pragma unroll
  for (int k = 0; k < kLBV + 2 * kLR; ++k) {
    float h[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) h[q] = hs[q][r0o + k][c];
#pragma unroll
    for (int o = 0; o < kLBV; ++o) {
      const int tap = k - o;
      if (tap < 0 || tap > 2 * kLR) continue;
      const float w = lg.g[tap];
#pragma unroll
      for (int q = 0; q < 3; ++q) f[o][q] += w * h[q];
    }
  }
#pragma unroll
  for (int o = 0; o < kLBV; ++o) {
    const int gr = ty * kLT + r0o + o, gc = tx * kLT + c;
    if (gr >= lg.H || gc >= lg.W) continue;
    const size_t oi = base + ((size_t)gr * lg.W + gc) * lg.chan;
    const float xv = xo[o], yv = yo[o], mval = mo[o];
    const float g_ssim = ssim_coef * (f[o][0] + 2.f * xv * f[o][1] + yv * f[o][2]);
    const float g_rec = recon_coef * (xv - yv) * (lg.recon ? 1.f + mval + yv * yv : 1.f);
    dL_dI[oi] = scale * (g_ssim + g_rec);
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

static LossGeom loss_geom(int n_img, int per_view, int planes, int H, int W, int chan = 1, int recon = 1) {
  LossGeom lg{};
  lg.H = H;
  lg.W = W;
  lg.n_img = n_img;
  lg.per_view = per_view;
  lg.planes = planes;
  lg.chan = chan;
  lg.recon = recon;
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

// exp(j phi) and the phase gradient Im(G exp(-j phi)) of the phase-only hologram
__global__ void k_phase_field(const float* __restrict__ phi, int64_t n, float2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float sn, cs;
  sincosf(phi[i], &sn, &cs);
  out[i] = make_float2(cs, sn);
}

__global__ void k_phase_grad(const float2* __restrict__ G, const float* __restrict__ phi, int64_t n,
                             float* __restrict__ dphi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float sn, cs;
  sincosf(phi[i], &sn, &cs);
  const float2 g = G[i];
  dphi[i] = g.y * cs - g.x * sn;
}

hipError_t launch_phase_field(const float* phi, int64_t n, float2* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_phase_field<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(phi, n, out);
  return hipGetLastError();
}

hipError_t launch_phase_grad(const float2* G, const float* phi, int64_t n, float* dphi, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_phase_grad<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(G, phi, n, dphi);
  return hipGetLastError();
}

// Adam update (Kingma and Ba, 2015) with bias correction, step t >= 1.
__global__ void k_adam(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  x[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

hipError_t launch_adam(float* x, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, t)));
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
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

// Phase-only conversion: mean |V - U|^2 over complex elements plus
// w (1 - mean SSIM) over the real and the imaginary parts of every image.
hipError_t launch_field_loss_forward(const float2* V, const float2* U, int n_img, int H, int W, float ssim_weight,
                                     float* dmaps, float* partial, float* loss_out, hipStream_t s) {
  const LossGeom lg = loss_geom(2 * n_img, 1, 1, H, W, 2, 0);
  const size_t map = (size_t)2 * n_img * H * W;
  const dim3 grid((unsigned)(lg.tiles_x * lg.tiles_y), (unsigned)(2 * n_img));
  k_loss_fwd<<<grid, kLThreads, 0, s>>>(reinterpret_cast<const float*>(V), reinterpret_cast<const float*>(U),
                                        nullptr, lg, dmaps, dmaps + map, dmaps + 2 * map, partial);
  const double numel = (double)n_img * H * W;
  k_loss_total<<<1, 1024, 0, s>>>(partial, (int64_t)grid.x * grid.y, 1.0 / numel, (double)ssim_weight,
                                  1.0 / (2.0 * numel), loss_out);
  return hipGetLastError();
}

hipError_t launch_field_loss_backward(const float2* V, const float2* U, int n_img, int H, int W, float ssim_weight,
                                      const float* dmaps, float2* dL_dV, hipStream_t s) {
  const LossGeom lg = loss_geom(2 * n_img, 1, 1, H, W, 2, 0);
  const size_t map = (size_t)2 * n_img * H * W;
  const dim3 grid((unsigned)(lg.tiles_x * lg.tiles_y), (unsigned)(2 * n_img));
  const double numel = (double)n_img * H * W;
  k_loss_bwd<<<grid, kLThreads, 0, s>>>(reinterpret_cast<const float*>(V), reinterpret_cast<const float*>(U),
                                        nullptr, lg, dmaps, dmaps + map, dmaps + 2 * map,
                                        (float)(-ssim_weight / (2.0 * numel)), (float)(2.0 / numel), nullptr,
                                        reinterpret_cast<float*>(dL_dV));
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
