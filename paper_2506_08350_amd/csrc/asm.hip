// Band-limited angular-spectrum propagation (Eqs. 7, 14, 16) and its adjoint
// as three fused passes over a zero-padded pH x pW grid, per (view, wavelength):
//
//   rows_forward   U rows (W) -> zero-pad to pW -> FFT                 -> X1 [H][pW]
//   cols_forward   X1 columns (H nonzero of pH) -> FFT -> for every plane k:
//                  x H_k / (pH pW) -> inverse FFT -> keep rows < H    -> Y_k [H][pW]
//   rows_inverse   Y_k rows -> inverse FFT -> keep columns < W -> u, |u|^2, MSE
//                  partials; for training, G = 2 u dL/dI is formed in place,
//                  zero-padded and transformed forward again           -> Z_k [H][pW]
//
// The adjoint (Supplementary D: dP/dU through the same propagation) mirrors it:
//   cols_adjoint   sum_k conj(H_k)/(pH pW) x FFT(Z_k columns) -> inverse FFT -> W1
//   rows_adjoint_out  W1 rows -> inverse FFT -> keep columns < W       -> dL/dU
//
// Only H of the pH rows of any column are ever nonzero or kept, so the padded
// half is never stored: the spectrum of a column lives in registers between the
// forward transform and the K inverse ones.  H_k is generated in FFT index
// order (no shifts or rolls) from integer bin tests for the band limits and
// a carrier/residual split of the phase: 2 pi z sqrt(1/lambda^2 - f^2) =
// 2 pi frac(z/lambda) - 2 pi z f^2 / (1/lambda + sqrt(1/lambda^2 - f^2)), the
// carrier taken mod 1 in double precision on the host, so single precision
// only sees the residual.
#include "internal.h"

namespace chrf {

constexpr int kFftThreads = 256;

__device__ inline cpx ld(const float2* p) {
  const float2 v = *p;
  return cpx{v.x, v.y};
}
__device__ inline void st(float2* p, cpx v) { *p = make_float2(v.x, v.y); }

__device__ inline int signed_bin(int k, int n) { return 2 * k < n ? k : k - n; }

// H_k(fx, fy) / (pH pW) at bins (kx, ky); zero outside the band (band modes
// 1 and 2).  Band mode 0 cuts nothing: a bin beyond 1 / lambda keeps the
// decaying continuation exp(-2 pi |z| sqrt(f^2 - 1/lambda^2)) of Eq. 7.
__device__ inline cpx transfer(const HParam& hp, int kx, int ky, const AsmGeom& g) {
  const int sx = signed_bin(kx, g.pW), sy = signed_bin(ky, g.pH);
  if (g.band_mode >= 2 && (abs(sx) > hp.kx_max || abs(sy) > hp.ky_max)) return cpx{0.f, 0.f};
  const long long lhs = (long long)sx * sx * g.pH * g.pH + (long long)sy * sy * g.pW * g.pW;
  const float fx = (float)sx * g.ax, fy = (float)sy * g.ay;
  const float f2 = fx * fx + fy * fy;
  if (lhs > hp.evan_bound) {
    if (g.band_mode != 0) return cpx{0.f, 0.f};
    return cpx{expf(-hp.decay * sqrtf(fmaxf(f2 - hp.inv_lam2, 0.0f))) * g.norm, 0.f};
  }
  const float root = sqrtf(fmaxf(hp.inv_lam2 - f2, 0.0f));
  float rev = hp.frac_rev - hp.z * f2 / (hp.inv_lam + root);
  rev -= rintf(rev);
  float s, c;
  sincospif(2.0f * rev, &s, &c);
  return cpx{c * g.norm, s * g.norm};
}

// Column groups of one (view, wavelength) that share 128-byte lines are given
// to consecutive workgroups of the same XCD (workgroups are dispatched to the
// 8 XCDs round-robin), so that each L2 fetches whole lines once.
__device__ inline int xcd_remap(int id, int nblocks, int span) {
  const int per = 8 * span;
  const int full = (nblocks / per) * per;
  if (id >= full) return id;
  const int xcd = id & 7, slot = id >> 3;
  return ((slot / span) * 8 + xcd) * span + slot % span;
}

// Row passes keep two LDS rows (ping-pong stages): 2 * pW complex values.
__global__ __launch_bounds__(kFftThreads) void k_rows_forward(const float2* __restrict__ in, float2* __restrict__ out,
                                                              AsmGeom g, FftDesc fr) {
  extern __shared__ cpx buf[];
  const size_t row = blockIdx.x;
  const float2* src = in + row * g.W;
  for (int e = threadIdx.x; e < g.pW; e += kFftThreads) buf[e] = e < g.W ? ld(src + e) : cpx{0.f, 0.f};
  __syncthreads();
  const cpx* res = fft_lds<kFftThreads, false>(buf, buf + g.pW, g.pW, 1, 0, fr.radix, fr.nstages, fr.tw);
  float2* dst = out + row * g.pW;
  for (int e = threadIdx.x; e < g.pW; e += kFftThreads) st(dst + e, res[e]);
}

__global__ __launch_bounds__(kFftThreads) void k_rows_inverse(float2* __restrict__ y, AsmGeom g, FftDesc fr,
                                                              float2* __restrict__ prop_out,
                                                              float* __restrict__ intensity,
                                                              const float* __restrict__ target,
                                                              float* __restrict__ loss_partial, float grad_coef,
                                                              int fuse) {
  // the per-wave loss sums live in the dynamic allocation, behind the two rows
  extern __shared__ cpx buf[];
  float* red = reinterpret_cast<float*>(buf + 2 * g.pW);
  const size_t row = blockIdx.x;   // ((bl * K + k) * H + r)
  float2* yrow = y + row * g.pW;
  for (int e = threadIdx.x; e < g.pW; e += kFftThreads) buf[e] = ld(yrow + e);
  __syncthreads();
  cpx* res = fft_lds<kFftThreads, true>(buf, buf + g.pW, g.pW, 1, 0, fr.radix, fr.nstages, fr.tw);
  cpx* other = res == buf ? buf + g.pW : buf;
  float lsum = 0.f;
  const size_t ob = row * g.W;
  for (int e = threadIdx.x; e < g.pW; e += kFftThreads) {
    if (e < g.W) {
      const cpx u = res[e];
      if (prop_out) st(prop_out + ob + e, u);
      const float I = u.x * u.x + u.y * u.y;
      if (intensity) intensity[ob + e] = I;
      if (target) {
        const float d = I - target[ob + e];
        lsum += d * d;
        if (fuse) res[e] = u * (2.0f * grad_coef * d);   // G = 2 u dL/dI, dL/dI = coef * (I - I_gt)
      }
    } else if (fuse) {
      res[e] = cpx{0.f, 0.f};
    }
  }
  if (target) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.f;
      for (int w = 0; w < kFftThreads / 64; ++w) t += red[w];
      loss_partial[row] = t;
    }
  }
  if (fuse) {
    __syncthreads();
    const cpx* r2 = fft_lds<kFftThreads, false>(res, other, g.pW, 1, 0, fr.radix, fr.nstages, fr.tw);
    for (int e = threadIdx.x; e < g.pW; e += kFftThreads) st(yrow + e, r2[e]);
  }
}

__global__ __launch_bounds__(kFftThreads) void k_rows_adjoint_in(const float2* __restrict__ prop,
                                                                 const float* __restrict__ dL_dI,
                                                                 const float2* __restrict__ dL_dprop,
                                                                 float2* __restrict__ z, AsmGeom g, FftDesc fr) {
  extern __shared__ cpx buf[];
  const size_t row = blockIdx.x;
  const size_t ob = row * g.W;
  for (int e = threadIdx.x; e < g.pW; e += kFftThreads) {
    cpx G{0.f, 0.f};
    if (e < g.W) {
      if (dL_dI) G = ld(prop + ob + e) * (2.0f * dL_dI[ob + e]);
      if (dL_dprop) G = G + ld(dL_dprop + ob + e);
    }
    buf[e] = G;
  }
  __syncthreads();
  const cpx* res = fft_lds<kFftThreads, false>(buf, buf + g.pW, g.pW, 1, 0, fr.radix, fr.nstages, fr.tw);
  float2* zrow = z + row * g.pW;
  for (int e = threadIdx.x; e < g.pW; e += kFftThreads) st(zrow + e, res[e]);
}

__global__ __launch_bounds__(kFftThreads) void k_rows_adjoint_out(const float2* __restrict__ w1,
                                                                  const float2* __restrict__ dL_dfield,
                                                                  float2* __restrict__ grad_field, AsmGeom g,
                                                                  FftDesc fr) {
  extern __shared__ cpx buf[];
  const size_t row = blockIdx.x;
  const float2* src = w1 + row * g.pW;
  for (int e = threadIdx.x; e < g.pW; e += kFftThreads) buf[e] = ld(src + e);
  __syncthreads();
  const cpx* res = fft_lds<kFftThreads, true>(buf, buf + g.pW, g.pW, 1, 0, fr.radix, fr.nstages, fr.tw);
  const size_t ob = row * g.W;
  for (int e = threadIdx.x; e < g.W; e += kFftThreads) {
    cpx v = res[e];
    if (dL_dfield) v = v + ld(dL_dfield + ob + e);
    st(grad_field + ob + e, v);
  }
}

template <int EPT>
__global__ __launch_bounds__(kFftThreads) void k_cols_forward(const float2* __restrict__ x1, float2* __restrict__ y,
                                                              AsmGeom g, FftDesc fc, int C, int logC, int ngroups,
                                                              int span) {
  extern __shared__ cpx buf[];
  const int gid = xcd_remap(blockIdx.x, gridDim.x, span);
  const int bl = gid / ngroups;
  const int c0 = (gid % ngroups) * C;
  const int lam = bl % g.n_lambda;
  const int total = g.pH * C;
  const int keep = g.H * C;
  for (int e = threadIdx.x; e < total; e += kFftThreads) {
    const int r = e >> logC, s = e & (C - 1);
    buf[e] = r < g.H ? ld(x1 + ((size_t)bl * g.H + r) * g.pW + c0 + s) : cpx{0.f, 0.f};
  }
  __syncthreads();
  cpx* const buf1 = buf + total;
  const cpx* res = fft_lds<kFftThreads, false>(buf, buf1, g.pH, C, logC, fc.radix, fc.nstages, fc.tw);
  cpx S[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kFftThreads;
    S[i] = e < total ? res[e] : cpx{0.f, 0.f};
  }
  __syncthreads();
  for (int k = 0; k < g.K; ++k) {
    const HParam hp = g.hp[lam * g.K + k];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kFftThreads;
      if (e < total) buf[e] = cmul(S[i], transfer(hp, c0 + (e & (C - 1)), e >> logC, g));
    }
    __syncthreads();
    const cpx* rk = fft_lds<kFftThreads, true>(buf, buf1, g.pH, C, logC, fc.radix, fc.nstages, fc.tw);
    float2* yk = y + ((size_t)bl * g.K + k) * g.H * g.pW;
    for (int e = threadIdx.x; e < keep; e += kFftThreads) st(yk + (size_t)(e >> logC) * g.pW + c0 + (e & (C - 1)), rk[e]);
    __syncthreads();
  }
}

template <int EPT>
__global__ __launch_bounds__(kFftThreads) void k_cols_adjoint(const float2* __restrict__ z, float2* __restrict__ w1,
                                                              AsmGeom g, FftDesc fc, int C, int logC, int ngroups,
                                                              int span) {
  extern __shared__ cpx buf[];
  const int gid = xcd_remap(blockIdx.x, gridDim.x, span);
  const int bl = gid / ngroups;
  const int c0 = (gid % ngroups) * C;
  const int lam = bl % g.n_lambda;
  const int total = g.pH * C;
  const int keep = g.H * C;
  cpx* const buf1 = buf + total;
  cpx A[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) A[i] = cpx{0.f, 0.f};
  for (int k = 0; k < g.K; ++k) {
    const float2* zk = z + ((size_t)bl * g.K + k) * g.H * g.pW;
    for (int e = threadIdx.x; e < total; e += kFftThreads) {
      const int r = e >> logC, s = e & (C - 1);
      buf[e] = r < g.H ? ld(zk + (size_t)r * g.pW + c0 + s) : cpx{0.f, 0.f};
    }
    __syncthreads();
    const cpx* rk = fft_lds<kFftThreads, false>(buf, buf1, g.pH, C, logC, fc.radix, fc.nstages, fc.tw);
    const HParam hp = g.hp[lam * g.K + k];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kFftThreads;
      if (e < total) A[i] = A[i] + cmulc(rk[e], transfer(hp, c0 + (e & (C - 1)), e >> logC, g));
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kFftThreads;
    if (e < total) buf[e] = A[i];
  }
  __syncthreads();
  const cpx* res = fft_lds<kFftThreads, true>(buf, buf1, g.pH, C, logC, fc.radix, fc.nstages, fc.tw);
  for (int e = threadIdx.x; e < keep; e += kFftThreads)
    st(w1 + ((size_t)bl * g.H + (e >> logC)) * g.pW + c0 + (e & (C - 1)), res[e]);
}

__global__ __launch_bounds__(1024) void k_reduce_loss(const float* __restrict__ partial, int64_t n, float scale,
                                                      float* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += (double)partial[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    *out = (float)(t * (double)scale);
  }
}

// ------------------------------------------------------------ dispatch ---
static int ept_for(int elems) {
  const int need = (elems + kFftThreads - 1) / kFftThreads;
  const int tiers[] = {4, 8, 12, 16, 20, 24, 32, 40, 48, 64};
  for (int t : tiers)
    if (need <= t) return t;
  return -1;
}

#define CHRF_EPT_SWITCH(EPTV, CALL)                  \
  switch (EPTV) {                                    \
    case 4: { constexpr int E = 4; CALL; } break;    \
    case 8: { constexpr int E = 8; CALL; } break;    \
    case 12: { constexpr int E = 12; CALL; } break;  \
    case 16: { constexpr int E = 16; CALL; } break;  \
    case 20: { constexpr int E = 20; CALL; } break;  \
    case 24: { constexpr int E = 24; CALL; } break;  \
    case 32: { constexpr int E = 32; CALL; } break;  \
    case 40: { constexpr int E = 40; CALL; } break;  \
    case 48: { constexpr int E = 48; CALL; } break;  \
    case 64: { constexpr int E = 64; CALL; } break;  \
    default: return hipErrorInvalidValue;            \
  }

static size_t row_lds(const AsmGeom& g) { return 2 * sizeof(cpx) * g.pW; }

hipError_t launch_rows_forward(const float2* in, float2* out, const AsmGeom& g, const FftDesc& fr, hipStream_t s) {
  if (tuned_rows(g)) return launch_rows_forward_t(in, out, g, fr, s);
  const unsigned rows = (unsigned)(g.n_bl * g.H);
  k_rows_forward<<<rows, kFftThreads, row_lds(g), s>>>(in, out, g, fr);
  return hipGetLastError();
}

hipError_t launch_rows_inverse(float2* y, const AsmGeom& g, const FftDesc& fr, float2* prop_out, float* intensity,
                               const float* target, float* loss_partial, float grad_coef, bool fuse_adjoint,
                               hipStream_t s) {
  if (tuned_rows(g))
    return launch_rows_inverse_t(y, g, fr, prop_out, intensity, target, loss_partial, grad_coef, fuse_adjoint, s);
  const unsigned rows = (unsigned)(g.n_bl * g.K * g.H);
  k_rows_inverse<<<rows, kFftThreads, row_lds(g) + sizeof(float) * (kFftThreads / 64), s>>>(
      y, g, fr, prop_out, intensity, target, loss_partial, grad_coef, fuse_adjoint ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rows_adjoint_in(const float2* prop, const float* dL_dI, const float2* dL_dprop, float2* z,
                                  const AsmGeom& g, const FftDesc& fr, hipStream_t s) {
  if (tuned_rows(g)) return launch_rows_adjoint_in_t(prop, dL_dI, dL_dprop, z, g, fr, s);
  const unsigned rows = (unsigned)(g.n_bl * g.K * g.H);
  k_rows_adjoint_in<<<rows, kFftThreads, row_lds(g), s>>>(prop, dL_dI, dL_dprop, z, g, fr);
  return hipGetLastError();
}

hipError_t launch_rows_adjoint_out(const float2* w1, const float2* dL_dfield, float2* grad_field, const AsmGeom& g,
                                   const FftDesc& fr, hipStream_t s) {
  if (tuned_rows(g)) return launch_rows_adjoint_out_t(w1, dL_dfield, grad_field, g, fr, s);
  const unsigned rows = (unsigned)(g.n_bl * g.H);
  k_rows_adjoint_out<<<rows, kFftThreads, row_lds(g), s>>>(w1, dL_dfield, grad_field, g, fr);
  return hipGetLastError();
}

static int ilog2(int c) {
  int l = 0;
  while ((1 << l) < c) ++l;
  return l;
}

size_t col_lds_bytes(int pH, int C) { return 2 * sizeof(cpx) * (size_t)pH * C; }

hipError_t launch_cols_forward(const float2* x1, float2* y, const AsmGeom& g, const FftDesc& fc, int C,
                               hipStream_t s) {
  if (tuned_cols(g)) return launch_cols_forward_t(x1, y, g, fc, C, s);
  const int ngroups = g.pW / C;
  const unsigned blocks = (unsigned)(g.n_bl * ngroups);
  const int span = C * 8 >= 128 ? 1 : 128 / (C * 8);
  const int logC = ilog2(C);
  CHRF_EPT_SWITCH(ept_for(g.pH * C), (k_cols_forward<E><<<blocks, kFftThreads, col_lds_bytes(g.pH, C), s>>>(
                                         x1, y, g, fc, C, logC, ngroups, span)));
  return hipGetLastError();
}

hipError_t launch_cols_adjoint(const float2* z, float2* w1, const AsmGeom& g, const FftDesc& fc, int C,
                               hipStream_t s) {
  if (tuned_cols(g)) return launch_cols_adjoint_t(z, w1, g, fc, C, s);
  const int ngroups = g.pW / C;
  const unsigned blocks = (unsigned)(g.n_bl * ngroups);
  const int span = C * 8 >= 128 ? 1 : 128 / (C * 8);
  const int logC = ilog2(C);
  CHRF_EPT_SWITCH(ept_for(g.pH * C), (k_cols_adjoint<E><<<blocks, kFftThreads, col_lds_bytes(g.pH, C), s>>>(
                                         z, w1, g, fc, C, logC, ngroups, span)));
  return hipGetLastError();
}

hipError_t launch_reduce_loss(const float* partial, int64_t n, float scale, float* out, hipStream_t s) {
  k_reduce_loss<<<1, 1024, 0, s>>>(partial, n, scale, out);
  return hipGetLastError();
}

// Allow the column passes to use more than the default dynamic LDS.
hipError_t asm_allow_lds(int bytes) {
  hipError_t e = hipSuccess;
#define CHRF_ATTR(E)                                                                                         \
  if (e == hipSuccess)                                                                                       \
    e = hipFuncSetAttribute((const void*)k_cols_forward<E>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes); \
  if (e == hipSuccess)                                                                                       \
    e = hipFuncSetAttribute((const void*)k_cols_adjoint<E>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  CHRF_ATTR(4) CHRF_ATTR(8) CHRF_ATTR(12) CHRF_ATTR(16) CHRF_ATTR(20) CHRF_ATTR(24) CHRF_ATTR(32) CHRF_ATTR(40)
  CHRF_ATTR(48) CHRF_ATTR(64)
#undef CHRF_ATTR
  const void* rows[] = {(const void*)k_rows_forward, (const void*)k_rows_inverse, (const void*)k_rows_adjoint_in,
                        (const void*)k_rows_adjoint_out};
  for (const void* f : rows)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

// Largest supported elements-per-thread: C * pH and pW must not exceed it times the block size.
int fft_max_elems() { return 64 * kFftThreads; }

}  // namespace chrf
