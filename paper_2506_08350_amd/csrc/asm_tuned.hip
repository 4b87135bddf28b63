// Tuned propagation passes for the padded grid of the 1080 x 1920 workloads
// (rows of 3840 = 16 * 16 * 15, columns of 2160 = 16 * 15 * 9), built on the
// compile-time three-stage transform of fft.h.  Same data flow and layouts as
// the generic passes in asm.hip; the differences are that
//   * every butterfly of every stage fits one thread (no stage loops), so
//     a single in-place LDS buffer suffices and occupancy is higher;
//   * the first stage reads HBM directly into registers and the last stage
//     writes HBM directly, skipping two LDS round trips per transform;
//   * fused transforms hand their registers to the next one without LDS:
//     an inverse row FFT (16,16,15) followed by the adjoint's forward row FFT
//     (15,16,16), and in the column pass the forward spectrum (16,15,9) stays
//     in registers, is multiplied by H_k and fed to the inverse (9,15,16);
//   * a column workgroup covers 4 adjacent columns with 1024 threads.
#include "internal.h"

namespace chrf {

__device__ inline cpx ldc(const float2* p) {
  const float2 v = *p;
  return cpx{v.x, v.y};
}
__device__ inline void stc(float2* p, cpx v) { *p = make_float2(v.x, v.y); }

__device__ inline int sbin(int k, int n) { return 2 * k < n ? k : k - n; }

// Values that do not change across the plane loop would otherwise be hoisted
// out of it (twiddles of every stage, per-element frequency terms) and kept
// live in registers for the whole loop; passing them through an empty asm
// statement makes each iteration recompute them instead.
template <typename T>
__device__ inline T opaque_s(T v) {
  asm volatile("" : "+s"(v));
  return v;
}
__device__ inline int opaque_v(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Plane parameters are read-only during a launch: read through the constant
// address space, a uniform index becomes a scalar load, which neither waits
// on nor is waited on with the vector-memory traffic (output stores, copies).
__device__ inline HParam load_hparam(const HParam* hp, int i) {
  static_assert(sizeof(HParam) % 4 == 0, "read as 32-bit words");
  typedef const __attribute__((address_space(4))) uint32_t* const_words;
  const const_words src = (const_words)(hp + i);
  uint32_t w[sizeof(HParam) / 4];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(HParam) / 4); ++k) w[k] = src[k];
  HParam r;
  __builtin_memcpy(&r, w, sizeof r);
  return r;
}

// Transfer function H_k at the bins of one column.  The column terms are
// computed once; per element the band tests are integer compares, the
// residual phase is formed in revolutions with the hardware square root and
// reciprocal, reduced to [-0.5, 0.5] (exact) and fed to the hardware sine and
// cosine, which take their argument in revolutions.  The 1 / (pH pW)
// normalisation is applied by the callers outside the plane loop.
struct ColFreq {
  long long cterm;   // sx^2 pH^2 of the evanescent bin test
  float fx2;         // fx^2
  bool pass;         // column inside the sampling band limit
};

__device__ inline ColFreq col_freq(const HParam& hp, int kx, const AsmGeom& g) {
  const int sx = sbin(kx, g.pW);
  ColFreq c;
  c.cterm = (long long)(sx * sx) * (long long)(g.pH * g.pH);
  const float fx = (float)sx * g.ax;
  c.fx2 = fx * fx;
  c.pass = g.band_mode < 2 || abs(sx) <= hp.kx_max;
  return c;
}

// The transfer function split into its plane-independent part, computed
// once per bin before the plane loop: q = f^2 / (1/lambda + sqrt(1/lambda^2 -
// f^2)), so that the residual phase of plane z is -z q revolutions; -1 marks a
// bin beyond the evanescent cut.  Per plane only the carrier, one
// multiply-add, the reduction, sine/cosine and the sampling band test remain.
__device__ inline float transfer_q(const HParam& hp, const ColFreq& c, int ky, const AsmGeom& g) {
  const int sy = sbin(ky, g.pH);
  const long long lhs = c.cterm + (long long)(sy * sy) * (long long)(g.pW * g.pW);
  const float fy = (float)sy * g.ay;
  const float f2 = fy * fy + c.fx2;
  const float root = __builtin_amdgcn_sqrtf(fmaxf(hp.inv_lam2 - f2, 0.0f));
  const float q = f2 * __builtin_amdgcn_rcpf(hp.inv_lam + root);
  return lhs <= hp.evan_bound ? q : -1.0f;
}

__device__ inline cpx transfer_from_q(const HParam& hp, bool col_pass, float q, int ky, const AsmGeom& g) {
  const int sy = sbin(ky, g.pH);
  const bool pass = col_pass && q >= 0.0f && (g.band_mode < 2 || abs(sy) <= hp.ky_max);
  float rev = hp.frac_rev - hp.z * q;
  rev -= __builtin_rintf(rev);
  const float cs = __builtin_amdgcn_cosf(rev), sn = __builtin_amdgcn_sinf(rev);
  return pass ? cpx{cs, sn} : cpx{0.f, 0.f};
}

// The same when no bin of the grid is masked (AsmGeom::mask_free): no band
// tests, so the per-plane work per bin is one multiply-add, the range
// reduction and the sine and cosine.
__device__ inline cpx transfer_free(const HParam& hp, float q) {
  float rev = hp.frac_rev - hp.z * q;
  rev -= __builtin_rintf(rev);
  return cpx{__builtin_amdgcn_cosf(rev), __builtin_amdgcn_sinf(rev)};
}

template <int N_, int NT_, int R1_, int R2, int R3_>
struct RowT {
  static constexpr int N = N_, NT = NT_, R1 = R1_, R3 = R3_;
  // 512-thread rows keep 4 waves per SIMD (two workgroups per CU, as their
  // LDS allows): at most 128 VGPRs
  static constexpr int kMinWaves = NT > 256 ? 4 : 1;
  using Fwd = Fft3<N, 1, NT, R1, R2, R3, false>;
  using Inv = Fft3<N, 1, NT, R1, R2, R3, true>;
  using FwdRev = Fft3<N, 1, NT, R3, R2, R1, false>;   // takes Inv's outputs as inputs
  static_assert(Fwd::M1 == 1 && Fwd::M3 == 1 && FwdRev::M1 == 1 && FwdRev::M3 == 1, "one butterfly per thread");
  static constexpr int S1 = N / R1, S3 = N / R3;
};

// HALF: the field is half the padded extent (W = pW / 2 for rows, H = pH / 2
// for columns), so which inputs are zero padding and which outputs are
// cropped is known at compile time and the corresponding butterfly
// arithmetic folds away.
template <class RT, bool HALF>
__global__ __launch_bounds__(RT::NT, RT::kMinWaves) void k_rows_forward_t(const float2* __restrict__ in, float2* __restrict__ out,
                                                        AsmGeom g, FftDesc fr) {
  __shared__ cpx lds[lds_padded_size(RT::N)];
  const size_t row = blockIdx.x;
  const float2* src = in + row * g.W;
  const int j = threadIdx.x;
  cpx v1[1][RT::R1], v3[1][RT::R3];
  if (j < RT::S1) {
#pragma unroll
    for (int r = 0; r < RT::R1; ++r) {
      const int e = j + r * RT::S1;
      const bool live = (HALF && RT::R1 % 2 == 0) ? r < RT::R1 / 2 : e < g.W;
      v1[0][r] = live ? ldc(src + e) : cpx{0.f, 0.f};
    }
  }
  RT::Fwd::run(v1, v3, lds, fr.tw);
  float2* dst = out + row * (size_t)g.pW;
  if (j < RT::S3) {
#pragma unroll
    for (int q = 0; q < RT::R3; ++q) stc(dst + j + q * RT::S3, v3[0][q]);
  }
}

template <class RT, bool HALF>
__global__ __launch_bounds__(RT::NT, RT::kMinWaves) void k_rows_inverse_t(float2* __restrict__ y, AsmGeom g, FftDesc fr,
                                                        float2* __restrict__ prop_out, float* __restrict__ intensity,
                                                        const float* __restrict__ target,
                                                        float* __restrict__ loss_partial, float grad_coef, int fuse) {
  __shared__ cpx lds[lds_padded_size(RT::N)];
  __shared__ float red[RT::NT / 64];
  const size_t row = blockIdx.x;
  float2* yrow = y + row * (size_t)g.pW;
  const int j = threadIdx.x;
  cpx v1[1][RT::R1], v3[1][RT::R3];
  if (j < RT::S1) {
#pragma unroll
    for (int r = 0; r < RT::R1; ++r) v1[0][r] = ldc(yrow + j + r * RT::S1);
  }
  RT::Inv::run(v1, v3, lds, fr.tw);
  // v3[0][q] = u at column j + q * S3 (threads j >= S3 hold no outputs)
  const size_t ob = row * (size_t)g.W;
  float lsum = 0.f;
#pragma unroll
  for (int q = 0; q < RT::R3; ++q) {
    const int e = j + q * RT::S3;
    if (j < RT::S3 && !(HALF && q * RT::S3 >= RT::N / 2) && e < g.W) {
      const cpx u = v3[0][q];
      if (prop_out) stc(prop_out + ob + e, u);
      const float I = u.x * u.x + u.y * u.y;
      if (intensity) intensity[ob + e] = I;
      if (target) {
        const float d = I - target[ob + e];
        lsum += d * d;
        v3[0][q] = u * (2.0f * grad_coef * d);
      }
    } else {
      v3[0][q] = cpx{0.f, 0.f};
    }
  }
  if (target) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = red[0];
#pragma unroll
      for (int w = 1; w < RT::NT / 64; ++w) t += red[w];
      loss_partial[row] = t;
    }
  }
  if (fuse) {
    cpx w3[1][RT::R1];
    RT::FwdRev::run(v3, w3, lds, fr.tw);
    if (j < RT::S1) {
#pragma unroll
      for (int q = 0; q < RT::R1; ++q) stc(yrow + j + q * RT::S1, w3[0][q]);
    }
  }
}

template <class RT, bool HALF>
__global__ __launch_bounds__(RT::NT, RT::kMinWaves) void k_rows_adjoint_in_t(const float2* __restrict__ prop,
                                                           const float* __restrict__ dL_dI,
                                                           const float2* __restrict__ dL_dprop,
                                                           float2* __restrict__ z, AsmGeom g, FftDesc fr) {
  __shared__ cpx lds[lds_padded_size(RT::N)];
  const size_t row = blockIdx.x;
  const size_t ob = row * (size_t)g.W;
  const int j = threadIdx.x;
  cpx v1[1][RT::R1], v3[1][RT::R3];
  if (j < RT::S1) {
#pragma unroll
    for (int r = 0; r < RT::R1; ++r) {
      const int e = j + r * RT::S1;
      cpx G{0.f, 0.f};
      if ((HALF && RT::R1 % 2 == 0) ? r < RT::R1 / 2 : e < g.W) {
        if (dL_dI) G = ldc(prop + ob + e) * (2.0f * dL_dI[ob + e]);
        if (dL_dprop) G = G + ldc(dL_dprop + ob + e);
      }
      v1[0][r] = G;
    }
  }
  RT::Fwd::run(v1, v3, lds, fr.tw);
  float2* zrow = z + row * (size_t)g.pW;
  if (j < RT::S3) {
#pragma unroll
    for (int q = 0; q < RT::R3; ++q) stc(zrow + j + q * RT::S3, v3[0][q]);
  }
}

template <class RT, bool HALF>
__global__ __launch_bounds__(RT::NT, RT::kMinWaves) void k_rows_adjoint_out_t(const float2* __restrict__ w1,
                                                            const float2* __restrict__ dL_dfield,
                                                            float2* __restrict__ grad_field, AsmGeom g, FftDesc fr) {
  __shared__ cpx lds[lds_padded_size(RT::N)];
  const size_t row = blockIdx.x;
  const float2* src = w1 + row * (size_t)g.pW;
  const int j = threadIdx.x;
  cpx v1[1][RT::R1], v3[1][RT::R3];
  if (j < RT::S1) {
#pragma unroll
    for (int r = 0; r < RT::R1; ++r) v1[0][r] = ldc(src + j + r * RT::S1);
  }
  RT::Inv::run(v1, v3, lds, fr.tw);
  const size_t ob = row * (size_t)g.W;
#pragma unroll
  for (int q = 0; q < RT::R3; ++q) {
    const int e = j + q * RT::S3;
    if (j < RT::S3 && !(HALF && q * RT::S3 >= RT::N / 2) && e < g.W) {   // threads j >= S3 hold no outputs
      cpx v = v3[0][q];
      if (dL_dfield) v = v + ldc(dL_dfield + ob + e);
      stc(grad_field + ob + e, v);
    }
  }
}

// ---------------------------------------------------------------- columns ---
// C adjacent columns per workgroup, one butterfly per thread.
//   C = 4: 1024 threads, one workgroup per CU; LDS holds the work buffer, the
//          twiddles and, in the forward pass, the spectrum reused for every
//          plane.
//   C = 2: 512 threads; the spectrum stays in registers (each thread keeps the
//          9 values its forward transform produced, which are the inputs its
//          inverse transforms read) and the twiddles are read through the
//          vector cache, so the LDS holds only the work buffer and two
//          workgroups share a CU.
// R1 R2 R3: radices of the forward column transform in stage order; the
// inverse runs them in reverse order, so that each thread's R3 forward
// outputs are the inputs of its inverse butterfly.  N: column length; NT:
// threads, at least the butterflies of every stage.
template <int C_, int R1_ = 16, int R2_ = 15, int R3_ = 9, int N_ = 2160, int NT_ = 256 * C_>
struct ColT {
  static constexpr int C = C_, R1 = R1_, R2 = R2_, R3 = R3_, N = N_;
  static constexpr int NT = NT_;
  static constexpr int S1 = N / R1, S3 = N / R3;
  // LDS layouts with the fewest bank conflicts for the column strides: one
  // padding slot per 16 values in the forward transform, none in the inverse
  // (which then needs no address arithmetic either)
  static constexpr int kPadFwd = 4, kPadInv = 0;
  static constexpr int kLdsElems = lds_padded_size(N * C, kPadFwd);
  using Fwd = Fft3<N, C, NT, R1, R2, R3, false, kPadFwd>;
  using Inv = Fft3<N, C, NT, R3, R2, R1, true, kPadInv>;
  static_assert(Fwd::M1 == 1 && Fwd::M3 == 1 && Inv::M1 == 1 && Inv::M3 == 1, "one butterfly per thread");
  static_assert(Fwd::B3 == Inv::B1, "forward outputs feed the inverse inputs");
  static constexpr int SPAN = 128 / (8 * C);   // column groups per 128-byte line
  static constexpr bool kRegSpec = C <= 2;      // spectrum in registers, twiddles from memory
  static constexpr bool kLdsTw = !kRegSpec;     // twiddle table in LDS, read per power
  // occupancy hint, in waves per SIMD (bounds the VGPRs: 512 / waves)
  static constexpr int kMinWaves = C == 1 ? 4 : (C == 2 ? 2 : 1);
  // half-height field: input (and kept output) r of a first-stage butterfly
  // is a field row iff r < R1 / 2 when R1 is even; otherwise decided per row
  static constexpr bool kEvenSplit = R1 % 2 == 0;
};

__device__ inline int col_remap(int id, int nblocks, int span) {
  // column groups that share a 128-byte line go to consecutive workgroups of
  // the same XCD (dispatch is round-robin over the 8 XCDs)
  const int per = 8 * span;
  const int full = (nblocks / per) * per;
  if (id >= full) return id;
  const int xcd = id & 7, slot = id >> 3;
  return ((slot / span) * 8 + xcd) * span + slot % span;
}

// The N twiddles are copied to LDS once per workgroup: the stages of every
// plane read them there instead of through the vector caches.
template <int N, int NT>
__device__ inline const cpx* stage_twiddles(cpx* s_tw, const cpx* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += NT) s_tw[i] = tw[i];
  __syncthreads();
  return s_tw;
}

template <class CT, bool HALF>
__global__ __launch_bounds__(CT::NT, CT::kMinWaves) void k_cols_forward_t(const float2* __restrict__ x1,
                                                                          float2* __restrict__ y, AsmGeom g,
                                                                          FftDesc fc) {
  constexpr int C = CT::C, R1 = CT::R1, R3 = CT::R3;
  __shared__ cpx lds[CT::kLdsElems];
  __shared__ cpx spec[CT::kRegSpec ? 1 : CT::N * C];
  __shared__ cpx s_tw[CT::kLdsTw ? CT::N : 1];
  const cpx* twl = CT::kLdsTw ? stage_twiddles<CT::N, CT::NT>(s_tw, fc.tw) : fc.tw;
  cpx sreg[CT::kRegSpec ? R3 : 1];
  const int ngroups = g.pW / C;
  const int gid = col_remap(blockIdx.x, gridDim.x, CT::SPAN);
  const int bl = gid / ngroups;
  const int c0 = (gid % ngroups) * C;
  const int lam = bl % g.n_lambda;
  const int b = threadIdx.x;
  const int s = b % C, j = b / C;
  float qv[R3];   // plane-independent transfer terms of this thread's R3 bins
  {
    cpx v1[1][R1], v3[1][R3];
    if (b < CT::Fwd::B1) {
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int n = j + r * CT::S1;
        const bool live = (HALF && CT::kEvenSplit) ? r < R1 / 2 : n < g.H;
        v1[0][r] = live ? ldc(x1 + ((size_t)bl * g.H + n) * g.pW + c0 + s) : cpx{0.f, 0.f};
      }
    }
    // formed while the column loads are in flight
    if (b < CT::Inv::B1) {
      const HParam hp0 = load_hparam(g.hp, lam * g.K);
      const ColFreq cf = col_freq(hp0, c0 + s, g);
#pragma unroll
      for (int q = 0; q < R3; ++q) qv[q] = transfer_q(hp0, cf, j + q * CT::S3, g);
    }
    CT::Fwd::template run<CT::kLdsTw>(v1, v3, lds, twl);
    if (b < CT::Fwd::B3) {
#pragma unroll
      for (int q = 0; q < R3; ++q) {
        if constexpr (CT::kRegSpec)
          sreg[q] = v3[0][q] * g.norm;
        else
          spec[b + q * CT::Fwd::B3] = v3[0][q] * g.norm;
      }
    }
  }
  // inverse-transform twiddles, the same for every plane: read once, so that
  // the plane loop issues no vector load that would wait on its stores
  const typename CT::Inv::StageTw itw = CT::Inv::stage_twiddles_of(fc.tw, b);
  for (int k = 0; k < g.K; ++k) {
    const HParam hp = load_hparam(g.hp, lam * g.K + k);
    const int jj = opaque_v(j), kx = opaque_v(c0 + s);
    cpx w1[1][R3], w3[1][R1];
    if (b < CT::Inv::B1) {
      if (g.mask_free) {   // uniform
#pragma unroll
        for (int q = 0; q < R3; ++q) {
          const cpx sv = CT::kRegSpec ? sreg[CT::kRegSpec ? q : 0] : spec[b + q * CT::Inv::B1];
          w1[0][q] = cmul(sv, transfer_free(hp, qv[q]));
        }
      } else {
        const bool col_pass = g.band_mode < 2 || abs(sbin(kx, g.pW)) <= hp.kx_max;
#pragma unroll
        for (int q = 0; q < R3; ++q) {
          const cpx sv = CT::kRegSpec ? sreg[CT::kRegSpec ? q : 0] : spec[b + q * CT::Inv::B1];
          w1[0][q] = cmul(sv, transfer_from_q(hp, col_pass, qv[q], jj + q * CT::S3, g));
        }
      }
    }
    if constexpr (CT::kLdsTw)
      CT::Inv::template run<CT::kLdsTw>(w1, w3, lds, twl, opaque_v(b));
    else
      CT::Inv::run_with_twiddles(w1, w3, lds, itw, opaque_v(b));
    if (b < CT::Inv::B3) {
      float2* yk = y + ((size_t)bl * g.K + k) * g.H * g.pW + kx;
#pragma unroll
      for (int q = 0; q < R1; ++q) {
        const int n = jj + q * CT::S1;
        if ((HALF && CT::kEvenSplit) ? q < R1 / 2 : n < g.H) stc(yk + (size_t)n * g.pW, w3[0][q]);
      }
    }
  }
}

// The adjoint reads K input columns, one per plane.  With two columns per
// workgroup and half-height inputs, plane k + 1 is copied from HBM straight
// into an LDS buffer (global_load_lds, 16 bytes = one row of both columns
// per lane) while plane k's transform runs; its stage-1 inputs are read from
// that buffer.  The stage twiddles are read before the copy is started, so
// that only the explicit wait before the next plane waits on it.
typedef __attribute__((address_space(1))) void gmem_void;
typedef __attribute__((address_space(3))) void lds_void;

template <class CT, bool HALF>
__global__ __launch_bounds__(CT::NT, CT::kMinWaves) void k_cols_adjoint_t(const float2* __restrict__ z,
                                                                          float2* __restrict__ w1out, AsmGeom g,
                                                                          FftDesc fc) {
  constexpr int C = CT::C, R1 = CT::R1, R3 = CT::R3;
  constexpr bool kDma = HALF && C == 2;
  constexpr int kLiveRows = CT::N / 2;
  __shared__ cpx lds[CT::kLdsElems];
  __shared__ cpx s_tw[CT::kLdsTw ? CT::N : 1];
  __shared__ cpx s_in[kDma ? kLiveRows * C : 1];   // [row][column]
  const cpx* twl = CT::kLdsTw ? stage_twiddles<CT::N, CT::NT>(s_tw, fc.tw) : fc.tw;
  const int ngroups = g.pW / C;
  const int gid = col_remap(blockIdx.x, gridDim.x, CT::SPAN);
  const int bl = gid / ngroups;
  const int c0 = (gid % ngroups) * C;
  const int lam = bl % g.n_lambda;
  const int b = threadIdx.x;
  const int s = b % C, j = b / C;
  cpx acc[1][R3];
#pragma unroll
  for (int q = 0; q < R3; ++q) acc[0][q] = cpx{0.f, 0.f};
  // plane-independent transfer terms of this thread's R3 bins, kept in LDS
  // (each thread reads back only its own entries) to spare registers
  __shared__ float s_q[R3][CT::NT];
  // wave w copies rows 64 i .. 64 i + 63 for i = w, w + NT / 64, ...
  auto copy_plane = [&](int k) {
    if constexpr (kDma) {
      const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
      const float2* zk = z + ((size_t)bl * g.K + k) * g.H * g.pW + c0;
      for (int i = w; i * 64 < kLiveRows; i += CT::NT / 64) {
        const int row = i * 64 + lane;
        if (row < kLiveRows)
          __builtin_amdgcn_global_load_lds((const gmem_void*)(zk + (size_t)row * g.pW), (lds_void*)&s_in[i * 64 * C], 16,
                                           0, 0);
      }
    }
  };
  // the copies of this wave are complete and every wave has passed here
  auto copies_visible = [] {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
  };
  if constexpr (kDma) copy_plane(0);
  if (b < CT::Fwd::B3) {
    const HParam hp0 = load_hparam(g.hp, lam * g.K);
    const ColFreq cf = col_freq(hp0, c0 + s, g);
#pragma unroll
    for (int q = 0; q < R3; ++q) s_q[q][b] = transfer_q(hp0, cf, j + q * CT::S3, g);
  }
  if constexpr (kDma) copies_visible();   // the terms above were formed while plane 0 arrived
  for (int k = 0; k < g.K; ++k) {
    const float2* zk = z + ((size_t)bl * g.K + k) * g.H * g.pW + c0 + s;
    const int jj = opaque_v(j), kx = opaque_v(c0 + s);
    const HParam hp = load_hparam(g.hp, lam * g.K + k);
    cpx v1[1][R1], v3[1][R3];
    if (b < CT::Fwd::B1) {
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int n = jj + r * CT::S1;
        const bool live = CT::kEvenSplit ? r < R1 / 2 : n < kLiveRows;
        if constexpr (kDma) {
          v1[0][r] = live ? s_in[(live ? n : 0) * C + s] : cpx{0.f, 0.f};
        } else {
          v1[0][r] = ((HALF && CT::kEvenSplit) ? r < R1 / 2 : n < g.H) ? ldc(zk + (size_t)n * g.pW)
                                                                       : cpx{0.f, 0.f};
        }
      }
    }
    // stage 1 has read its inputs once the hook runs: the buffer is free
    auto start_next = [&] {
      if (k + 1 < g.K) copy_plane(k + 1);
    };
    // C = 4 would spill with the table
    CT::Fwd::template run_hooked<CT::kLdsTw && CT::kRegSpec, 1, kDma>(v1, v3, lds, twl, start_next, opaque_v(b));
    if (b < CT::Fwd::B3) {
      if (g.mask_free) {   // uniform
#pragma unroll
        for (int q = 0; q < R3; ++q) acc[0][q] = acc[0][q] + cmulc(v3[0][q], transfer_free(hp, s_q[q][b]));
      } else {
        const bool col_pass = g.band_mode < 2 || abs(sbin(kx, g.pW)) <= hp.kx_max;
#pragma unroll
        for (int q = 0; q < R3; ++q)
          acc[0][q] = acc[0][q] + cmulc(v3[0][q], transfer_from_q(hp, col_pass, s_q[q][b], jj + q * CT::S3, g));
      }
    }
    if constexpr (kDma)
      if (k + 1 < g.K) copies_visible();
  }
#pragma unroll
  for (int q = 0; q < R3; ++q) acc[0][q] = acc[0][q] * g.norm;
  cpx w3[1][R1];
  CT::Inv::template run<CT::kLdsTw>(acc, w3, lds, twl);
  if (b < CT::Inv::B3) {
    float2* dst = w1out + (size_t)bl * g.H * g.pW + c0 + s;
#pragma unroll
    for (int q = 0; q < R1; ++q) {
      const int n = j + q * CT::S1;
      if ((HALF && CT::kEvenSplit) ? q < R1 / 2 : n < g.H) stc(dst + (size_t)n * g.pW, w3[0][q]);
    }
  }
}

// ------------------------------------------------- columns of 2 x 2160 ---
// Columns of pH = 2 NH whose lower half is zero padding (H = NH) as two
// transforms of NH.  With w = exp(-2 pi i / pH), the spectrum's even bins 2m
// are the NH-point transform of x[n] and its odd bins 2m + 1 that of
// x[n] w^n; after the transfer function, the kept rows n < NH of the inverse
// are a[n] + w^-n b[n], a and b the (unnormalised) NH-point inverse
// transforms of the even and of the odd bins.  A workgroup takes P adjacent
// columns, whose 2P halves run as the interleaved sequences of a C = 2P
// transform of NH (sequence s: column s / 2, h = s mod 2: 0 even bins, 1 odd
// bins), so the columns take the layout, schedules and occupancy of the
// tuned NH transforms; the lanes (h = 0, 1) of each column and butterfly
// index j hold a and b at the same rows and exchange them to combine.  w^n,
// n < NH, is staged in LDS once per workgroup.
template <class CT>
__device__ inline void stage_split_twiddles(cpx* s_w, const cpx* __restrict__ tw) {
  for (int i = threadIdx.x; i < CT::N; i += CT::NT) s_w[i] = tw[i];
}

// Rows n = j + q S1 of a (h = 0) and b (h = 1) in w3: the lane of half h
// stores the rows with q = h mod 2, out[n] = a[n] + conj(w^n) b[n] (column
// pointer col).
template <class CT>
__device__ inline void store_split(cpx (&w3)[1][CT::R1], const cpx* s_w, float2* col, int pW, int j, int h) {
#pragma unroll
  for (int q = 0; q < CT::R1; ++q) {
    const cpx mine = w3[0][q];
    const cpx other{__shfl_xor(mine.x, 1, 64), __shfl_xor(mine.y, 1, 64)};
    if ((q & 1) == h) {
      const int n = j + q * CT::S1;
      const cpx a = h ? other : mine, b = h ? mine : other;
      stc(col + (size_t)n * pW, a + cmulc(b, s_w[n]));
    }
  }
}

template <class CT>
__global__ __launch_bounds__(CT::NT, 4) void k_cols_forward_split(const float2* __restrict__ x1,
                                                                  float2* __restrict__ y, AsmGeom g, FftDesc fc) {
  constexpr int C = CT::C, P = C / 2, R1 = CT::R1, R3 = CT::R3;
  static_assert(C == 2 || C == 4, "one or two columns of two halves");
  __shared__ cpx lds[CT::kLdsElems];
  __shared__ cpx s_w[CT::N];
  __shared__ float s_q[R3][CT::NT];   // plane-independent transfer terms (each thread reads its own)
  const int ngroups = g.pW / P;
  const int gid = col_remap(blockIdx.x, gridDim.x, 16 / P);
  const int bl = gid / ngroups;
  const int b = threadIdx.x;
  const int s = b % C, h = s & 1, j = b / C;
  const int col = (gid % ngroups) * P + (s >> 1);
  const int lam = bl % g.n_lambda;
  stage_split_twiddles<CT>(s_w, fc.tw);
  __syncthreads();
  cpx sreg[R3];
  {
    cpx v1[1][R1], v3[1][R3];
    if (b < CT::Fwd::B1) {
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int n = j + r * CT::S1;
        const cpx x = ldc(x1 + ((size_t)bl * g.H + n) * g.pW + col);
        v1[0][r] = h ? cmul(x, s_w[n]) : x;
      }
    }
    if (b < CT::Inv::B1) {
      const HParam hp0 = load_hparam(g.hp, lam * g.K);
      const ColFreq cf = col_freq(hp0, col, g);
#pragma unroll
      for (int q = 0; q < R3; ++q) s_q[q][b] = transfer_q(hp0, cf, 2 * (j + q * CT::S3) + h, g);
    }
    CT::Fwd::template run<false>(v1, v3, lds, fc.tw_half);
    if (b < CT::Fwd::B3) {
#pragma unroll
      for (int q = 0; q < R3; ++q) sreg[q] = v3[0][q] * g.norm;
    }
  }
  const typename CT::Inv::StageTw itw = CT::Inv::stage_twiddles_of(fc.tw_half, b);
  for (int k = 0; k < g.K; ++k) {
    const HParam hp = load_hparam(g.hp, lam * g.K + k);
    const int jj = opaque_v(j), kx = opaque_v(col);
    cpx w1[1][R3], w3[1][R1];
    if (b < CT::Inv::B1) {
      if (g.mask_free) {   // uniform
#pragma unroll
        for (int q = 0; q < R3; ++q) w1[0][q] = cmul(sreg[q], transfer_free(hp, s_q[q][b]));
      } else {
        const bool col_pass = g.band_mode < 2 || abs(sbin(kx, g.pW)) <= hp.kx_max;
#pragma unroll
        for (int q = 0; q < R3; ++q)
          w1[0][q] = cmul(sreg[q], transfer_from_q(hp, col_pass, s_q[q][b], 2 * (jj + q * CT::S3) + h, g));
      }
    }
    CT::Inv::run_with_twiddles(w1, w3, lds, itw, opaque_v(b));
    if (b < CT::Inv::B3)
      store_split<CT>(w3, s_w, y + ((size_t)bl * g.K + k) * g.H * g.pW + kx, g.pW, jj, h);
  }
}

// The adjoint reads K input columns, one per plane: plane k + 1 is copied
// from HBM straight into an LDS buffer (global_load_lds: a lane moves 4
// bytes of one column, or one row of both columns) while plane k's transform
// runs.  The transfer terms are formed per plane (the LDS holds the copy
// instead).
template <class CT>
__global__ __launch_bounds__(CT::NT, 4) void k_cols_adjoint_split(const float2* __restrict__ z,
                                                                  float2* __restrict__ w1out, AsmGeom g,
                                                                  FftDesc fc) {
  constexpr int C = CT::C, P = C / 2, R1 = CT::R1, R3 = CT::R3;
  static_assert(C == 2 || C == 4, "one or two columns of two halves");
  constexpr int kLaneBytes = P == 1 ? 4 : 16;
  constexpr int kUnits = CT::N * P * 8 / kLaneBytes;   // copy units of one plane
  __shared__ cpx lds[CT::kLdsElems];
  __shared__ float s_in[CT::N * P * 2];   // [row][column] of one plane
  __shared__ cpx s_w[CT::N];
  const int ngroups = g.pW / P;
  const int gid = col_remap(blockIdx.x, gridDim.x, 16 / P);
  const int bl = gid / ngroups;
  const int c0 = (gid % ngroups) * P;
  const int b = threadIdx.x;
  const int s = b % C, h = s & 1, j = b / C;
  const int col = c0 + (s >> 1);
  const int lam = bl % g.n_lambda;
  // wave w copies units 64 i .. 64 i + 63 of the plane for i = w, w + NT / 64, ...
  auto copy_plane = [&](int k) {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const float* zk = reinterpret_cast<const float*>(z + ((size_t)bl * g.K + k) * g.H * g.pW + c0);
    for (int i = w; i * 64 < kUnits; i += CT::NT / 64) {
      const int e = i * 64 + lane;
      if (e < kUnits) {
        if constexpr (P == 1)   // float e of the column (row e / 2)
          __builtin_amdgcn_global_load_lds((const gmem_void*)(zk + (size_t)(e >> 1) * 2 * g.pW + (e & 1)),
                                           (lds_void*)&s_in[i * 64], 4, 0, 0);
        else   // row e, both columns
          __builtin_amdgcn_global_load_lds((const gmem_void*)(zk + (size_t)e * 2 * g.pW), (lds_void*)&s_in[i * 64 * 4],
                                           16, 0, 0);
      }
    }
  };
  auto copies_visible = [] {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
  };
  stage_split_twiddles<CT>(s_w, fc.tw);
  copy_plane(0);
  copies_visible();
  cpx acc[1][R3];
#pragma unroll
  for (int q = 0; q < R3; ++q) acc[0][q] = cpx{0.f, 0.f};
  for (int k = 0; k < g.K; ++k) {
    const HParam hp = load_hparam(g.hp, lam * g.K + k);
    const int jj = opaque_v(j), kx = opaque_v(col);
    cpx v1[1][R1], v3[1][R3];
    if (b < CT::Fwd::B1) {
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int n = jj + r * CT::S1;
        const int e = 2 * (n * P + (s >> 1));
        const cpx x{s_in[e], s_in[e + 1]};
        v1[0][r] = h ? cmul(x, s_w[n]) : x;
      }
    }
    // stage 1 has read its inputs once the hook runs: the buffer is free
    auto start_next = [&] {
      if (k + 1 < g.K) copy_plane(k + 1);
    };
    CT::Fwd::template run_hooked<false, 1, true>(v1, v3, lds, fc.tw_half, start_next, opaque_v(b));
    if (b < CT::Fwd::B3) {
      const ColFreq cf = col_freq(hp, kx, g);
      if (g.mask_free) {   // uniform
#pragma unroll
        for (int q = 0; q < R3; ++q)
          acc[0][q] = acc[0][q] + cmulc(v3[0][q], transfer_free(hp, transfer_q(hp, cf, 2 * (jj + q * CT::S3) + h, g)));
      } else {
#pragma unroll
        for (int q = 0; q < R3; ++q) {
          const int ky = 2 * (jj + q * CT::S3) + h;
          acc[0][q] = acc[0][q] + cmulc(v3[0][q], transfer_from_q(hp, cf.pass, transfer_q(hp, cf, ky, g), ky, g));
        }
      }
    }
    if (k + 1 < g.K) copies_visible();
  }
#pragma unroll
  for (int q = 0; q < R3; ++q) acc[0][q] = acc[0][q] * g.norm;
  cpx w3[1][R1];
  CT::Inv::template run<false>(acc, w3, lds, fc.tw_half);
  if (b < CT::Inv::B3) store_split<CT>(w3, s_w, w1out + (size_t)bl * g.H * g.pW + col, g.pW, j, h);
}

// Radix schedules of the tuned transforms (AsmGeom::row_plan, col_plan):
//   rows of 3840 (256 threads):     0: 16 16 15   1: 16 15 16   2: 15 16 16
//   rows of 7680 (512 threads):     0: 16 20 24   1: 16 24 20   2: 24 20 16
//   columns of 2160 (C = 2), and
//   columns of 4320 as two of 2160: 0: 16 15 9    1: 16 9 15    2: 15 16 9    3: 12 12 15
// (forward stage order).  Every schedule keeps one butterfly per thread in
// the first and the last stage.
using Row3840 = RowT<3840, 256, 16, 16, 15>;

bool tuned_rows(const AsmGeom& g) { return g.pW == 3840 || g.pW == 7680; }
// (band mode 0 with evanescent bins present needs the decaying continuation,
// which only the generic passes form)
// (columns of 4320 run as two transforms of 2160, which needs the lower
// half to be zero padding)
bool tuned_cols(const AsmGeom& g) {
  return (g.pH == 2160 || (g.pH == 4320 && 2 * g.H == g.pH)) && g.pW % 128 == 0 &&
         !(g.band_mode == 0 && g.evanescent);
}
int tuned_row_plans(const AsmGeom&) { return 3; }
int tuned_col_plans(const AsmGeom&) { return 4; }
bool tuned_col_plan_fits(const AsmGeom& g, int C) { return g.pH == 4320 ? (C == 1 || C == 2) : C == 2; }

static bool rows_half(const AsmGeom& g) { return 2 * g.W == g.pW; }
static bool cols_half(const AsmGeom& g) { return 2 * g.H == g.pH; }

// Calls f(RT{}) with the row transform type of the plan's radix schedule.
template <class F>
static hipError_t with_row_plan(const AsmGeom& g, F&& f) {
  if (g.pW == 7680) {
    switch (g.row_plan) {
      case 1: f(RowT<7680, 512, 16, 24, 20>{}); break;
      case 2: f(RowT<7680, 512, 24, 20, 16>{}); break;
      default: f(RowT<7680, 512, 16, 20, 24>{}); break;
    }
  } else {
    switch (g.row_plan) {
      case 1: f(RowT<3840, 256, 16, 15, 16>{}); break;
      case 2: f(RowT<3840, 256, 15, 16, 16>{}); break;
      default: f(Row3840{}); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_rows_forward_t(const float2* in, float2* out, const AsmGeom& g, const FftDesc& fr, hipStream_t s) {
  const unsigned grid = (unsigned)(g.n_bl * g.H);
  return with_row_plan(g, [&](auto rt) {
    using RT = decltype(rt);
    if (rows_half(g))
      k_rows_forward_t<RT, true><<<grid, RT::NT, 0, s>>>(in, out, g, fr);
    else
      k_rows_forward_t<RT, false><<<grid, RT::NT, 0, s>>>(in, out, g, fr);
  });
}
hipError_t launch_rows_inverse_t(float2* y, const AsmGeom& g, const FftDesc& fr, float2* prop_out, float* intensity,
                                 const float* target, float* loss_partial, float grad_coef, bool fuse, hipStream_t s) {
  const unsigned grid = (unsigned)(g.n_bl * g.K * g.H);
  return with_row_plan(g, [&](auto rt) {
    using RT = decltype(rt);
    if (rows_half(g))
      k_rows_inverse_t<RT, true><<<grid, RT::NT, 0, s>>>(y, g, fr, prop_out, intensity, target, loss_partial, grad_coef,
                                                      fuse ? 1 : 0);
    else
      k_rows_inverse_t<RT, false><<<grid, RT::NT, 0, s>>>(y, g, fr, prop_out, intensity, target, loss_partial, grad_coef,
                                                       fuse ? 1 : 0);
  });
}
hipError_t launch_rows_adjoint_in_t(const float2* prop, const float* dL_dI, const float2* dL_dprop, float2* z,
                                    const AsmGeom& g, const FftDesc& fr, hipStream_t s) {
  const unsigned grid = (unsigned)(g.n_bl * g.K * g.H);
  return with_row_plan(g, [&](auto rt) {
    using RT = decltype(rt);
    if (rows_half(g))
      k_rows_adjoint_in_t<RT, true><<<grid, RT::NT, 0, s>>>(prop, dL_dI, dL_dprop, z, g, fr);
    else
      k_rows_adjoint_in_t<RT, false><<<grid, RT::NT, 0, s>>>(prop, dL_dI, dL_dprop, z, g, fr);
  });
}
hipError_t launch_rows_adjoint_out_t(const float2* w1, const float2* dL_dfield, float2* grad_field, const AsmGeom& g,
                                     const FftDesc& fr, hipStream_t s) {
  const unsigned grid = (unsigned)(g.n_bl * g.H);
  return with_row_plan(g, [&](auto rt) {
    using RT = decltype(rt);
    if (rows_half(g))
      k_rows_adjoint_out_t<RT, true><<<grid, RT::NT, 0, s>>>(w1, dL_dfield, grad_field, g, fr);
    else
      k_rows_adjoint_out_t<RT, false><<<grid, RT::NT, 0, s>>>(w1, dL_dfield, grad_field, g, fr);
  });
}

// Calls f(CT{}) with the column transform type of (C, the plan's radix
// schedule); at height 2160, schedules other than 0 exist for C = 2 only
// (plan creation checks this).
template <class F>
static hipError_t with_col_plan(const AsmGeom& g, int C, F&& f) {
  if (C == 1) {
    f(ColT<1>{});
  } else if (C == 4) {
    f(ColT<4>{});
  } else {
    switch (g.col_plan) {
      case 1: f(ColT<2, 16, 9, 15>{}); break;
      case 2: f(ColT<2, 15, 16, 9>{}); break;
      case 3: f(ColT<2, 12, 12, 15>{}); break;
      default: f(ColT<2>{}); break;
    }
  }
  return hipGetLastError();
}

// Columns of 4320 as two transforms of 2160 (the 2160 schedules), one (C =
// 2) or two (C = 4) columns per workgroup.
template <int C, class F>
static void split_plans(const AsmGeom& g, F&& f) {
  switch (g.col_plan) {
    case 1: f(ColT<C, 16, 9, 15>{}); break;
    case 2: f(ColT<C, 15, 16, 9>{}); break;
    case 3: f(ColT<C, 12, 12, 15>{}); break;
    default: f(ColT<C>{}); break;
  }
}
template <class F>
static hipError_t with_split_plan(const AsmGeom& g, int P, F&& f) {
  if (P == 2)
    split_plans<4>(g, f);
  else
    split_plans<2>(g, f);
  return hipGetLastError();
}
static bool cols_split(const AsmGeom& g) { return g.pH == 4320; }

hipError_t launch_cols_forward_t(const float2* x1, float2* y, const AsmGeom& g, const FftDesc& fc, int C,
                                 hipStream_t s) {
  if (cols_split(g))
    return with_split_plan(g, C, [&](auto ct) {
      using CT = decltype(ct);
      k_cols_forward_split<CT><<<(unsigned)(g.n_bl * (g.pW / (CT::C / 2))), CT::NT, 0, s>>>(x1, y, g, fc);
    });
  const unsigned grid = (unsigned)(g.n_bl * (g.pW / C));
  return with_col_plan(g, C, [&](auto ct) {
    using CT = decltype(ct);
    if (cols_half(g))
      k_cols_forward_t<CT, true><<<grid, CT::NT, 0, s>>>(x1, y, g, fc);
    else
      k_cols_forward_t<CT, false><<<grid, CT::NT, 0, s>>>(x1, y, g, fc);
  });
}
hipError_t launch_cols_adjoint_t(const float2* z, float2* w1, const AsmGeom& g, const FftDesc& fc, int C,
                                 hipStream_t s) {
  if (cols_split(g))
    return with_split_plan(g, C, [&](auto ct) {
      using CT = decltype(ct);
      k_cols_adjoint_split<CT><<<(unsigned)(g.n_bl * (g.pW / (CT::C / 2))), CT::NT, 0, s>>>(z, w1, g, fc);
    });
  const unsigned grid = (unsigned)(g.n_bl * (g.pW / C));
  return with_col_plan(g, C, [&](auto ct) {
    using CT = decltype(ct);
    if (cols_half(g))
      k_cols_adjoint_t<CT, true><<<grid, CT::NT, 0, s>>>(z, w1, g, fc);
    else
      k_cols_adjoint_t<CT, false><<<grid, CT::NT, 0, s>>>(z, w1, g, fc);
  });
}

}  // namespace chrf
