// Complex front-to-back compositing per tile (Algorithm 2 with one plane;
// Sec. 4.2) and its reverse-order backward.
//
// One workgroup per (view, tile); one thread per pixel, and every 64-lane
// wave covers an 8x8 pixel block so that a Gaussian touches as few waves as
// possible.  The tile's sorted pair list is walked in batches: each thread
// stages one Gaussian record (centre, conic, opacity, support rectangle and
// the per-wavelength value c exp(j phi)) in LDS, then every pixel consumes the
// whole batch from LDS with broadcast reads.
//
// Forward per pixel:  a = min(alpha_max, o exp(-power)); if the pixel is in
// the support rectangle, power <= k^2/2 and a >= alpha_min:
//   U_l += v_l a T,  T *= 1 - a,  stop after T < T_min.
// Backward per pixel, from its last contributor down:  T_g = T / (1 - a),
//   dL/da = T_g sum_l Re(conj(G_l)(v_l - B_l)),  B_l <- a v_l + (1 - a) B_l,
// and the per-pair gradients (d mu, d conic, d opacity, d v) are summed over
// the wave with DPP row shifts/broadcasts, over the workgroup in LDS, and
// added to the per-(view, Gaussian) accumulators with one atomic per value.
#include "internal.h"

namespace chrf {

constexpr int kBatch = kRasterThreads;

__device__ inline void tile_pixel(int tile_w, int& lx, int& ly) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpr = tile_w >> 3;   // 8x8 blocks per tile row
  lx = (wave % wpr) * 8 + (lane & 7);
  ly = (wave / wpr) * 8 + (lane >> 3);
}

template <int NL>
__global__ __launch_bounds__(kRasterThreads) void k_raster_fwd(RasterArgs a) {
  __shared__ float4 s_g0[kBatch];
  __shared__ float4 s_g1[kBatch];
  __shared__ int4 s_rc[kBatch];
  __shared__ float2 s_v[NL][kBatch];

  const int n_tiles = a.tiles_x * a.tiles_y;
  const int view = blockIdx.x / n_tiles;
  const int tile = blockIdx.x % n_tiles;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  int lx, ly;
  tile_pixel(a.tile_w, lx, ly);
  const int px = tx * a.tile_w + lx, py = ty * a.tile_h + ly;
  const bool inside = px < a.width && py < a.height;
  const float pxf = (float)px + 0.5f, pyf = (float)py + 0.5f;
  const uint2 rg = a.ranges[blockIdx.x];
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;

  float T = 1.0f;
  float2 U[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) U[l] = make_float2(0.f, 0.f);
  uint32_t last = 0;
  bool done = !inside;

  const int tid = threadIdx.x;
  const uint32_t nbatch = blockDim.x;   // tile_w * tile_h <= kBatch
  for (uint32_t start = rg.x; start < rg.y; start += nbatch) {
    if (__syncthreads_count(done) == (int)blockDim.x) break;
    const uint32_t idx = start + tid;
    if (idx < rg.y) {
      const uint32_t rid = a.pair_val[idx];
      s_g0[tid] = a.rec_g0[rid];
      s_g1[tid] = a.rec_g1[rid];
      s_rc[tid] = a.rec_rect[rid];
      const uint32_t g = rid % (uint32_t)a.n_stride;
#pragma unroll
      for (int l = 0; l < NL; ++l) s_v[l][tid] = a.v[(size_t)g * NL + l];
    }
    __syncthreads();
    const int cnt = (int)min(rg.y - start, nbatch);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 g0 = s_g0[j];
        const float4 g1 = s_g1[j];
        const int4 rc = s_rc[j];
        const float dx = pxf - g0.x, dy = pyf - g0.y;
        const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
        const bool in_rect = (unsigned)(px - rc.x) <= (unsigned)rc.y && (unsigned)(py - rc.z) <= (unsigned)rc.w;
        const float aval = fminf(a.alpha_max, g1.y * __expf(-power));
        if (in_rect && power <= half_k2 && aval >= a.alpha_min) {
          const float wgt = aval * T;
#pragma unroll
          for (int l = 0; l < NL; ++l) {
            const float2 v = s_v[l][j];
            U[l].x += v.x * wgt;
            U[l].y += v.y * wgt;
          }
          T *= 1.0f - aval;
          last = start + j + 1;
          if (T < a.t_min) {
            done = true;
            break;
          }
        }
      }
    }
  }
  if (inside) {
    const size_t pix = ((size_t)view * a.height + py) * a.width + px;
    const size_t plane = (size_t)a.height * a.width;
#pragma unroll
    for (int l = 0; l < NL; ++l) a.field[((size_t)view * NL + l) * plane + (size_t)py * a.width + px] = U[l];
    a.t_final[pix] = T;
    a.last[pix] = last;
  }
}

// Sum over the 64 lanes; the result is valid in lane 63.
__device__ inline float wave_sum_to_last(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));  // row_shr:1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));  // row_shr:2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));  // row_shr:4
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));  // row_shr:8
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false)); // row_bcast:15
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false)); // row_bcast:31
  return v;
}

template <int NL>
__global__ __launch_bounds__(kRasterThreads) void k_raster_bwd(RasterArgs a) {
  constexpr int G2 = 6 + 2 * NL;
  __shared__ float4 s_g0[kBatch];
  __shared__ float4 s_g1[kBatch];
  __shared__ int4 s_rc[kBatch];
  __shared__ float2 s_v[NL][kBatch];
  __shared__ uint32_t s_rid[kBatch];
  __shared__ float s_grad[kBatch][G2];
  __shared__ uint32_t s_maxlast;

  const int n_tiles = a.tiles_x * a.tiles_y;
  const int view = blockIdx.x / n_tiles;
  const int tile = blockIdx.x % n_tiles;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  int lx, ly;
  tile_pixel(a.tile_w, lx, ly);
  const int px = tx * a.tile_w + lx, py = ty * a.tile_h + ly;
  const bool inside = px < a.width && py < a.height;
  const float pxf = (float)px + 0.5f, pyf = (float)py + 0.5f;
  const uint2 rg = a.ranges[blockIdx.x];
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;
  const int tid = threadIdx.x, lane = tid & 63;

  float T = 1.0f;
  uint32_t mylast = 0;
  float2 G[NL], Bacc[NL];
  const float scale = a.grad_scale ? *a.grad_scale : 1.0f;
  if (inside) {
    const size_t pix = ((size_t)view * a.height + py) * a.width + px;
    T = a.t_final[pix];
    mylast = a.last[pix];
    const size_t plane = (size_t)a.height * a.width;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const float2 gg = a.grad_field[((size_t)view * NL + l) * plane + (size_t)py * a.width + px];
      G[l] = make_float2(gg.x * scale, gg.y * scale);
    }
  } else {
#pragma unroll
    for (int l = 0; l < NL; ++l) G[l] = make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int l = 0; l < NL; ++l) Bacc[l] = make_float2(0.f, 0.f);
  if (tid == 0) s_maxlast = 0;
  for (int i = tid; i < kBatch * G2; i += blockDim.x) (&s_grad[0][0])[i] = 0.f;
  __syncthreads();
  atomicMax(&s_maxlast, mylast);
  __syncthreads();
  const uint32_t end = s_maxlast;   // one past the last pair any pixel used
  if (end <= rg.x) return;

  for (uint32_t top = end; top > rg.x;) {
    const uint32_t cnt = min(top - rg.x, (uint32_t)blockDim.x);
    // stage pairs top-1, top-2, ... so that s[j] is the j-th pair from the back
    if ((uint32_t)tid < cnt) {
      const uint32_t idx = top - 1 - tid;
      const uint32_t rid = a.pair_val[idx];
      s_rid[tid] = rid;
      s_g0[tid] = a.rec_g0[rid];
      s_g1[tid] = a.rec_g1[rid];
      s_rc[tid] = a.rec_rect[rid];
      const uint32_t g = rid % (uint32_t)a.n_stride;
#pragma unroll
      for (int l = 0; l < NL; ++l) s_v[l][tid] = a.v[(size_t)g * NL + l];
    }
    __syncthreads();
    for (uint32_t j = 0; j < cnt; ++j) {
      const uint32_t pidx = top - 1 - j;   // index in the sorted pair list
      const float4 g0 = s_g0[j];
      const float4 g1 = s_g1[j];
      const int4 rc = s_rc[j];
      const float dx = pxf - g0.x, dy = pyf - g0.y;
      const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
      const bool in_rect = (unsigned)(px - rc.x) <= (unsigned)rc.y && (unsigned)(py - rc.z) <= (unsigned)rc.w;
      const float Gv = __expf(-power);
      const float oG = g1.y * Gv;
      const bool clamped = oG > a.alpha_max;
      const float aval = clamped ? a.alpha_max : oG;
      const bool contrib = inside && pidx < mylast && in_rect && power <= half_k2 && aval >= a.alpha_min;
      float gr[G2];
#pragma unroll
      for (int c = 0; c < G2; ++c) gr[c] = 0.f;
      if (contrib) {
        T = T / (1.0f - aval);
        float dLda = 0.f;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const float2 v = s_v[l][j];
          dLda += G[l].x * (v.x - Bacc[l].x) + G[l].y * (v.y - Bacc[l].y);
          const float aT = aval * T;
          gr[6 + 2 * l] = aT * G[l].x;
          gr[7 + 2 * l] = aT * G[l].y;
          Bacc[l].x = aval * v.x + (1.0f - aval) * Bacc[l].x;
          Bacc[l].y = aval * v.y + (1.0f - aval) * Bacc[l].y;
        }
        dLda *= T;
        if (!clamped) {
          gr[5] = Gv * dLda;
          const float dpow = -aval * dLda;
          gr[2] = 0.5f * dx * dx * dpow;
          gr[3] = dx * dy * dpow;
          gr[4] = 0.5f * dy * dy * dpow;
          gr[0] = -(g0.z * dx + g0.w * dy) * dpow;
          gr[1] = -(g0.w * dx + g1.x * dy) * dpow;
        }
      }
      if (__ballot(contrib) != 0ull) {
#pragma unroll
        for (int c = 0; c < G2; ++c) {
          const float s = wave_sum_to_last(gr[c]);
          if (lane == 63) atomicAdd(&s_grad[j][c], s);
        }
      }
    }
    __syncthreads();
    if ((uint32_t)tid < cnt) {
      float* dst = a.grad2d + (size_t)s_rid[tid] * a.g2stride;
#pragma unroll
      for (int c = 0; c < G2; ++c) {
        const float s = s_grad[tid][c];
        if (s != 0.f) unsafeAtomicAdd(dst + c, s);
        s_grad[tid][c] = 0.f;
      }
    }
    __syncthreads();
    top -= cnt;
  }
}

hipError_t launch_raster_forward(const RasterArgs& a, hipStream_t s) {
  const int blocks = a.n_views * a.tiles_x * a.tiles_y;
  if (blocks == 0) return hipSuccess;
  const int threads = a.tile_w * a.tile_h;
  switch (a.n_lambda) {
    case 1: k_raster_fwd<1><<<blocks, threads, 0, s>>>(a); break;
    case 2: k_raster_fwd<2><<<blocks, threads, 0, s>>>(a); break;
    case 3: k_raster_fwd<3><<<blocks, threads, 0, s>>>(a); break;
    case 4: k_raster_fwd<4><<<blocks, threads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_raster_backward(const RasterArgs& a, hipStream_t s) {
  const int blocks = a.n_views * a.tiles_x * a.tiles_y;
  if (blocks == 0) return hipSuccess;
  const int threads = a.tile_w * a.tile_h;
  switch (a.n_lambda) {
    case 1: k_raster_bwd<1><<<blocks, threads, 0, s>>>(a); break;
    case 2: k_raster_bwd<2><<<blocks, threads, 0, s>>>(a); break;
    case 3: k_raster_bwd<3><<<blocks, threads, 0, s>>>(a); break;
    case 4: k_raster_bwd<4><<<blocks, threads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace chrf
