// Complex front-to-back compositing per tile (Algorithm 2 with one plane;
// Sec. 4.2) and its reverse-order backward.
//
// One workgroup (a single wave) per (view, tile).  The tile's sorted pair list
// is walked in batches: the lanes stage Gaussian records (centre, conic,
// opacity, support rectangle and the per-wavelength value c exp(j phi)) in
// LDS, then every pixel consumes the whole batch with broadcast reads.
//
// Forward per pixel:  a = min(alpha_max, o exp(-power)); if the pixel is in
// the support rectangle, power <= k^2/2 and a >= alpha_min:
//   U_l += v_l a T,  T *= 1 - a,  stop after T < T_min.
// Backward per pixel, from its last contributor down:  T_g = T / (1 - a),
//   dL/da = T_g sum_l Re(conj(G_l)(v_l - B_l)),  B_l <- a v_l + (1 - a) B_l,
// and the per-pair gradients (d mu, d conic, d opacity, d v) are summed over a
// lane's pixels, then over the wave with DPP row shifts/broadcasts, and added
// to the per-(view, Gaussian) accumulators with one atomic per value.
#include "internal.h"

namespace chrf {

// One wave (64 lanes) per tile.  Lane l sits at (l % 8, l / 8) of an 8x8
// block and owns the pixel at that position in each of the tile's
// PPT = tile_w * tile_h / 64 blocks, so per-pair costs that do not depend on
// the pixel (record loads, the gradient reduction over the wave) are shared by
// PPT pixels.  Records are staged in LDS in batches of kBatch pairs.
constexpr int kLanes = 64;
constexpr int kBatch = 128;

struct TileGeom {
  int view, tx, ty;
};

__device__ inline TileGeom tile_of(const RasterArgs& a) {
  const int n_tiles = a.tiles_x * a.tiles_y;
  TileGeom t;
  t.view = blockIdx.x / n_tiles;
  const int tile = blockIdx.x % n_tiles;
  t.tx = tile % a.tiles_x;
  t.ty = tile / a.tiles_x;
  return t;
}

// Origin of the 8x8 block that holds a lane's p-th pixel (the same for all lanes).
__device__ inline void block_of(const RasterArgs& a, const TileGeom& t, int p, int& bx, int& by) {
  const int bpr = a.tile_w >> 3;
  bx = t.tx * a.tile_w + (p % bpr) * 8;
  by = t.ty * a.tile_h + (p / bpr) * 8;
}

// Does the support rectangle rc = (c0, c1 - c0, r0, r1 - r0) reach the 8x8
// block at (bx, by)?  Uniform over the wave, so a miss skips the block's
// pixel work for every lane.
__device__ inline bool rect_hits_block(const int4& rc, int bx, int by) {
  return rc.x <= bx + 7 && bx <= rc.x + rc.y && rc.z <= by + 7 && by <= rc.z + rc.w;
}

template <int PPT>
__device__ inline void pixel_of(const RasterArgs& a, const TileGeom& t, int p, int& px, int& py) {
  const int lane = threadIdx.x;
  const int bpr = a.tile_w >> 3;   // 8x8 blocks per tile row
  px = t.tx * a.tile_w + (p % bpr) * 8 + (lane & 7);
  py = t.ty * a.tile_h + (p / bpr) * 8 + (lane >> 3);
}

template <int NL>
struct Stage {
  float4 g0[kBatch];
  float4 g1[kBatch];
  int4 rc[kBatch];
  float2 v[NL][kBatch];
  uint32_t rid[kBatch];
};

template <int NL>
__device__ inline void stage_records(Stage<NL>& st, const RasterArgs& a, uint32_t first, int cnt, bool reverse) {
  for (int i = threadIdx.x; i < cnt; i += kLanes) {
    const uint32_t idx = reverse ? first - i : first + i;
    const uint32_t rid = a.pair_val[idx];
    st.rid[i] = rid;
    st.g0[i] = a.rec_g0[rid];
    st.g1[i] = a.rec_g1[rid];
    st.rc[i] = a.rec_rect[rid];
    const uint32_t g = rid % (uint32_t)a.n_stride;
#pragma unroll
    for (int l = 0; l < NL; ++l) st.v[l][i] = a.v[(size_t)g * NL + l];
  }
}

template <int NL, int PPT>
__global__ __launch_bounds__(kLanes) void k_raster_fwd(RasterArgs a) {
  __shared__ Stage<NL> st;
  const TileGeom t = tile_of(a);
  int px[PPT], py[PPT], bx[PPT], by[PPT];
  float pxf[PPT], pyf[PPT];
  bool inside[PPT], done[PPT];
  float T[PPT];
  float2 U[PPT][NL];
  uint32_t last[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    pixel_of<PPT>(a, t, p, px[p], py[p]);
    block_of(a, t, p, bx[p], by[p]);
    pxf[p] = (float)px[p] + 0.5f;
    pyf[p] = (float)py[p] + 0.5f;
    inside[p] = px[p] < a.width && py[p] < a.height;
    done[p] = !inside[p];
    T[p] = 1.0f;
    last[p] = 0;
#pragma unroll
    for (int l = 0; l < NL; ++l) U[p][l] = make_float2(0.f, 0.f);
  }
  const uint2 rg = a.ranges[blockIdx.x];
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;
  for (uint32_t start = rg.x; start < rg.y; start += kBatch) {
    bool all_done = true;
#pragma unroll
    for (int p = 0; p < PPT; ++p) all_done = all_done && done[p];
    if (__all(all_done)) break;
    const int cnt = (int)min(rg.y - start, (uint32_t)kBatch);
    __syncthreads();
    stage_records<NL>(st, a, start, cnt, false);
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 g0 = st.g0[j];
      const float4 g1 = st.g1[j];
      const int4 rc = st.rc[j];
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (done[p] || !rect_hits_block(rc, bx[p], by[p])) continue;
        const float dx = pxf[p] - g0.x, dy = pyf[p] - g0.y;
        const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
        const bool in_rect =
            (unsigned)(px[p] - rc.x) <= (unsigned)rc.y && (unsigned)(py[p] - rc.z) <= (unsigned)rc.w;
        const float aval = fminf(a.alpha_max, g1.y * __expf(-power));
        if (in_rect && power <= half_k2 && aval >= a.alpha_min) {
          const float wgt = aval * T[p];
#pragma unroll
          for (int l = 0; l < NL; ++l) {
            const float2 v = st.v[l][j];
            U[p][l].x += v.x * wgt;
            U[p][l].y += v.y * wgt;
          }
          T[p] *= 1.0f - aval;
          last[p] = start + j + 1;
          if (T[p] < a.t_min) done[p] = true;
        }
      }
    }
  }
  const size_t plane = (size_t)a.height * a.width;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (!inside[p]) continue;
    const size_t pix = (size_t)py[p] * a.width + px[p];
#pragma unroll
    for (int l = 0; l < NL; ++l) a.field[((size_t)t.view * NL + l) * plane + pix] = U[p][l];
    a.t_final[(size_t)t.view * plane + pix] = T[p];
    a.last[(size_t)t.view * plane + pix] = last[p];
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

template <int NL, int PPT>
__global__ __launch_bounds__(kLanes) void k_raster_bwd(RasterArgs a) {
  constexpr int G2 = 6 + 2 * NL;
  __shared__ Stage<NL> st;
  __shared__ float s_grad[kBatch][G2];
  const TileGeom t = tile_of(a);
  const int lane = threadIdx.x;
  int px[PPT], py[PPT], bx[PPT], by[PPT];
  float pxf[PPT], pyf[PPT];
  bool inside[PPT];
  float T[PPT];
  uint32_t mylast[PPT];
  float2 G[PPT][NL], Bacc[PPT][NL];
  const float scale = a.grad_scale ? *a.grad_scale : 1.0f;
  const size_t plane = (size_t)a.height * a.width;
  uint32_t tile_last = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    pixel_of<PPT>(a, t, p, px[p], py[p]);
    block_of(a, t, p, bx[p], by[p]);
    pxf[p] = (float)px[p] + 0.5f;
    pyf[p] = (float)py[p] + 0.5f;
    inside[p] = px[p] < a.width && py[p] < a.height;
    T[p] = 1.0f;
    mylast[p] = 0;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      G[p][l] = make_float2(0.f, 0.f);
      Bacc[p][l] = make_float2(0.f, 0.f);
    }
    if (inside[p]) {
      const size_t pix = (size_t)py[p] * a.width + px[p];
      T[p] = a.t_final[(size_t)t.view * plane + pix];
      mylast[p] = a.last[(size_t)t.view * plane + pix];
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const float2 gg = a.grad_field[((size_t)t.view * NL + l) * plane + pix];
        G[p][l] = make_float2(gg.x * scale, gg.y * scale);
      }
    }
    tile_last = max(tile_last, mylast[p]);
  }
  // one past the last pair any pixel of the tile used
  for (int off = 32; off > 0; off >>= 1) tile_last = max(tile_last, (uint32_t)__shfl_xor((int)tile_last, off, 64));
  const uint2 rg = a.ranges[blockIdx.x];
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;
  for (int i = lane; i < kBatch * G2; i += kLanes) (&s_grad[0][0])[i] = 0.f;

  for (uint32_t top = tile_last; top > rg.x;) {
    const int cnt = (int)min(top - rg.x, (uint32_t)kBatch);
    __syncthreads();
    stage_records<NL>(st, a, top - 1, cnt, true);   // st[j] is the j-th pair from the back
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const uint32_t pidx = top - 1 - j;
      const float4 g0 = st.g0[j];
      const float4 g1 = st.g1[j];
      const int4 rc = st.rc[j];
      float gr[G2];
#pragma unroll
      for (int c = 0; c < G2; ++c) gr[c] = 0.f;
      bool any = false;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (!rect_hits_block(rc, bx[p], by[p])) continue;
        const float dx = pxf[p] - g0.x, dy = pyf[p] - g0.y;
        const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
        const bool in_rect =
            (unsigned)(px[p] - rc.x) <= (unsigned)rc.y && (unsigned)(py[p] - rc.z) <= (unsigned)rc.w;
        const float Gv = __expf(-power);
        const float oG = g1.y * Gv;
        const bool clamped = oG > a.alpha_max;
        const float aval = clamped ? a.alpha_max : oG;
        if (pidx < mylast[p] && in_rect && power <= half_k2 && aval >= a.alpha_min) {
          any = true;
          T[p] = T[p] * __builtin_amdgcn_rcpf(1.0f - aval);
          float dLda = 0.f;
          const float aT = aval * T[p];
#pragma unroll
          for (int l = 0; l < NL; ++l) {
            const float2 v = st.v[l][j];
            dLda += G[p][l].x * (v.x - Bacc[p][l].x) + G[p][l].y * (v.y - Bacc[p][l].y);
            gr[6 + 2 * l] += aT * G[p][l].x;
            gr[7 + 2 * l] += aT * G[p][l].y;
            Bacc[p][l].x = aval * v.x + (1.0f - aval) * Bacc[p][l].x;
            Bacc[p][l].y = aval * v.y + (1.0f - aval) * Bacc[p][l].y;
          }
          dLda *= T[p];
          if (!clamped) {
            gr[5] += Gv * dLda;
            const float dpow = -aval * dLda;
            gr[2] += 0.5f * dx * dx * dpow;
            gr[3] += dx * dy * dpow;
            gr[4] += 0.5f * dy * dy * dpow;
            gr[0] -= (g0.z * dx + g0.w * dy) * dpow;
            gr[1] -= (g0.w * dx + g1.x * dy) * dpow;
          }
        }
      }
      if (__ballot(any) != 0ull) {
#pragma unroll
        for (int c = 0; c < G2; ++c) {
          const float sum = wave_sum_to_last(gr[c]);
          if (lane == 63) s_grad[j][c] = sum;
        }
      }
    }
    __syncthreads();
    // lanes take consecutive components of consecutive pairs, so one atomic
    // instruction touches a handful of 64-byte gradient rows, not 64 of them
    for (int t = lane; t < cnt * G2; t += kLanes) {
      const int i = t / G2, c = t - i * G2;
      const float sum = s_grad[i][c];
      if (sum != 0.f) unsafeAtomicAdd(a.grad2d + (size_t)st.rid[i] * a.g2stride + c, sum);
      s_grad[i][c] = 0.f;
    }
    top -= cnt;
  }
}

#define CHRF_RASTER_DISPATCH(KERNEL)                                                          \
  const int blocks = a.n_views * a.tiles_x * a.tiles_y;                                      \
  if (blocks == 0) return hipSuccess;                                                        \
  const int ppt = a.tile_w * a.tile_h / kLanes;                                              \
  if (a.n_lambda < 1 || a.n_lambda > 4 || (ppt != 1 && ppt != 2 && ppt != 4))                 \
    return hipErrorInvalidValue;                                                             \
  switch (a.n_lambda * 8 + ppt) {                                                            \
    case 9: KERNEL<1, 1><<<blocks, kLanes, 0, s>>>(a); break;                                \
    case 10: KERNEL<1, 2><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 12: KERNEL<1, 4><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 17: KERNEL<2, 1><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 18: KERNEL<2, 2><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 20: KERNEL<2, 4><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 25: KERNEL<3, 1><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 26: KERNEL<3, 2><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 28: KERNEL<3, 4><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 33: KERNEL<4, 1><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 34: KERNEL<4, 2><<<blocks, kLanes, 0, s>>>(a); break;                               \
    case 36: KERNEL<4, 4><<<blocks, kLanes, 0, s>>>(a); break;                               \
    default: return hipErrorInvalidValue;                                                    \
  }                                                                                          \
  return hipGetLastError();

hipError_t launch_raster_forward(const RasterArgs& a, hipStream_t s) { CHRF_RASTER_DISPATCH(k_raster_fwd) }

hipError_t launch_raster_backward(const RasterArgs& a, hipStream_t s) { CHRF_RASTER_DISPATCH(k_raster_bwd) }

}  // namespace chrf
