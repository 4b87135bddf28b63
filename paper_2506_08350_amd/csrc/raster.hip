// Complex front-to-back compositing per tile (Algorithm 2 with one plane;
// Sec. 4.2) and its reverse-order backward.
//
// One workgroup per (view, tile), its waves sharing the tile's 8x8 pixel
// blocks.  The tile's sorted pair list is walked in batches: the lanes stage
// Gaussian records (centre, conic, opacity, support rectangle and the
// per-wavelength value c exp(j phi)) in LDS, then every pixel consumes the
// whole batch with broadcast reads.
//
// Forward per pixel:  a = min(alpha_max, o exp(-power)); if the pixel is in
// the support rectangle, power <= k^2/2 and a >= alpha_min:
//   U_l += v_l a T,  T *= 1 - a,  stop after T < T_min.
// Backward per pixel, from its last contributor down:  T_g = T / (1 - a),
//   dL/da = T_g sum_l Re(conj(G_l)(v_l - B_l)),  B_l <- a v_l + (1 - a) B_l.
// B enters only through the real number K = sum_l Re(conj(G_l) B_l), which is
// what a pixel keeps: dL/da = T_g (D - K) with D = sum_l Re(conj(G_l) v_l),
// and K <- K + a (D - K).  The per-pair gradients (d mu, d conic, d opacity, d v) are summed over a
// lane's pixels, then over the wave (32- and 16-lane swaps, then DPP row
// shifts), then over the tile's waves in LDS, and added to the per-(view,
// Gaussian) accumulators with one atomic per value.
#include "raster_common.h"

namespace chrf {

// NW waves per tile, each owning PPT of the tile's 8x8 blocks (NW * PPT =
// tile_w * tile_h / 64); the staged records are shared by the waves.
template <int NL, int PPT, int NW>
__global__ __launch_bounds__(kLanes * NW) void k_raster_fwd(RasterArgs a) {
  __shared__ Stage<NL> st;
  const TileGeom t = tile_of(a);
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kLanes));
  int px[PPT], py[PPT], bx[PPT], by[PPT];
  float pxf[PPT], pyf[PPT];
  bool inside[PPT];
  float T[PPT];
  float2 U[PPT][NL];
  uint32_t last[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int pb = wave * PPT + p;
    block_of(a, t, pb, bx[p], by[p]);
    px[p] = bx[p] + (lane & 7);
    py[p] = by[p] + (lane >> 3);
    pxf[p] = (float)px[p] + 0.5f;
    pyf[p] = (float)py[p] + 0.5f;
    inside[p] = px[p] < a.width && py[p] < a.height;
    T[p] = inside[p] ? 1.0f : -1.0f;   // finished once T < T_min (which is >= 0)
    last[p] = 0;
#pragma unroll
    for (int l = 0; l < NL; ++l) U[p][l] = make_float2(0.f, 0.f);
  }
  const uint2 rg = a.ranges[t.id];
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;
  for (uint32_t start = rg.x; start < rg.y; start += kBatch) {
    bool all_done = true;
#pragma unroll
    for (int p = 0; p < PPT; ++p) all_done = all_done && T[p] < a.t_min;
    // also the barrier before the next batch overwrites the staged records
    if constexpr (NW == 1) {
      if (__all(all_done)) break;
      __syncthreads();
    } else {
      if (!__syncthreads_or(!all_done)) break;
    }
    const int cnt = (int)min(rg.y - start, (uint32_t)kBatch);
    stage_records<NL>(st, a, start, cnt, false);
    __syncthreads();
    uint64_t hits[PPT], todo = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      hits[p] = block_hits(st.g0, st.g1, st.rc, 0, cnt, bx[p], by[p]);
      todo |= hits[p];
    }
    if (__all(all_done)) todo = 0;   // a finished wave only keeps the barriers
    while (todo) {
      const int j = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const float4 g0 = st.g0[j];
      const float4 g1 = st.g1[j];
      const int4 rc = st.rc[j];
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (PPT > 1 && !((hits[p] >> j) & 1u)) continue;
        const float dx = pxf[p] - g0.x, dy = pyf[p] - g0.y;
        const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
        const bool in_rect =
            (unsigned)(px[p] - rc.x) <= (unsigned)rc.y && (unsigned)(py[p] - rc.z) <= (unsigned)rc.w;
        const float aval = fminf(a.alpha_max, g1.y * __expf(-power));
        if (T[p] >= a.t_min && in_rect && power <= half_k2 && aval >= a.alpha_min) {
          const float wgt = aval * T[p];
#pragma unroll
          for (int l = 0; l < NL; ++l) {
            const float2 v = st.v[l][j];
            U[p][l].x += v.x * wgt;
            U[p][l].y += v.y * wgt;
          }
          T[p] *= 1.0f - aval;
          last[p] = start + j + 1;
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

// NW waves per tile as in the forward; the waves' per-pair sums meet in LDS.
template <int NL, int PPT, int NW>
__global__ __launch_bounds__(kLanes * NW) void k_raster_bwd(RasterArgs a) {
  constexpr int G2 = 6 + 2 * NL;
  constexpr int G2P = (G2 + 3) & ~3;   // padded for the row-wise wave reduction
  __shared__ Stage<NL> st;
  __shared__ float s_grad[kBatch][G2];
  __shared__ uint32_t s_last[NW];
  const TileGeom t = tile_of(a);
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kLanes));
  int px[PPT], py[PPT], bx[PPT], by[PPT];
  float pxf[PPT], pyf[PPT];
  bool inside[PPT];
  float T[PPT];
  uint32_t mylast[PPT];
  float2 G[PPT][NL];
  float K[PPT];   // sum over wavelengths of Re(conj(G) B)
  const float scale = a.grad_scale ? *a.grad_scale : 1.0f;
  const size_t plane = (size_t)a.height * a.width;
  uint32_t tile_last = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    block_of(a, t, wave * PPT + p, bx[p], by[p]);
    px[p] = bx[p] + (lane & 7);
    py[p] = by[p] + (lane >> 3);
    pxf[p] = (float)px[p] + 0.5f;
    pyf[p] = (float)py[p] + 0.5f;
    inside[p] = px[p] < a.width && py[p] < a.height;
    T[p] = 1.0f;
    mylast[p] = 0;
    K[p] = 0.f;
#pragma unroll
    for (int l = 0; l < NL; ++l) G[p][l] = make_float2(0.f, 0.f);
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
  // this wave's pixels used no pair at or past it (equal in every lane after the reduction)
  const uint32_t wave_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)tile_last);
  if constexpr (NW > 1) {
    if (lane == 0) s_last[wave] = tile_last;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) tile_last = max(tile_last, s_last[w]);
    tile_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)tile_last);
  }
  const uint2 rg = a.ranges[t.id];
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;
  for (int i = threadIdx.x; i < kBatch * G2; i += kLanes * NW) (&s_grad[0][0])[i] = 0.f;

  for (uint32_t top = tile_last; top > rg.x;) {
    const int cnt = (int)min(top - rg.x, (uint32_t)kBatch);
    __syncthreads();
    stage_records<NL>(st, a, top - 1, cnt, true);   // st[j] is the j-th pair from the back
    __syncthreads();
    // pairs at or past wave_last touch none of this wave's pixels
    const int j0 = top > wave_last ? (int)min(top - wave_last, (uint32_t)cnt) : 0;
    uint64_t hits[PPT], todo = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      hits[p] = block_hits(st.g0, st.g1, st.rc, j0, cnt, bx[p], by[p]);
      todo |= hits[p];
    }
    while (todo) {
      const int j = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const uint32_t pidx = top - 1 - j;
      const float4 g0 = st.g0[j];
      const float4 g1 = st.g1[j];
      const int4 rc = st.rc[j];
      // Branch-free per pixel: a pixel outside the support takes alpha = 0,
      // which leaves its T and B exactly unchanged and adds exact zeros to
      // the alpha- and colour-gradient terms.
      float gr[G2P];   // read only when some pixel of the wave was supported
      if constexpr (PPT > 1)
#pragma unroll
        for (int c = 0; c < G2P; ++c) gr[c] = 0.f;
      bool any = false;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (PPT > 1 && !((hits[p] >> j) & 1u)) continue;
        const float dx = pxf[p] - g0.x, dy = pyf[p] - g0.y;
        const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
        const bool in_rect =
            (unsigned)(px[p] - rc.x) <= (unsigned)rc.y && (unsigned)(py[p] - rc.z) <= (unsigned)rc.w;
        const float Gv = __expf(-power);
        const float oG = g1.y * Gv;
        const bool clamped = oG > a.alpha_max;
        const float aval = clamped ? a.alpha_max : oG;
        const bool sup = pidx < mylast[p] && in_rect && power <= half_k2 && aval >= a.alpha_min;
        if (!__any(sup)) continue;
        any = true;
        const float ae = sup ? aval : 0.f;
        const float Tb = T[p] * __builtin_amdgcn_rcpf(1.0f - ae);
        const float aT = ae * Tb;
        float D = 0.f;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const float2 v = st.v[l][j];
          D += G[p][l].x * v.x + G[p][l].y * v.y;
          const float gx = aT * G[p][l].x, gy = aT * G[p][l].y;
          gr[6 + 2 * l] = PPT == 1 ? gx : gr[6 + 2 * l] + gx;
          gr[7 + 2 * l] = PPT == 1 ? gy : gr[7 + 2 * l] + gy;
        }
        // D - K serves dL/da and the update B <- B + a (v - B), i.e. K <- K + a (D - K)
        const float dLda = D - K[p];
        K[p] += ae * dLda;
        T[p] = Tb;
        // clamped pixels pass no gradient to the opacity or the conic
        const float dl = (sup && !clamped) ? dLda * Tb : 0.f;
        const float dpow = -aval * dl;
        const float g5 = Gv * dl;
        const float g2 = 0.5f * dx * dx * dpow;
        const float g3 = dx * dy * dpow;
        const float g4 = 0.5f * dy * dy * dpow;
        const float g0v = -(g0.z * dx + g0.w * dy) * dpow;
        const float g1v = -(g0.w * dx + g1.x * dy) * dpow;
        gr[0] = PPT == 1 ? g0v : gr[0] + g0v;
        gr[1] = PPT == 1 ? g1v : gr[1] + g1v;
        gr[2] = PPT == 1 ? g2 : gr[2] + g2;
        gr[3] = PPT == 1 ? g3 : gr[3] + g3;
        gr[4] = PPT == 1 ? g4 : gr[4] + g4;
        gr[5] = PPT == 1 ? g5 : gr[5] + g5;
      }
#pragma unroll
      for (int c = G2; c < G2P; ++c) gr[c] = 0.f;
      if (any) {
        wave_sums_by_row<G2P>(gr);
        if ((lane & 15) == 15) {
          const int row = lane >> 4;
#pragma unroll
          for (int k = 0; k < G2P / 4; ++k) {
            const int c = k + row * (G2P / 4);
            if (c < G2) {
              if constexpr (NW == 1)
                s_grad[j][c] = gr[k];
              else   // at most two waves: 0 + x + y rounds the same in either order
                atomicAdd(&s_grad[j][c], gr[k]);
            }
          }
        }
      }
    }
    __syncthreads();
    // lanes take consecutive components of consecutive pairs, so one atomic
    // instruction touches a handful of 64-byte gradient rows, not 64 of them
    for (int t = threadIdx.x; t < cnt * G2; t += kLanes * NW) {
      const int i = t / G2, c = t - i * G2;
      const float sum = s_grad[i][c];
      if (sum != 0.f) {
        if (a.pair_grad)   // deterministic mode: the row of pair top - 1 - i, summed later in a fixed order
          a.pair_grad[(size_t)(top - 1 - i) * a.g2stride + c] = sum;
        else
          unsafeAtomicAdd(a.grad2d + (size_t)st.rid[i] * a.g2stride + c, sum);
      }
      s_grad[i][c] = 0.f;
    }
    top -= cnt;
  }
}

// Waves per tile of the forward: up to kFwdWaves, one or more 8x8 blocks
// each.  One wave per 8x8 block of a 16x16 tile: each wave walks only the
// pairs that reach its block, and the CU overlaps one wave's record loads
// with the others' compositing.
#ifndef CHRF_FWD_WAVES
#define CHRF_FWD_WAVES 4
#endif
constexpr int kFwdWaves = CHRF_FWD_WAVES;

template <int NL, int BPT>
static void launch_fwd_nl(const RasterArgs& a, int blocks, hipStream_t s) {
  constexpr int NW = BPT < kFwdWaves ? BPT : kFwdWaves;
  k_raster_fwd<NL, BPT / NW, NW><<<blocks, kLanes * NW, 0, s>>>(a);
}

// Waves per tile of the backward: two waves of two 8x8 blocks each at 16x16
// tiles, so one per-pair wave reduction serves two pixels per lane while two
// waves still overlap record gathers and atomics.
#ifndef CHRF_BWD_WAVES
#define CHRF_BWD_WAVES 2
#endif
constexpr int kBwdWaves = CHRF_BWD_WAVES;

template <int NL, int BPT>
static void launch_bwd_nl(const RasterArgs& a, int blocks, hipStream_t s) {
  constexpr int NW = BPT < kBwdWaves ? BPT : kBwdWaves;
  static_assert(NW <= 2, "the per-pair LDS sums are reproducible for at most two waves");
  k_raster_bwd<NL, BPT / NW, NW><<<blocks, kLanes * NW, 0, s>>>(a);
}

hipError_t launch_raster_forward(const RasterArgs& a, hipStream_t s) {
  const int blocks = a.n_views * a.tiles_x * a.tiles_y;
  if (blocks == 0) return hipSuccess;
  const int bpt = a.tile_w * a.tile_h / kLanes;   // 8x8 blocks per tile
  if (a.n_lambda < 1 || a.n_lambda > 4 || (bpt != 1 && bpt != 2 && bpt != 4)) return hipErrorInvalidValue;
  switch (a.n_lambda * 8 + bpt) {
    case 9: launch_fwd_nl<1, 1>(a, blocks, s); break;
    case 10: launch_fwd_nl<1, 2>(a, blocks, s); break;
    case 12: launch_fwd_nl<1, 4>(a, blocks, s); break;
    case 17: launch_fwd_nl<2, 1>(a, blocks, s); break;
    case 18: launch_fwd_nl<2, 2>(a, blocks, s); break;
    case 20: launch_fwd_nl<2, 4>(a, blocks, s); break;
    case 25: launch_fwd_nl<3, 1>(a, blocks, s); break;
    case 26: launch_fwd_nl<3, 2>(a, blocks, s); break;
    case 28: launch_fwd_nl<3, 4>(a, blocks, s); break;
    case 33: launch_fwd_nl<4, 1>(a, blocks, s); break;
    case 34: launch_fwd_nl<4, 2>(a, blocks, s); break;
    case 36: launch_fwd_nl<4, 4>(a, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_raster_backward(const RasterArgs& a, hipStream_t s) {
  const int blocks = a.n_views * a.tiles_x * a.tiles_y;
  if (blocks == 0) return hipSuccess;
  const int bpt = a.tile_w * a.tile_h / kLanes;   // 8x8 blocks per tile
  if (a.n_lambda < 1 || a.n_lambda > 4 || (bpt != 1 && bpt != 2 && bpt != 4)) return hipErrorInvalidValue;
  switch (a.n_lambda * 8 + bpt) {
    case 9: launch_bwd_nl<1, 1>(a, blocks, s); break;
    case 10: launch_bwd_nl<1, 2>(a, blocks, s); break;
    case 12: launch_bwd_nl<1, 4>(a, blocks, s); break;
    case 17: launch_bwd_nl<2, 1>(a, blocks, s); break;
    case 18: launch_bwd_nl<2, 2>(a, blocks, s); break;
    case 20: launch_bwd_nl<2, 4>(a, blocks, s); break;
    case 25: launch_bwd_nl<3, 1>(a, blocks, s); break;
    case 26: launch_bwd_nl<3, 2>(a, blocks, s); break;
    case 28: launch_bwd_nl<3, 4>(a, blocks, s); break;
    case 33: launch_bwd_nl<4, 1>(a, blocks, s); break;
    case 34: launch_bwd_nl<4, 2>(a, blocks, s); break;
    case 36: launch_bwd_nl<4, 4>(a, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace chrf
