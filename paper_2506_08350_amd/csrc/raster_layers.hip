// Multi-layer complex compositing with hard plane assignment (Sec. 4.1,
// Eqs. 12-13; per-layer transmittance of Supplementary D) and its backward,
// including the straight-through gradient of the layer logits.
//
// Each Gaussian belongs to the layer of its largest logit (ties: lowest
// index).  A pixel walks its tile's pair list once, front to back; a Gaussian
// adds to and attenuates only its own layer:
//   U_q += v a T_q,  T_q *= 1 - a,  layer q stops after T_q < T_min.
// The walk ends when every layer has stopped.
//
// Backward, in reverse from where the walk ended.  For every layer q that had
// not stopped before the pair, with T_q the transmittance of layer q in front
// of the Gaussian and B_q the field of layer q behind it,
//   s_q = T_q sum_l Re(conj(G_ql) (v_l - B_ql)),   dL/drho_q = a s_q,
// which for the Gaussian's own layer is also dL/da; there T_q is recovered as
// T_q / (1 - a) and B_q <- a v + (1 - a) B_q.  B_q enters only through the
// real number K_q = sum_l Re(conj(G_ql) B_ql), so that is what a pixel keeps:
// s_q = T_q (D_q - K_q) with D_q = sum_l Re(conj(G_ql) v_l), and the update
// of B_q becomes K_q <- K_q + a (D_q - K_q).  The per-pair gradient vector
// (d mu, d conic, d opacity, d v, d rho) is reduced over the wave and added
// to the per-(view, Gaussian) accumulators; k_logits_backward then applies
// the straight-through weights softmax(logits / tau).
//
// One workgroup per tile with one wave per 8x8 block of the tile and one pixel
// per lane, so the per-layer state (T, B, G per wavelength) stays in
// registers; the waves share the LDS staging of the tile's records, and in
// the backward each wave's reduced gradient of a pair is added to the
// workgroup's LDS row of that pair before one global atomic per value.
#include <type_traits>

#include "raster_common.h"

namespace chrf {

// Layer byte of each Gaussian: bits 0-2 its hard layer (argmax of the
// logits, ties to the lowest), bits 4-7 the layers whose straight-through
// weight softmax(logits / tau)_q is nonzero in single precision.  The
// logits gradient is dL/drho_q times that weight, so the backward need not
// form dL/drho_q for a layer outside the mask: its product is exactly zero.
__device__ inline uint32_t ste_live_layers(const float* r, int nlay, float inv_tau) {
  float mx = r[0] * inv_tau;
  for (int q = 1; q < nlay; ++q) mx = fmaxf(mx, r[q] * inv_tau);
  uint32_t live = 0;
  for (int q = 0; q < nlay; ++q)
    if (expf(r[q] * inv_tau - mx) != 0.0f) live |= 1u << q;
  return live;
}

__global__ void k_assign_layers(const float* __restrict__ logits, int n, int nlay, float inv_tau,
                                uint8_t* __restrict__ layer_of) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float* r = logits + (size_t)g * nlay;
  int best = 0;
  float bv = r[0];
  for (int q = 1; q < nlay; ++q)
    if (r[q] > bv) {
      bv = r[q];
      best = q;
    }
  layer_of[g] = (uint8_t)(best | (ste_live_layers(r, nlay, inv_tau) << 4));
}

// Calls f(std::integral_constant<int, lay>()) for lay in [Q, N): the
// layer becomes a compile-time constant inside f.
template <int Q, int N, class F>
__device__ inline void with_layer(int lay, F&& f) {
  if constexpr (Q < N) {
    if (lay == Q)
      f(std::integral_constant<int, Q>());
    else
      with_layer<Q + 1, N>(lay, f);
  }
}

template <int NL>
struct StageL {
  Stage<NL> s;
  int lay[kBatch];
};

template <int NL>
__device__ inline void stage_records_l(StageL<NL>& st, const RasterArgs& a, uint32_t first, int cnt, bool reverse) {
  stage_records<NL>(st.s, a, first, cnt, reverse);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const uint32_t idx = reverse ? first - i : first + i;
    const uint32_t g = a.pair_val[idx] % (uint32_t)a.n_stride;
    st.lay[i] = a.layer_of[g];
  }
}

// PPT pixels per lane (one in each of the wave's PPT 8x8 blocks) share the
// pair's record reads and scalar bookkeeping.  One pixel per lane runs at
// eight waves per SIMD (a 64-VGPR budget, met without spills) and is the
// default: two pixels per lane need 114 VGPRs (four waves) and the walk,
// bound by latency, then takes longer (1080p, four layers: 0.65 against
// 0.52 ms).
template <int NL, int NLAY, int NWAVE, int PPT>
__global__ __launch_bounds__(64 * NWAVE, PPT == 1 ? 8 : 4) void k_raster_layers_fwd(RasterArgs a) {
  __shared__ StageL<NL> st;
  const TileGeom t = tile_of(a);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int px[PPT], py[PPT], bx[PPT], by[PPT];
  float pxf[PPT], pyf[PPT];
  bool inside[PPT];
  float T[PPT][NLAY];
  float2 U[PPT][NLAY][NL];
  uint32_t stop[PPT][NLAY];
  uint32_t live[PPT];   // layers still accepting contributions
  uint32_t walk_end[PPT];
  const uint2 rg = a.ranges[t.id];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    block_of(a, t, wave * PPT + p, bx[p], by[p]);
    px[p] = bx[p] + (lane & 7);
    py[p] = by[p] + (lane >> 3);
    pxf[p] = (float)px[p] + 0.5f;
    pyf[p] = (float)py[p] + 0.5f;
    inside[p] = px[p] < a.width && py[p] < a.height;
#pragma unroll
    for (int q = 0; q < NLAY; ++q) {
      T[p][q] = 1.0f;
      stop[p][q] = ~0u;
#pragma unroll
      for (int l = 0; l < NL; ++l) U[p][q][l] = make_float2(0.f, 0.f);
    }
    live[p] = inside[p] ? (1u << a.n_layers) - 1u : 0u;
    walk_end[p] = inside[p] ? rg.y : 0u;
  }
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;
  for (uint32_t start = rg.x; start < rg.y; start += kBatch) {
    uint32_t any_live = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) any_live |= live[p];
    if (!__syncthreads_or(any_live != 0u)) break;   // every layer of every pixel has stopped
    const int cnt = (int)min(rg.y - start, (uint32_t)kBatch);
    stage_records_l<NL>(st, a, start, cnt, false);
    __syncthreads();
    if (__any(any_live != 0u)) {
      // layers still live at some pixel of the wave; pairs of other layers are skipped
      uint32_t wave_live = 0;
#pragma unroll
      for (int q = 0; q < NLAY; ++q)
        if (__any((any_live >> q) & 1u)) wave_live |= 1u << q;
      uint64_t hits[PPT], todo = 0;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        hits[p] = block_hits(st.s.g0, st.s.g1, st.s.rc, 0, cnt, bx[p], by[p]);
        todo |= hits[p];
      }
      const int lane_lay = lane < cnt ? st.lay[lane] : 0;   // lane j holds pair j's layer byte
      todo &= __ballot(lane < cnt && ((wave_live >> (lane_lay & 7)) & 1u));
      while (todo) {
        const int j = (int)__builtin_ctzll(todo);
        todo &= todo - 1;
        const int4 rc = st.s.rc[j];
        const int lay = __builtin_amdgcn_readlane(lane_lay, j) & 7;
        const float4 g0 = st.s.g0[j];
        const float4 g1 = st.s.g1[j];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          if (PPT > 1 && !((hits[p] >> j) & 1u)) continue;
          const float dx = pxf[p] - g0.x, dy = pyf[p] - g0.y;
          const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
          const bool in_rect =
              (unsigned)(px[p] - rc.x) <= (unsigned)rc.y && (unsigned)(py[p] - rc.z) <= (unsigned)rc.w;
          const float aval = fminf(a.alpha_max, g1.y * __expf(-power));
          if (((live[p] >> lay) & 1u) && in_rect && power <= half_k2 && aval >= a.alpha_min) {
#pragma unroll
            for (int q = 0; q < NLAY; ++q) {
              if (q != lay) continue;   // wave-uniform
              const float wgt = aval * T[p][q];
#pragma unroll
              for (int l = 0; l < NL; ++l) {
                const float2 v = st.s.v[l][j];
                U[p][q][l].x += v.x * wgt;
                U[p][q][l].y += v.y * wgt;
              }
              T[p][q] *= 1.0f - aval;
              if (T[p][q] < a.t_min) {
                stop[p][q] = start + j + 1;
                live[p] &= ~(1u << q);
                if (live[p] == 0u) walk_end[p] = start + j + 1;
              }
            }
          }
        }
      }
    }
    __syncthreads();   // the next batch overwrites the staged records
  }
  const size_t plane = (size_t)a.height * a.width;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (!inside[p]) continue;
    const size_t pix = (size_t)py[p] * a.width + px[p];
#pragma unroll
    for (int q = 0; q < NLAY; ++q) {
      const size_t lp = ((size_t)t.view * a.n_layers + q) * plane + pix;
#pragma unroll
      for (int l = 0; l < NL; ++l)
        a.field[(((size_t)t.view * NL + l) * a.n_layers + q) * plane + pix] = U[p][q][l];
      a.t_final[lp] = T[p][q];
      a.layer_stop[lp] = stop[p][q];
    }
    a.last[(size_t)t.view * plane + pix] = walk_end[p];
  }
}

// PPT pixels per lane (one in each of the wave's PPT 8x8 blocks) share the
// pair's record reads and its wave reduction.  One pixel per lane keeps the
// state in 80 registers (six waves per SIMD); two pixels per lane need about
// twice the per-pixel state (36 registers per pixel at four layers and three
// wavelengths) at four waves per SIMD.
template <int NL, int NLAY, int NWAVE, int PPT>
__global__ __launch_bounds__(64 * NWAVE, PPT == 1 ? 5 : 4) void k_raster_layers_bwd(RasterArgs a) {
  constexpr int G2 = 6 + 2 * NL + NLAY;
  constexpr int G2P = (G2 + 3) & ~3;
  __shared__ StageL<NL> st;
  __shared__ float s_grad[kBatch][G2];
  __shared__ uint32_t s_last[NWAVE];
  const TileGeom t = tile_of(a);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const float scale = a.grad_scale ? *a.grad_scale : 1.0f;
  const size_t plane = (size_t)a.height * a.width;
  int px[PPT], py[PPT], bx[PPT], by[PPT];
  float pxf[PPT], pyf[PPT];
  float T[PPT][NLAY];
  uint32_t stop[PPT][NLAY];
  float2 G[PPT][NLAY][NL];
  float K[PPT][NLAY];   // sum over wavelengths of Re(conj(G) B) of each layer
  uint32_t mylast[PPT];
  uint32_t wave_last = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    block_of(a, t, wave * PPT + p, bx[p], by[p]);
    px[p] = bx[p] + (lane & 7);
    py[p] = by[p] + (lane >> 3);
    pxf[p] = (float)px[p] + 0.5f;
    pyf[p] = (float)py[p] + 0.5f;
    const bool inside = px[p] < a.width && py[p] < a.height;
    const size_t pix = (size_t)py[p] * a.width + px[p];
    mylast[p] = inside ? a.last[(size_t)t.view * plane + pix] : 0u;
    wave_last = max(wave_last, mylast[p]);
#pragma unroll
    for (int q = 0; q < NLAY; ++q) {
      T[p][q] = 1.0f;
      stop[p][q] = 0u;
      K[p][q] = 0.f;
#pragma unroll
      for (int l = 0; l < NL; ++l) G[p][q][l] = make_float2(0.f, 0.f);
      if (inside) {
        const size_t lp = ((size_t)t.view * a.n_layers + q) * plane + pix;
        T[p][q] = a.t_final[lp];
        stop[p][q] = a.layer_stop[lp];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const float2 gg = a.grad_field[(((size_t)t.view * NL + l) * a.n_layers + q) * plane + pix];
          G[p][q][l] = make_float2(gg.x * scale, gg.y * scale);
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, off, 64));
  wave_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_last);
  if (lane == 0) s_last[wave] = wave_last;
  for (int i = threadIdx.x; i < kBatch * G2; i += blockDim.x) (&s_grad[0][0])[i] = 0.f;
  __syncthreads();
  uint32_t tile_last = 0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) tile_last = max(tile_last, s_last[w]);
  tile_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)tile_last);
  const uint2 rg = a.ranges[t.id];
  const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;

  for (uint32_t top = tile_last; top > rg.x;) {
    const int cnt = (int)min(top - rg.x, (uint32_t)kBatch);
    stage_records_l<NL>(st, a, top - 1, cnt, true);   // st[j] is the j-th pair from the back
    __syncthreads();
    if (top - cnt < wave_last) {   // this wave has work in the batch
      // pairs at or past wave_last touch none of this wave's pixels
      const int j0 = top > wave_last ? (int)min(top - wave_last, (uint32_t)cnt) : 0;
      uint64_t hits[PPT], todo = 0;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        hits[p] = block_hits(st.s.g0, st.s.g1, st.s.rc, j0, cnt, bx[p], by[p]);
        todo |= hits[p];
      }
      while (todo) {
        const int j = (int)__builtin_ctzll(todo);
        todo &= todo - 1;
        const int4 rc = st.s.rc[j];
        const uint32_t pidx = top - 1 - j;
        const int packed = __builtin_amdgcn_readfirstlane(st.lay[j]);
        const uint32_t ste_live = (uint32_t)packed >> 4;
        // One copy of the pair's work per layer, chosen by the Gaussian's own
        // layer (wave-uniform): inside a copy that layer is a constant, so
        // only its T and K change and nothing else crosses the branches.
        with_layer<0, NLAY>(packed & 7, [&](auto own_layer) {
          constexpr int LAY = decltype(own_layer)::value;
          const float4 g0 = st.s.g0[j];
          const float4 g1 = st.s.g1[j];
          float2 v[NL];
#pragma unroll
          for (int l = 0; l < NL; ++l) v[l] = st.s.v[l][j];
          // per-pair sums over the lane's pixels (with one pixel, the terms
          // every supported pixel writes are assigned, not added to zero)
          float gr[G2P];
#pragma unroll
          for (int c = 0; c < G2P; ++c)
            if (PPT > 1 || c >= 6 + 2 * NL) gr[c] = 0.f;
          auto acc = [&](float& g, float x) { g = PPT == 1 ? x : g + x; };
          bool any = false;
#pragma unroll
          for (int p = 0; p < PPT; ++p) {
            if (PPT > 1 && !((hits[p] >> j) & 1u)) continue;
            // A pixel gains nothing from this pair past its own layer's stop
            // unless it is still live in another layer with a nonzero
            // straight-through weight.
            uint32_t reach = stop[p][LAY];
#pragma unroll
            for (int q = 0; q < NLAY; ++q)
              if (q != LAY && ((ste_live >> q) & 1u)) reach = max(reach, stop[p][q]);
            const float dx = pxf[p] - g0.x, dy = pyf[p] - g0.y;
            const float power = 0.5f * (g0.z * dx * dx + g1.x * dy * dy) + g0.w * dx * dy;
            const bool in_rect =
                (unsigned)(px[p] - rc.x) <= (unsigned)rc.y && (unsigned)(py[p] - rc.z) <= (unsigned)rc.w;
            const float Gv = __expf(-power);
            const float oG = g1.y * Gv;
            const bool clamped = oG > a.alpha_max;
            const float aval = clamped ? a.alpha_max : oG;
            const bool sup =
                pidx < reach && pidx < mylast[p] && in_rect && power <= half_k2 && aval >= a.alpha_min;
            if (!__any(sup)) continue;
            any = true;
            // Branch-free per pixel: where the own layer is not active it
            // takes alpha = 0 (its T and K stay exactly unchanged), and
            // another layer's straight-through term is zero.
            const bool act = sup && pidx < stop[p][LAY];   // the own layer had not stopped before this pair
            float dq = 0.f;
#pragma unroll
            for (int l = 0; l < NL; ++l) dq += G[p][LAY][l].x * v[l].x + G[p][LAY][l].y * v[l].y;
            const float raw = dq - K[p][LAY];   // sum_l Re(conj(G) (v - B)) of the own layer
            const float ae = act ? aval : 0.f;
            const float Tb = T[p][LAY] * __builtin_amdgcn_rcpf(1.0f - ae);
            const float so = raw * Tb;
            acc(gr[6 + 2 * NL + LAY], ae * so);
            const float dLda = act ? so : 0.f;
            const float aT = ae * Tb;
#pragma unroll
            for (int l = 0; l < NL; ++l) {
              acc(gr[6 + 2 * l], aT * G[p][LAY][l].x);
              acc(gr[7 + 2 * l], aT * G[p][LAY][l].y);
            }
            K[p][LAY] += ae * raw;   // B <- B + a (v - B)
            T[p][LAY] = Tb;
#pragma unroll
            for (int q = 0; q < NLAY; ++q) {
              if (q == LAY || !((ste_live >> q) & 1u)) continue;   // zero straight-through weight
              float d = 0.f;
#pragma unroll
              for (int l = 0; l < NL; ++l) d += G[p][q][l].x * v[l].x + G[p][q][l].y * v[l].y;
              // zero where layer q had stopped before this pair
              const bool act_q = sup && pidx < stop[p][q];
              acc(gr[6 + 2 * NL + q], act_q ? aval * ((d - K[p][q]) * T[p][q]) : 0.f);
            }
            // clamped pixels pass no gradient to the opacity or the conic
            const float dl = clamped ? 0.f : dLda;
            const float dpow = -aval * dl;
            acc(gr[5], Gv * dl);
            acc(gr[2], 0.5f * dx * dx * dpow);
            acc(gr[3], dx * dy * dpow);
            acc(gr[4], 0.5f * dy * dy * dpow);
            acc(gr[0], -(g0.z * dx + g0.w * dy) * dpow);
            acc(gr[1], -(g0.w * dx + g1.x * dy) * dpow);
          }
          if (!any) return;
          wave_sums_by_row<G2P>(gr);
          if ((lane & 15) == 15) {
            const int row = lane >> 4;
#pragma unroll
            for (int k = 0; k < G2P / 4; ++k) {
              const int c = k + row * (G2P / 4);
              if (c < G2) {
                if (NWAVE == 1)
                  s_grad[j][c] = gr[k];
                else
                  atomicAdd(&s_grad[j][c], gr[k]);
              }
            }
          }
        });
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * G2; i += blockDim.x) {
      const int r = i / G2, c = i - r * G2;
      const float sum = s_grad[r][c];
      if (sum != 0.f) unsafeAtomicAdd(a.grad2d + (size_t)st.s.rid[r] * a.g2stride + c, sum);
      s_grad[r][c] = 0.f;
    }
    __syncthreads();   // the next batch overwrites the staged records
    top -= cnt;
  }
}

// Straight-through estimator (Eq. 12, backward): the summed dL/drho of every
// view times softmax(logits / tau).
__global__ void k_logits_backward(const float* __restrict__ logits, const float* __restrict__ grad2d, int g2s,
                                  int rho_off, const uint32_t* __restrict__ count, int n, int n_stride, int n_views,
                                  int nlay, float inv_tau, float* __restrict__ d_logits) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float drho[kMaxLayers], w[kMaxLayers];
  float mx = logits[(size_t)g * nlay] * inv_tau;
  for (int q = 0; q < nlay; ++q) {
    drho[q] = 0.f;
    w[q] = logits[(size_t)g * nlay + q] * inv_tau;
    mx = fmaxf(mx, w[q]);
  }
  for (int b = 0; b < n_views; ++b) {
    const size_t rid = (size_t)b * n_stride + g;
    if (count[rid] == 0) continue;
    for (int q = 0; q < nlay; ++q) drho[q] += grad2d[rid * g2s + rho_off + q];
  }
  float sum = 0.f;
  for (int q = 0; q < nlay; ++q) {
    w[q] = expf(w[q] - mx);
    sum += w[q];
  }
  const uint32_t live = ste_live_layers(logits + (size_t)g * nlay, nlay, inv_tau);
  for (int q = 0; q < nlay; ++q)
    d_logits[(size_t)g * nlay + q] = ((live >> q) & 1u) ? drho[q] * (w[q] / sum) : 0.0f;
}

hipError_t launch_assign_layers(const float* logits, int n, int n_layers, float tau, uint8_t* layer_of,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n_layers < 1 || n_layers > kMaxLayers) return hipErrorInvalidValue;
  k_assign_layers<<<(n + 255) / 256, 256, 0, s>>>(logits, n, n_layers, 1.0f / tau, layer_of);
  return hipGetLastError();
}

hipError_t launch_logits_backward(const float* logits, const float* grad2d, int g2stride, int rho_offset,
                                  const uint32_t* count, int n, int n_stride, int n_views, int n_layers, float tau,
                                  float* d_logits, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_logits_backward<<<(n + 255) / 256, 256, 0, s>>>(logits, grad2d, g2stride, rho_offset, count, n, n_stride,
                                                    n_views, n_layers, 1.0f / tau, d_logits);
  return hipGetLastError();
}

// Pixels per lane of the forward at two or more 8x8 blocks per tile.
#ifndef CHRF_LAYERS_FWD_PPT
#define CHRF_LAYERS_FWD_PPT 1
#endif

template <int NL, int NLAY>
static void launch_layers_fwd_nl(const RasterArgs& a, int blocks, int bpt, hipStream_t s) {
  constexpr int P = CHRF_LAYERS_FWD_PPT;
  static_assert(P == 1 || P == 2, "one or two pixels per lane");
  if (bpt == 1)
    k_raster_layers_fwd<NL, NLAY, 1, 1><<<blocks, 64, 0, s>>>(a);
  else if (bpt == 2)
    k_raster_layers_fwd<NL, NLAY, 2 / P, P><<<blocks, 64 * (2 / P), 0, s>>>(a);
  else
    k_raster_layers_fwd<NL, NLAY, 4 / P, P><<<blocks, 64 * (4 / P), 0, s>>>(a);
}



// Pixels per lane of the backward at two or more 8x8 blocks per tile, where
// two pixels' state fits the 128-VGPR budget: a pixel keeps T, the stop index
// and K per layer plus G per layer and wavelength, NLAY (2 NL + 3) registers;
// beyond 36 (three wavelengths and four layers) one pixel per lane spills less.
#ifndef CHRF_LAYERS_BWD_PPT
#define CHRF_LAYERS_BWD_PPT 2
#endif

template <int NL, int NLAY>
static void launch_layers_bwd_nl(const RasterArgs& a, int blocks, int bpt, hipStream_t s) {
  constexpr int P = NLAY * (2 * NL + 3) <= 36 ? CHRF_LAYERS_BWD_PPT : 1;
  static_assert(P == 1 || P == 2, "one or two pixels per lane");
  if (bpt == 1)
    k_raster_layers_bwd<NL, NLAY, 1, 1><<<blocks, 64, 0, s>>>(a);
  else if (bpt == 2)
    k_raster_layers_bwd<NL, NLAY, 2 / P, P><<<blocks, 64 * (2 / P), 0, s>>>(a);
  else
    k_raster_layers_bwd<NL, NLAY, 4 / P, P><<<blocks, 64 * (4 / P), 0, s>>>(a);
}

// Checks the launch shape and calls LAUNCH<n_lambda, n_layers>(a, blocks,
// 8x8 blocks per tile, s).
#define CHRF_LAYERS_CASE(LAUNCH, NL, NLAY) \
  case NL * 8 + NLAY:                      \
    LAUNCH<NL, NLAY>(a, blocks, bpt, s);   \
    break;
#define CHRF_LAYERS_DISPATCH(LAUNCH)                                                                     \
  const int blocks = a.n_views * a.tiles_x * a.tiles_y;                                                 \
  if (blocks == 0) return hipSuccess;                                                                   \
  const int bpt = a.tile_w * a.tile_h / 64;                                                             \
  if ((bpt != 1 && bpt != 2 && bpt != 4) || a.tile_w % 8 || a.tile_h % 8 || a.n_layers < 1 ||           \
      a.n_layers > kMaxLayers || a.n_lambda < 1 || a.n_lambda > 4)                                       \
    return hipErrorInvalidValue;                                                                        \
  switch (a.n_lambda * 8 + a.n_layers) {                                                                \
    CHRF_LAYERS_CASE(LAUNCH, 1, 1) CHRF_LAYERS_CASE(LAUNCH, 1, 2) CHRF_LAYERS_CASE(LAUNCH, 1, 3)        \
    CHRF_LAYERS_CASE(LAUNCH, 1, 4) CHRF_LAYERS_CASE(LAUNCH, 2, 1) CHRF_LAYERS_CASE(LAUNCH, 2, 2)        \
    CHRF_LAYERS_CASE(LAUNCH, 2, 3) CHRF_LAYERS_CASE(LAUNCH, 2, 4) CHRF_LAYERS_CASE(LAUNCH, 3, 1)        \
    CHRF_LAYERS_CASE(LAUNCH, 3, 2) CHRF_LAYERS_CASE(LAUNCH, 3, 3) CHRF_LAYERS_CASE(LAUNCH, 3, 4)        \
    CHRF_LAYERS_CASE(LAUNCH, 4, 1) CHRF_LAYERS_CASE(LAUNCH, 4, 2) CHRF_LAYERS_CASE(LAUNCH, 4, 3)        \
    CHRF_LAYERS_CASE(LAUNCH, 4, 4)                                                                      \
    default: return hipErrorInvalidValue;                                                               \
  }                                                                                                     \
  return hipGetLastError();

hipError_t launch_raster_layers_forward(const RasterArgs& a, hipStream_t s) {
  CHRF_LAYERS_DISPATCH(launch_layers_fwd_nl)
}

hipError_t launch_raster_layers_backward(const RasterArgs& a, hipStream_t s) {
  CHRF_LAYERS_DISPATCH(launch_layers_bwd_nl)
}

}  // namespace chrf
