// Tile walk helpers shared by the single-plane and the multi-layer raster
// kernels: tile and pixel geometry, LDS staging of Gaussian records, and the
// wave reductions of the backward passes.
#pragma once
#include "internal.h"

namespace chrf {

// A tile's 8x8 blocks are shared out among the waves (64 lanes) of its
// workgroup.  Lane l sits at (l % 8, l / 8) of an 8x8 block and owns the
// pixel at that position in each of its wave's PPT blocks, so per-pair costs
// that do not depend on the pixel (the gradient reduction over the wave) are
// shared by PPT pixels.  Records are staged in LDS in batches of kBatch pairs.
constexpr int kLanes = 64;
// One staged pair per lane of a wave: a wave finds the pairs that reach its
// block with one ballot per batch.
constexpr int kBatch = 64;

struct TileGeom {
  int id;   // (view, tile) index: view * tiles + tile
  int view, tx, ty;
};

// Workgroups take (view, tile) items in the order of a.tile_order (longest
// pair lists first, so that the short ones fill the end of the launch).
__device__ inline TileGeom tile_of(const RasterArgs& a) {
  const int n_tiles = a.tiles_x * a.tiles_y;
  TileGeom t;
  t.id = a.tile_order ? (int)a.tile_order[blockIdx.x] : (int)blockIdx.x;
  t.view = t.id / n_tiles;
  const int tile = t.id % n_tiles;
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

// Can the Gaussian support any pixel of the 8x8 block at (bx, by)?  A pixel
// is supported only inside the support rectangle rc = (c0, c1 - c0, r0,
// r1 - r0) and where power = d^T conic d / 2 <= pmax (g1.z, set by the
// projection; d = pixel centre - mu).  The test takes the minimum of the
// quadratic form over the box of pixel centres that lie in both the block
// and the rectangle: zero if mu is inside the box, else the smaller of its
// minima along the box edges that face mu (the minimiser of a positive
// definite form over a box that excludes its centre lies on such an edge).
// The margin covers the rounding of the per-pixel power and of this bound,
// so no block holding a supported pixel is ever skipped; a skipped block
// would have taken alpha = 0 at every pixel.
__device__ inline bool support_hits_block(const float4& g0, const float4& g1, const int4& rc, int bx, int by) {
  const int xlo = max(bx, rc.x), xhi = min(bx + 7, rc.x + rc.y);
  const int ylo = max(by, rc.z), yhi = min(by + 7, rc.z + rc.w);
  if (xlo > xhi || ylo > yhi) return false;
  const float x0 = ((float)xlo + 0.5f) - g0.x, x1 = ((float)xhi + 0.5f) - g0.x;
  const float y0 = ((float)ylo + 0.5f) - g0.y, y1 = ((float)yhi + 0.5f) - g0.y;
  const float A = g0.z, B = g0.w, C = g1.x;
  const bool xin = x0 <= 0.f && x1 >= 0.f, yin = y0 <= 0.f && y1 >= 0.f;
  // minimum along the vertical edge facing mu: x = xe, y = -B xe / C clamped
  const float xe = x0 > 0.f ? x0 : x1;
  const float ys = fminf(fmaxf(-B * xe * __builtin_amdgcn_rcpf(C), y0), y1);
  const float qx = 0.5f * (A * xe * xe + C * ys * ys) + B * xe * ys;
  // and along the horizontal edge facing mu
  const float ye = y0 > 0.f ? y0 : y1;
  const float xs = fminf(fmaxf(-B * ye * __builtin_amdgcn_rcpf(A), x0), x1);
  const float qy = 0.5f * (A * xs * xs + C * ye * ye) + B * xs * ye;
  const float lb = xin ? (yin ? 0.f : qy) : (yin ? qx : fminf(qx, qy));
  const float xm = fmaxf(-x0, x1), ym = fmaxf(-y0, y1);   // largest |dx|, |dy| over the box
  const float mag = 0.5f * (A * xm * xm + C * ym * ym) + fabsf(B) * xm * ym;
  return !(lb > g1.z + 1e-4f + 4e-6f * mag);   // NaN: not skipped
}

// Bit j: staged pair j, j_first <= j < cnt, can support a pixel of the 8x8
// block at (bx, by).  Lane j tests pair j; the mask is wave-uniform, so the
// pair walk visits only the set bits, in order, with scalar control.
__device__ inline uint64_t block_hits(const float4* g0, const float4* g1, const int4* rc, int j_first, int cnt,
                                      int bx, int by) {
  const int lane = threadIdx.x & 63;
  bool h = false;
  if (lane >= j_first && lane < cnt) h = support_hits_block(g0[lane], g1[lane], rc[lane], bx, by);
  return __ballot(h);
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
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
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

// Sums over the 16 lanes of each row; the result is valid in the row's last lane.
__device__ inline float row_sum_to_last(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));  // row_shr:1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));  // row_shr:2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));  // row_shr:4
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));  // row_shr:8
  return v;
}

// Wave sums of M values (M a multiple of 4) by recursive halving.  The
// 32-lane swap exchanges the upper half of one value with the lower half of
// another, so one add leaves half the values summed over lane pairs (l, l+32);
// the 16-lane swap does the same between neighbouring rows.  Afterwards row r
// (lanes 16r..16r+15) holds values k + r*M/4, k < M/4, each summed over four
// lanes; a row reduction finishes them.  Result: lane 16r+15 holds the wave
// sum of value k + r*M/4 in v[k].
template <int M>
__device__ inline void wave_sums_by_row(float (&v)[M]) {
  static_assert(M % 4 == 0, "pad the value count to a multiple of 4");
#pragma unroll
  for (int k = 0; k < M / 2; ++k) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + M / 2]), false,
                                                    false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int k = 0; k < M / 4; ++k) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[k]), __float_as_uint(v[k + M / 4]), false,
                                                    false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int k = 0; k < M / 4; ++k) v[k] = row_sum_to_last(v[k]);
}

}  // namespace chrf
