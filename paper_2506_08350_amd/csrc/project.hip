// Projection of complex 3D Gaussians to screen-space records (forward) and the
// chain of 2D gradients back to the 3D parameters (backward).
//
// Forward follows Sec. 3 (Eqs. 2-4) and Sec. 4.1 (Eqs. 8, 10):
//   Sigma = R S S^T R^T, Sigma' = J W Sigma W^T J^T, mu = pinhole(W x + t).
// It is written as Sigma' = T T^T with T = J W R diag(exp(s)) (2x3), which is
// the same matrix.  The depth key, the culling tests and the support
// rectangle decide integers (sort order, tile lists), so they follow a fixed
// single-precision recipe: every operation below is one IEEE float operation
// in source order, with contraction into fused multiply-adds disabled; the
// CPU reference reproduces the same recipe bit for bit.
#include "internal.h"

namespace chrf {

__global__ __launch_bounds__(256) void k_project(ProjArgs a) {
#pragma clang fp contract(off)
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  {
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x * gridDim.y;
    const int64_t tid = (int64_t)b * gridDim.x * blockDim.x + g;
    for (int64_t i = tid; i < a.n_clear_a; i += nthreads) a.clear_a[i] = 0u;
    for (int64_t i = tid; i < a.n_clear_b; i += nthreads) a.clear_b[i] = 0u;
  }
  if (b == 0 && g < a.n && a.v) {
    for (int l = 0; l < a.n_lambda; ++l) {
      float sn, cs;
      sincosf(a.phase[(size_t)g * a.n_lambda + l], &sn, &cs);
      const float am = a.amp[(size_t)g * a.n_lambda + l];
      a.v[(size_t)g * a.n_lambda + l] = make_float2(am * cs, am * sn);
    }
  }
  if (g >= a.n_stride) return;
  const size_t rid = (size_t)b * a.n_stride + g;
  if (a.grad2d) {   // every row of the view, used or not
    float* gp = a.grad2d + rid * a.grad2d_stride;
    if (a.grad2d_stride % 4 == 0 && (reinterpret_cast<uintptr_t>(a.grad2d) & 15u) == 0) {
      for (int c = 0; c < a.grad2d_stride; c += 4) *reinterpret_cast<float4*>(gp + c) = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      for (int c = 0; c < a.grad2d_stride; ++c) gp[c] = 0.0f;
    }
  }
  if (g >= a.n) {   // unused slots sort last and emit nothing
    a.count[rid] = 0;
    a.sort_key[rid] = ((uint64_t)b << 32) | 0xffffffffull;
    a.sort_val[rid] = (uint32_t)rid;
    return;
  }
  const Cam& cam = a.cams[b];

  const float mx = a.means[3 * g], my = a.means[3 * g + 1], mz = a.means[3 * g + 2];
  const float* R = cam.R;
  const float tcx = ((R[0] * mx + R[1] * my) + R[2] * mz) + cam.t[0];
  const float tcy = ((R[3] * mx + R[4] * my) + R[5] * mz) + cam.t[1];
  const float tcz = ((R[6] * mx + R[7] * my) + R[8] * mz) + cam.t[2];

  const float qw0 = a.quats[4 * g], qx0 = a.quats[4 * g + 1], qy0 = a.quats[4 * g + 2], qz0 = a.quats[4 * g + 3];
  const float n2 = ((qw0 * qw0 + qx0 * qx0) + qy0 * qy0) + qz0 * qz0;
  const float nq = __builtin_sqrtf(n2);
  const float w = qw0 / nq, x = qx0 / nq, y = qy0 / nq, z = qz0 / nq;
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  float Q[9];
  Q[0] = 1.0f - 2.0f * (yy + zz);
  Q[1] = 2.0f * (xy - wz);
  Q[2] = 2.0f * (xz + wy);
  Q[3] = 2.0f * (xy + wz);
  Q[4] = 1.0f - 2.0f * (xx + zz);
  Q[5] = 2.0f * (yz - wx);
  Q[6] = 2.0f * (xz - wy);
  Q[7] = 2.0f * (yz + wx);
  Q[8] = 1.0f - 2.0f * (xx + yy);
  float A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = (R[3 * i] * Q[j] + R[3 * i + 1] * Q[3 + j]) + R[3 * i + 2] * Q[6 + j];

  const float ux = tcx / tcz, uy = tcy / tcz;
  const float gx = cam.fx / tcz, gy = cam.fy / tcz;
  float es[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) es[j] = (float)exp((double)a.log_scales[3 * g + j]);
  float T0[3], T1[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T0[j] = (gx * (A[j] - ux * A[6 + j])) * es[j];
    T1[j] = (gy * (A[3 + j] - uy * A[6 + j])) * es[j];
  }
  const float sxx = (T0[0] * T0[0] + T0[1] * T0[1]) + T0[2] * T0[2];
  const float syy = (T1[0] * T1[0] + T1[1] * T1[1]) + T1[2] * T1[2];
  const float sxy = (T0[0] * T1[0] + T0[1] * T1[1]) + T0[2] * T1[2];
  const float det = sxx * syy - sxy * sxy;
  const float mux = cam.fx * ux + cam.cx;
  const float muy = cam.fy * uy + cam.cy;
  const float ex = a.k_sigma * __builtin_sqrtf(sxx) + 0.01f;
  const float ey = a.k_sigma * __builtin_sqrtf(syy) + 0.01f;
  bool ok = (tcz > cam.z_near) && (det > 0.0f);
  ok = ok && __builtin_isfinite(ex) && __builtin_isfinite(ey) && __builtin_isfinite(mux) && __builtin_isfinite(muy);
  int c0 = 0, c1 = -1, r0 = 0, r1 = -1;
  if (ok) {
    const float Wf = (float)a.width, Hf = (float)a.height;
    const float xl = fminf(fmaxf((mux - ex) - 0.5f, -1.0f), Wf);
    const float xh = fminf(fmaxf((mux + ex) - 0.5f, -1.0f), Wf);
    const float yl = fminf(fmaxf((muy - ey) - 0.5f, -1.0f), Hf);
    const float yh = fminf(fmaxf((muy + ey) - 0.5f, -1.0f), Hf);
    c0 = max((int)ceilf(xl), 0);
    c1 = min((int)floorf(xh), a.width - 1);
    r0 = max((int)ceilf(yl), 0);
    r1 = min((int)floorf(yh), a.height - 1);
  }
  const bool visible = ok && c0 <= c1 && r0 <= r1;
  uint32_t cnt = 0;
  if (visible) {
    const int tx0 = c0 / a.tile_w, tx1 = c1 / a.tile_w, ty0 = r0 / a.tile_h, ty1 = r1 / a.tile_h;
    cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    const float A_ = syy / det, B_ = -sxy / det, C_ = sxx / det;
    // Largest power at which the Gaussian can still support a pixel:
    // power <= k^2 / 2, and o exp(-power) >= alpha_min (alpha_min < alpha_max)
    // means power <= ln(o / alpha_min).  Pair emission uses it to bin a
    // Gaussian only to the tiles its ellipse can reach, the raster kernels to
    // skip 8x8 blocks.  The tile decision must be reproducible on the CPU, so
    // the logarithm is taken in double precision and rounded once to float
    // (equal to the correctly rounded float logarithm except when the exact
    // value lies within a double ulp of a float rounding boundary).
    const float op = a.opacity[g];
    const float half_k2 = 0.5f * a.k_sigma * a.k_sigma;
    const float pmax =
        a.alpha_min > 0.0f ? (float)fmin((double)half_k2, log((double)op / (double)a.alpha_min)) : half_k2;
    a.rec_g0[rid] = make_float4(mux, muy, A_, B_);
    a.rec_g1[rid] = make_float4(C_, op, pmax, 0.0f);
    a.rec_rect[rid] = make_int4(c0, c1 - c0, r0, r1 - r0);
  }
  a.count[rid] = cnt;
  const uint32_t depth_bits = visible ? __float_as_uint(tcz) : 0xffffffffu;
  a.sort_key[rid] = ((uint64_t)b << 32) | depth_bits;
  a.sort_val[rid] = (uint32_t)rid;
}

hipError_t launch_project(const ProjArgs& a, hipStream_t s) {
  if (a.n_stride == 0 || a.n_views == 0) return hipSuccess;
  dim3 grid((a.n_stride + 255) / 256, a.n_views);
  k_project<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Backward (Supplementary D backward pass).  One thread per Gaussian sums the
// per-view 2D gradients (d mu, d conic, d opacity, d v) chained through
//   conic = Sigma'^{-1}:      G_Sigma' = -Q G_Q Q
//   Sigma' = J M J^T:         G_M = J^T G_Sigma' J,  G_J = 2 G_Sigma' J M
//   M = W Sigma W^T:          G_Sigma = W^T G_M W
//   Sigma = Rq diag(e^{2s}) Rq^T:  dL/ds_j = 2 e^{2 s_j} (Rq^T G_Sigma Rq)_jj,
//                             G_Rq = 2 G_Sigma Rq diag(e^{2s})
//   Rq(q / |q|), the pinhole mean and J(t), t = W x + t0.
// The dependence of J on t is kept.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_project_backward(
    const float* __restrict__ means, const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ amp, const float* __restrict__ phase, const Cam* __restrict__ cams, int n,
    int n_stride, int n_views, int n_lambda, const uint32_t* __restrict__ count, const float* __restrict__ grad2d,
    int g2s, float* d_means, float* d_log_scales, float* d_quats, float* d_opacity, float* d_amp,
    float* d_phase) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float qw0 = quats[4 * g], qx0 = quats[4 * g + 1], qy0 = quats[4 * g + 2], qz0 = quats[4 * g + 3];
  const float qn = sqrtf(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
  const float w = qw0 / qn, x = qx0 / qn, y = qy0 / qn, z = qz0 / qn;
  float Rq[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                 2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                 2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
  float s2[3];
  for (int j = 0; j < 3; ++j) s2[j] = expf(2.0f * log_scales[3 * g + j]);
  // Sigma = Rq diag(s2) Rq^T
  float Sig[9];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Sig[3 * i + k] = Rq[3 * i] * s2[0] * Rq[3 * k] + Rq[3 * i + 1] * s2[1] * Rq[3 * k + 1] +
                                                 Rq[3 * i + 2] * s2[2] * Rq[3 * k + 2];
  float gm[3] = {0, 0, 0}, gsig[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gop = 0.f;
  float gv[2 * kMaxLambda];
  for (int l = 0; l < 2 * kMaxLambda; ++l) gv[l] = 0.f;
  const float mx = means[3 * g], my = means[3 * g + 1], mz = means[3 * g + 2];
  for (int b = 0; b < n_views; ++b) {
    const size_t rid = (size_t)b * n_stride + g;
    if (count[rid] == 0) continue;
    // the row's 6 + 2 n_lambda values, read as 16-byte words when the rows allow it
    float gp[6 + 2 * kMaxLambda + 2];
    const float* src = grad2d + rid * g2s;
    const int nv = 6 + 2 * n_lambda;
    if (g2s % 4 == 0 && (reinterpret_cast<uintptr_t>(grad2d) & 15u) == 0) {
#pragma unroll
      for (int c = 0; c < 6 + 2 * kMaxLambda + 2; c += 4) {
        if (c < nv) {
          const float4 q = *reinterpret_cast<const float4*>(src + c);
          gp[c] = q.x;
          gp[c + 1] = q.y;
          gp[c + 2] = q.z;
          gp[c + 3] = q.w;
        }
      }
    } else {
      for (int c = 0; c < nv; ++c) gp[c] = src[c];
    }
    const float dmx = gp[0], dmy = gp[1], dA = gp[2], dB = gp[3], dC = gp[4];
    gop += gp[5];
    for (int l = 0; l < 2 * n_lambda; ++l) gv[l] += gp[6 + l];
    const Cam& cam = cams[b];
    const float* W = cam.R;
    const float tx = W[0] * mx + W[1] * my + W[2] * mz + cam.t[0];
    const float ty = W[3] * mx + W[4] * my + W[5] * mz + cam.t[1];
    const float tz = W[6] * mx + W[7] * my + W[8] * mz + cam.t[2];
    const float iz = 1.0f / tz, iz2 = iz * iz;
    const float J00 = cam.fx * iz, J02 = -cam.fx * tx * iz2, J11 = cam.fy * iz, J12 = -cam.fy * ty * iz2;
    // M = W Sigma W^T
    float WS[9], M[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) WS[3 * i + k] = W[3 * i] * Sig[k] + W[3 * i + 1] * Sig[3 + k] + W[3 * i + 2] * Sig[6 + k];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) M[3 * i + k] = WS[3 * i] * W[3 * k] + WS[3 * i + 1] * W[3 * k + 1] + WS[3 * i + 2] * W[3 * k + 2];
    // Sigma' = J M J^T, J = [[J00, 0, J02], [0, J11, J12]]
    const float JM0[3] = {J00 * M[0] + J02 * M[6], J00 * M[1] + J02 * M[7], J00 * M[2] + J02 * M[8]};
    const float JM1[3] = {J11 * M[3] + J12 * M[6], J11 * M[4] + J12 * M[7], J11 * M[5] + J12 * M[8]};
    const float c00 = JM0[0] * J00 + JM0[2] * J02;
    const float c01 = JM0[1] * J11 + JM0[2] * J12;
    const float c11 = JM1[1] * J11 + JM1[2] * J12;
    const float det = c00 * c11 - c01 * c01;
    const float id = 1.0f / det;
    const float qa = c11 * id, qb = -c01 * id, qc = c00 * id;
    // G_Sigma' = -Q G_Q Q with G_Q = [[dA, dB/2], [dB/2, dC]]
    const float h = 0.5f * dB;
    const float t00 = qa * dA + qb * h, t01 = qa * h + qb * dC;
    const float t10 = qb * dA + qc * h, t11 = qb * h + qc * dC;
    const float G00 = -(t00 * qa + t01 * qb), G01 = -(t00 * qb + t01 * qc);
    const float G11 = -(t10 * qb + t11 * qc);
    // G_J = 2 G J M (2x3): rows of G J M = G00 JM0 + G01 JM1, G01 JM0 + G11 JM1
    float GJ0[3], GJ1[3];
    for (int k = 0; k < 3; ++k) {
      GJ0[k] = 2.0f * (G00 * JM0[k] + G01 * JM1[k]);
      GJ1[k] = 2.0f * (G01 * JM0[k] + G11 * JM1[k]);
    }
    // G_M = J^T G J (3x3), J rows j0 = (J00, 0, J02), j1 = (0, J11, J12)
    const float j0[3] = {J00, 0.f, J02}, j1[3] = {0.f, J11, J12};
    float GM[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k)
        GM[3 * i + k] = j0[i] * (G00 * j0[k] + G01 * j1[k]) + j1[i] * (G01 * j0[k] + G11 * j1[k]);
    // G_Sigma += W^T G_M W
    float T[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) T[3 * i + k] = GM[3 * i] * W[k] + GM[3 * i + 1] * W[3 + k] + GM[3 * i + 2] * W[6 + k];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) gsig[3 * i + k] += W[i] * T[k] + W[3 + i] * T[3 + k] + W[6 + i] * T[6 + k];
    // camera-space centre
    const float fx = cam.fx, fy = cam.fy;
    float dt0 = dmx * fx * iz + GJ0[2] * (-fx * iz2);
    float dt1 = dmy * fy * iz + GJ1[2] * (-fy * iz2);
    float dt2 = -dmx * fx * tx * iz2 - dmy * fy * ty * iz2 + GJ0[0] * (-fx * iz2) +
                GJ0[2] * (2.0f * fx * tx * iz2 * iz) + GJ1[1] * (-fy * iz2) + GJ1[2] * (2.0f * fy * ty * iz2 * iz);
    gm[0] += W[0] * dt0 + W[3] * dt1 + W[6] * dt2;
    gm[1] += W[1] * dt0 + W[4] * dt1 + W[7] * dt2;
    gm[2] += W[2] * dt0 + W[5] * dt1 + W[8] * dt2;
  }
  // scales and rotation
  float RtG[9], RtGR[9];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) RtG[3 * i + k] = Rq[i] * gsig[k] + Rq[3 + i] * gsig[3 + k] + Rq[6 + i] * gsig[6 + k];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) RtGR[3 * i + k] = RtG[3 * i] * Rq[k] + RtG[3 * i + 1] * Rq[3 + k] + RtG[3 * i + 2] * Rq[6 + k];
  for (int j = 0; j < 3; ++j) d_log_scales[3 * g + j] = 2.0f * s2[j] * RtGR[4 * j];
  float GR[9];   // 2 G_Sigma Rq diag(s2)
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      GR[3 * i + k] = 2.0f * (gsig[3 * i] * Rq[k] + gsig[3 * i + 1] * Rq[3 + k] + gsig[3 * i + 2] * Rq[6 + k]) * s2[k];
  const float dw = 2.f * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
  const float dx = 2.f * (y * GR[1] + z * GR[2] + y * GR[3] - 2.f * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7] -
                          2.f * x * GR[8]);
  const float dy = 2.f * (-2.f * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7] -
                          2.f * y * GR[8]);
  const float dz = 2.f * (-2.f * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2.f * z * GR[4] + y * GR[5] +
                          x * GR[6] + y * GR[7]);
  const float dot = w * dw + x * dx + y * dy + z * dz;
  d_quats[4 * g] = (dw - w * dot) / qn;
  d_quats[4 * g + 1] = (dx - x * dot) / qn;
  d_quats[4 * g + 2] = (dy - y * dot) / qn;
  d_quats[4 * g + 3] = (dz - z * dot) / qn;
  d_means[3 * g] = gm[0];
  d_means[3 * g + 1] = gm[1];
  d_means[3 * g + 2] = gm[2];
  d_opacity[g] = gop;
  for (int l = 0; l < n_lambda; ++l) {
    float s, c;
    sincosf(phase[g * n_lambda + l], &s, &c);
    const float gr = gv[2 * l], gi = gv[2 * l + 1];
    d_amp[g * n_lambda + l] = gr * c + gi * s;
    d_phase[g * n_lambda + l] = amp[g * n_lambda + l] * (-gr * s + gi * c);
  }
}

hipError_t launch_project_backward(const float* means, const float* log_scales, const float* quats, const float* amp,
                                   const float* phase, const Cam* cams, int n, int n_stride, int n_views,
                                   int n_lambda, const uint32_t* count, const float* grad2d, int g2stride,
                                   float* d_means, float* d_log_scales, float* d_quats, float* d_opacity,
                                   float* d_amp, float* d_phase, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_project_backward<<<(n + 255) / 256, 256, 0, s>>>(means, log_scales, quats, amp, phase, cams, n, n_stride,
                                                      n_views, n_lambda, count, grad2d, g2stride, d_means,
                                                      d_log_scales, d_quats, d_opacity, d_amp, d_phase);
  return hipGetLastError();
}

}  // namespace chrf
