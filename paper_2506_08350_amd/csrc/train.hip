// Training-loop kernels: the Adan update (Sec. 5) and the densification of
// the optimisation algorithm (Supplementary: prune, clone and split with
// phase perturbation, the 3DGS strategy), plus the view-space gradient
// statistics that drive it.
//
// Densification is a stream compaction: a count pass decides how many
// Gaussians each input becomes (0, 1 or 2), an exclusive scan places them,
// and an emit pass writes the output index map, the kinds and the three
// fields that change (means, log-scales, phases).  Other per-Gaussian arrays
// (parameters and optimiser state) follow the index map in a gather pass, so
// outputs keep the input order and are identical from run to run.
#include "internal.h"

namespace chrf {

// ---------------------------------------------------------------- Adan ---
// Decay-coefficient form: m, v, n keep the fractions b1, b2, b3 of their old
// values; d = g - g_prev (zero on the first step, where g_prev is set to g).
// inv_c* are the reciprocal bias corrections 1 / (1 - b^k), computed on the host.
__global__ void k_adan(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ g_prev,
                       float* __restrict__ m, float* __restrict__ v, float* __restrict__ nn, int64_t n, float lr,
                       float b1, float b2, float b3, float eps, float decay, float inv_c1, float inv_c2,
                       float inv_c3, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float d = first ? 0.f : gi - g_prev[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * d;
  const float w = gi + b2 * d;
  const float ni = b3 * nn[i] + (1.f - b3) * w * w;
  m[i] = mi;
  v[i] = vi;
  nn[i] = ni;
  g_prev[i] = gi;
  const float upd = (mi * inv_c1 + b2 * vi * inv_c2) / (sqrtf(ni * inv_c3) + eps);
  x[i] = (x[i] - lr * upd) * decay;
}

hipError_t launch_adan(float* x, const float* g, float* g_prev, float* m, float* v, float* nn, int64_t n, float lr,
                       float b1, float b2, float b3, float eps, float weight_decay, int step, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const double k = (double)step;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, k)));
  const float c2 = b2 > 0.f ? (float)(1.0 / (1.0 - std::pow((double)b2, k))) : 1.0f;
  const float c3 = (float)(1.0 / (1.0 - std::pow((double)b3, k)));
  const float decay = (float)(1.0 / (1.0 + (double)lr * weight_decay));
  k_adan<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, g, g_prev, m, v, nn, n, lr, b1, b2, b3, eps, decay, c1, c2,
                                                     c3, step == 1 ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------- statistics ---
// For every Gaussian, add the norm of dL/d mu_2D of each view that binned it
// (the first two entries of its per-view gradient record) and count the views.
__global__ void k_densify_stats(const float* __restrict__ grad2d, int g2s, const uint32_t* __restrict__ count,
                                int n, int n_stride, int n_views, float* __restrict__ accum,
                                float* __restrict__ seen) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float a = 0.f, c = 0.f;
  for (int b = 0; b < n_views; ++b) {
    const size_t rid = (size_t)b * n_stride + g;
    if (count[rid] == 0) continue;
    const float dx = grad2d[rid * g2s], dy = grad2d[rid * g2s + 1];
    a += sqrtf(dx * dx + dy * dy);
    c += 1.f;
  }
  accum[g] += a;
  seen[g] += c;
}

hipError_t launch_densify_stats(const float* grad2d, int g2stride, const uint32_t* count, int n, int n_stride,
                                int n_views, float* accum, float* seen, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_densify_stats<<<(n + 255) / 256, 256, 0, s>>>(grad2d, g2stride, count, n, n_stride, n_views, accum, seen);
  return hipGetLastError();
}

// ------------------------------------------------------- densification ---
struct Decision {
  bool split, clone, keep;
};

// The grow / split / prune decisions in single precision: the mean gradient
// test as accum >= fl(tau * count), log-scales against log thresholds, and a
// split child's largest log-scale as fl(max s - shrink) (rounding is
// monotonic, so this is the largest of the children's rounded log-scales).
__device__ inline Decision decide(const DensifyArgs& a, int i) {
  const float c = a.grad_count[i];
  const bool grow = c > 0.f && a.grad_accum[i] >= __fmul_rn(a.tau_grad, c);
  const float* s = a.log_scales + 3 * (size_t)i;
  const float smax = fmaxf(fmaxf(s[0], s[1]), s[2]);
  const bool op_ok = !(a.opacity[i] < a.min_opacity);
  Decision d;
  d.split = grow && smax > a.sigma_split;
  if (d.split) {
    d.keep = op_ok && !(__fsub_rn(smax, a.shrink) > a.sigma_prune);
    d.clone = false;
  } else {
    d.keep = op_ok && !(smax > a.sigma_prune);
    d.clone = grow && d.keep;   // a copy has the same opacity and scales
  }
  return d;
}

__global__ void k_densify_count(DensifyArgs a, uint32_t* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Decision d = decide(a, i);
  counts[i] = d.split ? (d.keep ? 2u : 0u) : (uint32_t)d.keep + (uint32_t)d.clone;
}

__device__ inline void write_out(const DensifyArgs& a, int64_t j, int i, int kind, const float m[3], const float s[3],
                                 const float* ph, float phase_sigma, const float* zeta) {
  if (j >= a.capacity) return;
  a.src[j] = i;
  a.kind[j] = kind;
  for (int k = 0; k < 3; ++k) {
    a.means_out[3 * j + k] = m[k];
    a.log_scales_out[3 * j + k] = s[k];
  }
  for (int l = 0; l < a.n_lambda; ++l)
    a.phase_out[(size_t)j * a.n_lambda + l] = zeta ? ph[l] + phase_sigma * zeta[l] : ph[l];
}

__global__ void k_densify_emit(DensifyArgs a, const uint64_t* __restrict__ offsets) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Decision d = decide(a, i);
  if (!d.keep) return;
  const int64_t o = (int64_t)offsets[i];
  const float* mu = a.means + 3 * (size_t)i;
  const float* s = a.log_scales + 3 * (size_t)i;
  const float* ph = a.phase + (size_t)i * a.n_lambda;
  if (!d.split) {
    write_out(a, o, i, 0, mu, s, ph, 0.f, nullptr);
    if (d.clone) write_out(a, o + 1, i, 1, mu, s, ph, a.phase_sigma, a.zeta + (size_t)i * 2 * a.n_lambda);
    return;
  }
  // children: mu + R(q) (exp(s) * xi_c), log-scales s - shrink
  const float* q = a.quats + 4 * (size_t)i;
  const float inv = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
  const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z),       2.f * (x * z + w * y),
                      2.f * (x * y + w * z),       1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                      2.f * (x * z - w * y),       2.f * (y * z + w * x),       1.f - 2.f * (x * x + y * y)};
  const float sc[3] = {expf(s[0]), expf(s[1]), expf(s[2])};
  const float sn[3] = {s[0] - a.shrink, s[1] - a.shrink, s[2] - a.shrink};
  for (int c = 0; c < 2; ++c) {
    const float* xi = a.xi + ((size_t)i * 2 + c) * 3;
    const float e[3] = {sc[0] * xi[0], sc[1] * xi[1], sc[2] * xi[2]};
    const float m[3] = {mu[0] + R[0] * e[0] + R[1] * e[1] + R[2] * e[2],
                        mu[1] + R[3] * e[0] + R[4] * e[1] + R[5] * e[2],
                        mu[2] + R[6] * e[0] + R[7] * e[1] + R[8] * e[2]};
    write_out(a, o + c, i, 2, m, sn, ph, a.phase_sigma, a.zeta + ((size_t)i * 2 + c) * a.n_lambda);
  }
}

hipError_t launch_densify(const DensifyArgs& a, uint32_t* counts, uint64_t* offsets, uint64_t* scan_tmp,
                          uint64_t* total, hipStream_t s) {
  if (a.n <= 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(total), 0u, 2, s);
  const unsigned blocks = (unsigned)((a.n + 255) / 256);
  k_densify_count<<<blocks, 256, 0, s>>>(a, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_u64_from_u32(counts, offsets, a.n, scan_tmp, total, s);
  if (e != hipSuccess) return e;
  k_densify_emit<<<blocks, 256, 0, s>>>(a, offsets);
  return hipGetLastError();
}

// Row j < min(live, capacity) of out is row src[j] of in, or zero for a new
// Gaussian (kind != 0) when zero_new is set.
__global__ void k_gather_rows(const float* __restrict__ in, int64_t row, const int32_t* __restrict__ src,
                              const int32_t* __restrict__ kind, const uint64_t* __restrict__ live, int64_t capacity,
                              int zero_new, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = e / row;
  const uint64_t lv = *live;
  const int64_t n = lv < (uint64_t)capacity ? (int64_t)lv : capacity;
  if (j >= n) return;
  const int64_t c = e - j * row;
  out[e] = (zero_new && kind[j] != 0) ? 0.f : in[(int64_t)src[j] * row + c];
}

hipError_t launch_gather_rows(const float* in, int64_t row, const int32_t* src, const int32_t* kind,
                              const uint64_t* live, int64_t capacity, int zero_new, float* out, hipStream_t s) {
  const int64_t total = capacity * row;
  if (total <= 0) return hipSuccess;
  k_gather_rows<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(in, row, src, kind, live, capacity, zero_new, out);
  return hipGetLastError();
}

}  // namespace chrf
