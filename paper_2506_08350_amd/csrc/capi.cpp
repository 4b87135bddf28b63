// C-ABI layer: contexts, plans, workspace layout and the launch sequences of
// the forward and backward passes.  All GPU work is enqueued on the caller's
// stream; nothing here synchronises except chrf_read_status / timing reports.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/chrf.h"
#include "internal.h"

using namespace chrf;

namespace {

thread_local std::string g_err = "no error";

chrf_status fail(chrf_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(CHRF_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

enum Reg {
  R_V, R_G0, R_G1, R_RECT, R_GKEY, R_GKEY_ALT, R_GVAL, R_GVAL_ALT, R_GCOUNT, R_CNT_SORTED, R_OFFSETS, R_SCAN_TMP,
  R_HIST, R_PKEY, R_PKEY_ALT, R_PVAL, R_PVAL_ALT, R_RANGES, R_STATUS, R_TFINAL, R_LAST, R_FIELD, R_X1, R_Y,
  R_GRAD_FIELD, R_GRAD2D, R_LOSS_PARTIAL,
  R_LAYER_OF, R_LFIELD, R_LTFINAL, R_LSTOP, R_LGRAD,   // layered plans only
  R_UPROP, R_INTEN, R_DMU, R_DEXX, R_DEXY, R_DLDI, R_LOSS2,   // loss_kind 1 only
  R_PO_P, R_PO_V, R_PO_GV, R_PO_D, R_PO_GP, R_PO_PART,       // phase_only plans only
  R_DET_RID, R_DET_INV, R_DET_GRAD,                          // deterministic plans only
  R_TILE_ORDER,
  R_NUM
};

struct TimingRec {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace

struct chrf_ctx {
  int device = 0;
  int lds_per_block = 65536;
  std::map<int, cpx*> twiddles;
  // Device tables and events of destroyed plans.  Freeing device memory is not
  // allowed while any stream of the process is being captured into a graph,
  // and a plan may be destroyed at such a time (a caller dropping a renderer
  // while it captures another one), so plans hand their resources here; they
  // are released by the next chrf_plan_create (which allocates, so it is not
  // called during a capture either) or by chrf_destroy.
  std::vector<void*> retired_mem;
  std::vector<hipEvent_t> retired_events;
  std::mutex mu;
};

struct chrf_plan {
  chrf_ctx* ctx = nullptr;
  chrf_plan_desc d{};
  int B = 0, H = 0, W = 0, L = 0, K = 0, N = 0;
  int pH = 0, pW = 0;
  int tiles_x = 0, tiles_y = 0, n_tiles = 0;
  int64_t cap = 0;
  int cols_per_block = 0;
  int g2 = 0;
  bool deterministic = false;
  bool evanescent = false;
  bool mask_free = false;   // no bin is masked by the band limits (and none is evanescent)
  bool grad2d_zeroed = false;   // the last forward zeroed the 2D gradient rows and no backward has used them
  bool layered = false;
  int loss_kind = 0;
  // loss_kind 1: buffers of the last forward that the backward reads again
  bool paper_ready = false;
  const float2* saved_prop = nullptr;
  const float* saved_inten = nullptr;
  const float* saved_target = nullptr;
  const uint8_t* saved_masks = nullptr;
  int gsort_bits = 0, psort_bits = 0;
  bool gsort_alt = false, psort_alt = false;
  FftDesc frow{}, fcol{};
  HParam* hp_dev = nullptr;
  size_t off[R_NUM] = {}, bytes[R_NUM] = {};
  size_t ws_bytes = 0;
  bool fused_ready = false;
  bool timing = false;
  std::vector<TimingRec> trec;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

template <typename T>
T* at(const chrf_plan* p, void* ws, int r) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + p->off[r]);
}

hipEvent_t take_event(chrf_plan* p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs `launch` and, when timing is on, brackets it with events on stream s.
template <typename F>
chrf_status timed(chrf_plan* p, const char* name, hipStream_t s, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (p->timing) {
    a = take_event(p);
    b = take_event(p);
    if (a && b) (void)hipEventRecord(a, s);
  }
  hipError_t e = launch();
  if (e != hipSuccess) return fail(CHRF_EHIP, std::string(name) + ": " + hipGetErrorString(e));
  if (p->timing && a && b) {
    (void)hipEventRecord(b, s);
    p->trec.push_back({name, a, b});
  }
  return CHRF_OK;
}

#define RUN(name, expr)                                                     \
  do {                                                                      \
    chrf_status st_ = timed(plan, name, s, [&]() -> hipError_t { return (expr); }); \
    if (st_ != CHRF_OK) return st_;                                         \
  } while (0)

int bits_for(int64_t max_key) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) <= max_key) ++b;
  return b;
}

chrf_status get_twiddles(chrf_ctx* ctx, int n, const cpx** out) {
  std::lock_guard<std::mutex> lock(ctx->mu);
  auto it = ctx->twiddles.find(n);
  if (it != ctx->twiddles.end()) {
    *out = it->second;
    return CHRF_OK;
  }
  std::vector<cpx> h(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    h[m] = cpx{(float)std::cos(a), (float)std::sin(a)};
  }
  cpx* d = nullptr;
  HIP_TRY(hipMalloc(&d, sizeof(cpx) * n));
  HIP_TRY(hipMemcpy(d, h.data(), sizeof(cpx) * n, hipMemcpyHostToDevice));
  ctx->twiddles[n] = d;
  *out = d;
  return CHRF_OK;
}

chrf_status make_fft(chrf_ctx* ctx, int n, FftDesc* fd) {
  fd->n = n;
  fd->nstages = fft_plan_radices(n, fd->radix);
  if (fd->nstages == 0 && n != 1) return fail(CHRF_EUNSUPPORTED, "FFT length " + std::to_string(n) + " is not 2^a 3^b 5^c");
  fd->tw_half = nullptr;
  if (n % 2 == 0 && n > 2) {
    const chrf_status st = get_twiddles(ctx, n / 2, &fd->tw_half);
    if (st != CHRF_OK) return st;
  }
  return get_twiddles(ctx, n, &fd->tw);
}

AsmGeom geom(const chrf_plan* p) {
  AsmGeom g{};
  g.H = p->H;
  g.W = p->W;
  g.pH = p->pH;
  g.pW = p->pW;
  g.n_bl = p->B * p->L;
  g.n_lambda = p->L;
  g.K = p->K;
  g.band_mode = p->d.band_limit;
  g.evanescent = p->evanescent ? 1 : 0;
  g.mask_free = p->mask_free ? 1 : 0;
  g.ax = (float)(1.0 / (p->pW * p->d.pitch));
  g.ay = (float)(1.0 / (p->pH * p->d.pitch));
  g.norm = (float)(1.0 / ((double)p->pH * (double)p->pW));
  g.hp = p->hp_dev;
  g.row_plan = p->d.fft_rows_plan;
  g.col_plan = p->d.fft_cols_plan;
  return g;
}

}  // namespace

// ------------------------------------------------------------ no-alloc ---
// chrf_densify_noalloc takes its scratch from this array instead of a caller
// buffer.  Every GPU the library runs on holds its own copy until the process
// ends; host code must never pass the array's name to a kernel (on the host it
// is only a stand-in for the symbol): it uses the per-device address that
// hipGetSymbolAddress returns.
constexpr int64_t kNoallocMaxN = CHRF_NOALLOC_MAX_GAUSSIANS;
constexpr size_t kNoallocBytes = ((sizeof(uint32_t) * kNoallocMaxN + 255) & ~size_t(255)) +
                                 ((sizeof(uint64_t) * kNoallocMaxN + 255) & ~size_t(255)) +
                                 ((sizeof(uint64_t) * ((kNoallocMaxN + kScanTile - 1) / kScanTile + 1 + 16) + 255) &
                                  ~size_t(255));
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
std::mutex g_noalloc_mu;
std::map<int, void*> g_noalloc_ptr;   // device -> address of that device's copy of `scratch`

// Address of `device`'s copy of the array, resolved once per device with that
// device current (the caller's current device is restored).
chrf_status noalloc_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(device);
  if (it != g_noalloc_ptr.end()) {
    *out = it->second;
    return CHRF_OK;
  }
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  HIP_TRY(hipSetDevice(device));
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  HIP_TRY(hipSetDevice(prev));
  if (e != hipSuccess || !ptr)
    return fail(CHRF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_noalloc_ptr[device] = ptr;
  *out = ptr;
  return CHRF_OK;
}
}  // namespace

extern "C" {

const char* chrf_last_error(void) { return g_err.c_str(); }
const char* chrf_version(void) { return "chrf 0.1 gfx950"; }

chrf_status chrf_create(int device, chrf_ctx** out) {
  if (!out) return fail(CHRF_EINVAL, "chrf_create: out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(CHRF_EINVAL, "chrf_create: no such device");
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  chrf_ctx* c = new (std::nothrow) chrf_ctx();
  if (!c) return fail(CHRF_ENOMEM, "chrf_create: out of host memory");
  c->device = device;
  c->lds_per_block = (int)prop.sharedMemPerBlock;
  if (c->lds_per_block > 65536) {
    // Opt in to the full LDS for the FFT passes; if the runtime refuses,
    // clear its sticky error and stay within 64 KiB.
    if (asm_allow_lds(c->lds_per_block - 1024) != hipSuccess) {
      (void)hipGetLastError();
      c->lds_per_block = 65536;
    } else {
      c->lds_per_block -= 1024;
    }
  }
  // resolve this device's copy of the allocation-free entry point's scratch
  // array now, outside any capture the caller may start later
  void* scratch_ptr = nullptr;
  const chrf_status st = noalloc_scratch(device, &scratch_ptr);
  if (st != CHRF_OK) {
    delete c;
    return st;
  }
  *out = c;
  return CHRF_OK;
}

static void release_retired(chrf_ctx* ctx) {
  std::lock_guard<std::mutex> lock(ctx->mu);
  for (void* m : ctx->retired_mem) (void)hipFree(m);
  for (hipEvent_t e : ctx->retired_events) (void)hipEventDestroy(e);
  ctx->retired_mem.clear();
  ctx->retired_events.clear();
}

void chrf_destroy(chrf_ctx* ctx) {
  if (!ctx) return;
  release_retired(ctx);
  for (auto& kv : ctx->twiddles) (void)hipFree(kv.second);
  delete ctx;
}

chrf_status chrf_plan_create(chrf_ctx* ctx, const chrf_plan_desc* desc, chrf_plan** out) {
  if (!ctx || !desc || !out) return fail(CHRF_EINVAL, "chrf_plan_create: NULL argument");
  *out = nullptr;
  const chrf_plan_desc& d = *desc;
  if (d.height <= 0 || d.width <= 0 || d.height > 4096 || d.width > 4096)
    return fail(CHRF_EINVAL, "plan: height and width must be in 1..4096");
  if (d.n_views <= 0 || d.n_views > 256) return fail(CHRF_EINVAL, "plan: n_views must be in 1..256");
  if (d.n_lambda < 1 || d.n_lambda > kMaxLambda) return fail(CHRF_EINVAL, "plan: n_lambda must be in 1..4");
  if (d.n_planes < 1 || d.n_planes > kMaxPlanes) return fail(CHRF_EINVAL, "plan: n_planes must be in 1..64");
  if (d.max_gaussians < 0 || (int64_t)d.max_gaussians * d.n_views >= ((int64_t)1 << 31))
    return fail(CHRF_EINVAL, "plan: n_views * max_gaussians must be below 2^31");
  if (d.pad_factor != 1 && d.pad_factor != 2) return fail(CHRF_EINVAL, "plan: pad_factor must be 1 or 2");
  if (d.band_limit < 0 || d.band_limit > 2) return fail(CHRF_EINVAL, "plan: band_limit must be 0, 1 or 2");
  if (!(d.pitch > 0)) return fail(CHRF_EINVAL, "plan: pitch must be positive");
  for (int l = 0; l < d.n_lambda; ++l)
    if (!(d.wavelengths[l] > 0)) return fail(CHRF_EINVAL, "plan: wavelengths must be positive");
  for (int k = 0; k < d.n_planes; ++k)
    if (!std::isfinite(d.distances[k])) return fail(CHRF_EINVAL, "plan: distances must be finite");
  // alpha_max < 1: the backward recovers T in front of a pair by dividing by 1 - alpha
  if (!(d.k_sigma > 0) || !(d.alpha_max > 0 && d.alpha_max < 1) || !(d.alpha_min >= 0) || !(d.t_min >= 0))
    return fail(CHRF_EINVAL, "plan: thresholds out of range (k_sigma > 0, 0 < alpha_max < 1, alpha_min >= 0, "
                             "t_min >= 0)");
  if (d.layered != 0 && d.layered != 1) return fail(CHRF_EINVAL, "plan: layered must be 0 or 1");
  if (d.loss_kind != 0 && d.loss_kind != 1) return fail(CHRF_EINVAL, "plan: loss_kind must be 0 or 1");
  if (!(d.ssim_weight >= 0) || !std::isfinite(d.ssim_weight)) return fail(CHRF_EINVAL, "plan: ssim_weight must be >= 0");
  if (d.layered && d.n_planes > kMaxLayers) return fail(CHRF_EUNSUPPORTED, "plan: a layered plan takes 1..4 layers");
  if (d.deterministic != 0 && d.deterministic != 1) return fail(CHRF_EINVAL, "plan: deterministic must be 0 or 1");
  if (d.deterministic && d.layered)
    return fail(CHRF_EUNSUPPORTED, "plan: deterministic gradients are available for single-plane plans only");
  int tw = d.tile_w, th = d.tile_h;
  if (tw == 0 && th == 0) tw = th = 16;
  if (tw <= 0 || th <= 0 || tw % 8 || th % 8 || (tw * th != 64 && tw * th != 128 && tw * th != 256))
    return fail(CHRF_EINVAL, "plan: tile_w, tile_h must be multiples of 8 with tile_w * tile_h in {64, 128, 256}");

  release_retired(ctx);
  chrf_plan* p = new (std::nothrow) chrf_plan();
  if (!p) return fail(CHRF_ENOMEM, "plan: out of host memory");
  p->ctx = ctx;
  p->d = d;
  p->d.tile_w = tw;
  p->d.tile_h = th;
  p->B = d.n_views;
  p->H = d.height;
  p->W = d.width;
  p->L = d.n_lambda;
  p->K = d.n_planes;
  p->N = d.max_gaussians;
  p->pH = d.pad_factor * d.height;
  p->pW = d.pad_factor * d.width;
  p->tiles_x = (d.width + tw - 1) / tw;
  p->tiles_y = (d.height + th - 1) / th;
  p->n_tiles = p->tiles_x * p->tiles_y;
  p->layered = d.layered != 0;
  p->deterministic = d.deterministic != 0;
  p->loss_kind = d.loss_kind;
  // per-(view, Gaussian) gradient row: 6 + 2 n_lambda values (+ n_layers), padded
  // to 16 floats (one 64-byte row) or the next multiple of 4
  p->g2 = std::max(16, (6 + 2 * p->L + (p->layered ? p->K : 0) + 3) & ~3);
  int64_t cap = d.max_pairs;
  if (cap <= 0) {
    cap = (int64_t)128 * p->B * (int64_t)(p->N > 0 ? p->N : 1);
    if (cap > ((int64_t)1 << 28)) cap = (int64_t)1 << 28;
  }
  if (cap >= ((int64_t)1 << 32) - 1) {
    delete p;
    return fail(CHRF_EINVAL, "plan: max_pairs must be below 2^32");
  }
  p->cap = cap;
  auto bad = [&](chrf_status st) {
    delete p;
    return st;
  };
  if (p->pW > 8192 || p->pH > 8192) return bad(fail(CHRF_EUNSUPPORTED, "plan: padded size above 8192"));
  chrf_status st = make_fft(ctx, p->pW, &p->frow);
  if (st != CHRF_OK) return bad(st);
  st = make_fft(ctx, p->pH, &p->fcol);
  if (st != CHRF_OK) return bad(st);
  // transfer-function parameters (before the column-pass choice, which
  // depends on whether any bin is evanescent)
  std::vector<HParam> hp(p->L * p->K);
  const double dfx = 1.0 / (p->pW * d.pitch), dfy = 1.0 / (p->pH * d.pitch);
  bool sampling_cut = false;   // some plane's sampling band limit removes a bin
  for (int l = 0; l < p->L; ++l)
    for (int k = 0; k < p->K; ++k) {
      // a layered plan propagates the hologram back to its layers (-Z_k);
      // the recording (+Z_l) is the adjoint of that map
      const double lam = d.wavelengths[l], z = p->layered ? -d.distances[k] : d.distances[k];
      HParam& h = hp[l * p->K + k];
      const double zl = z / lam;
      h.frac_rev = (float)(zl - std::floor(zl));
      h.z = (float)z;
      h.inv_lam = (float)(1.0 / lam);
      h.inv_lam2 = (float)(1.0 / (lam * lam));
      if (d.band_limit >= 2) {
        const double fxl = 1.0 / (lam * std::sqrt((2.0 * dfx * z) * (2.0 * dfx * z) + 1.0));
        const double fyl = 1.0 / (lam * std::sqrt((2.0 * dfy * z) * (2.0 * dfy * z) + 1.0));
        h.kx_max = (int)std::min(std::floor(fxl / dfx), 1e9);
        h.ky_max = (int)std::min(std::floor(fyl / dfy), 1e9);
        if (h.kx_max < p->pW / 2 || h.ky_max < p->pH / 2) sampling_cut = true;   // |signed bin| <= padded size / 2
      } else {
        h.kx_max = h.ky_max = 1 << 30;
      }
      const double e = (double)p->pW * p->pH * d.pitch / lam;
      const double bound = std::floor(e * e);
      h.evan_bound = bound > 9e18 ? (long long)9e18 : (long long)bound;
      h.decay = (float)(2.0 * M_PI * std::fabs(z));
      // the corner bin (pW/2, pH/2) has the largest |f|
      const double hx = (double)(p->pW / 2), hy = (double)(p->pH / 2);
      if (hx * hx * p->pH * (double)p->pH + hy * hy * p->pW * (double)p->pW > (double)h.evan_bound)
        p->evanescent = true;
    }
  p->mask_free = !p->evanescent && !sampling_cut;
  // columns per workgroup in the column passes (two LDS buffers of pH * C)
  if ((int64_t)2 * 8 * p->pW > ctx->lds_per_block)
    return bad(fail(CHRF_EUNSUPPORTED, "plan: a padded row does not fit the LDS"));
  int C = d.cols_per_block;
  if (tuned_cols(geom(p)) && p->pH == 4320) {
    // tuned column pass of 4320 (two transforms of 2160): one or two columns per workgroup
    if (C != 0 && C != 1 && C != 2)
      return bad(fail(CHRF_EUNSUPPORTED, "plan: cols_per_block must be 1 or 2 for a padded height of 4320"));
    if (C == 0) C = 2;
  } else if (tuned_cols(geom(p))) {
    // tuned column pass: 2 columns x 512 threads (default), 1 x 256 or 4 x 1024
    if (C != 0 && C != 1 && C != 2 && C != 4)
      return bad(fail(CHRF_EUNSUPPORTED, "plan: cols_per_block must be 1, 2 or 4 for this padded height"));
    if (C == 0) C = 2;
  } else {
    if (C == 0) {
      const int lds_cap = ctx->lds_per_block < 81920 ? ctx->lds_per_block : 81920;
      C = 16;
      while (C > 1 && ((int64_t)col_lds_bytes(p->pH, C) > lds_cap || p->pH * C > fft_max_elems() || p->pW % C))
        C >>= 1;
    }
    if (C < 1 || (C & (C - 1)) || p->pW % C || (int64_t)col_lds_bytes(p->pH, C) > ctx->lds_per_block ||
        p->pH * C > fft_max_elems())
      return bad(fail(CHRF_EUNSUPPORTED, "plan: cols_per_block does not fit the LDS or the padded width"));
  }
  p->cols_per_block = C;
  // radix schedules of the tuned transforms
  if (d.fft_rows_plan != 0 && (!tuned_rows(geom(p)) || d.fft_rows_plan < 0 ||
                               d.fft_rows_plan >= tuned_row_plans(geom(p))))
    return bad(fail(CHRF_EUNSUPPORTED, "plan: fft_rows_plan must be 0 unless the padded width is 3840 or 7680 (then "
                                       "0.." + std::to_string(tuned_row_plans(geom(p)) - 1) + ")"));
  if (d.fft_cols_plan != 0 && (!tuned_cols(geom(p)) || !tuned_col_plan_fits(geom(p), C) || d.fft_cols_plan < 0 ||
                               d.fft_cols_plan >= tuned_col_plans(geom(p))))
    return bad(fail(CHRF_EUNSUPPORTED, "plan: fft_cols_plan must be 0 unless the padded height is 2160 with two "
                                       "columns per workgroup, or 4320 (then 0..3)"));
  {
    hipError_t e = hipMalloc(&p->hp_dev, sizeof(HParam) * hp.size());
    if (e == hipSuccess) e = hipMemcpy(p->hp_dev, hp.data(), sizeof(HParam) * hp.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bad(fail(CHRF_EHIP, std::string("plan: ") + hipGetErrorString(e)));
  }
  // sort geometry
  p->gsort_bits = 32 + bits_for(p->B - 1);
  // pair keys are view << psort_bits | tile; the sort orders their low bits
  p->psort_bits = bits_for((int64_t)p->n_tiles - 1);
  p->gsort_alt = ((p->gsort_bits + 7) / 8) % 2 == 1;
  p->psort_alt = ((p->psort_bits + 7) / 8) % 2 == 1;
  // workspace layout
  const int64_t BN = (int64_t)p->B * (p->N > 0 ? p->N : 1);
  const int64_t hist = std::max(radix_hist_elems(cap), radix_hist_elems(BN));   // both sorts share it
  const int64_t scan_tmp = scan_tmp_elems(std::max<int64_t>(hist, BN)) + 16;
  const int64_t pix = (int64_t)p->B * p->H * p->W;
  size_t sz[R_NUM];
  sz[R_V] = sizeof(float2) * (size_t)std::max(p->N, 1) * p->L;
  sz[R_G0] = sizeof(float4) * BN;
  sz[R_G1] = sizeof(float4) * BN;
  sz[R_RECT] = sizeof(int4) * BN;
  sz[R_GKEY] = sz[R_GKEY_ALT] = sizeof(uint64_t) * BN;
  sz[R_GVAL] = sz[R_GVAL_ALT] = sizeof(uint32_t) * BN;
  sz[R_GCOUNT] = sz[R_CNT_SORTED] = sizeof(uint32_t) * BN;
  sz[R_OFFSETS] = sizeof(uint64_t) * BN;
  sz[R_SCAN_TMP] = sizeof(uint64_t) * scan_tmp;
  sz[R_HIST] = sizeof(uint32_t) * hist;
  sz[R_PKEY] = sz[R_PKEY_ALT] = sz[R_PVAL] = sz[R_PVAL_ALT] = sizeof(uint32_t) * cap;
  sz[R_RANGES] = sizeof(uint2) * (size_t)p->B * p->n_tiles;
  sz[R_TILE_ORDER] = sizeof(uint32_t) * (size_t)p->B * p->n_tiles;
  sz[R_STATUS] = 256;
  sz[R_TFINAL] = sizeof(float) * pix;
  sz[R_LAST] = sizeof(uint32_t) * pix;
  sz[R_FIELD] = sizeof(float2) * pix * p->L;
  sz[R_X1] = sizeof(float2) * (size_t)p->B * p->L * p->H * p->pW;
  sz[R_Y] = sizeof(float2) * (size_t)p->B * p->L * p->K * p->H * p->pW;
  sz[R_GRAD_FIELD] = sizeof(float2) * pix * p->L;
  sz[R_GRAD2D] = sizeof(float) * BN * p->g2;
  sz[R_LOSS_PARTIAL] = sizeof(float) * (size_t)p->B * p->L * p->K * p->H;
  const size_t lpix = p->layered ? (size_t)pix * p->K : 0;
  sz[R_LAYER_OF] = p->layered ? (size_t)std::max(p->N, 1) : 0;
  sz[R_LFIELD] = sz[R_LGRAD] = sizeof(float2) * lpix * p->L;
  sz[R_LTFINAL] = sizeof(float) * lpix;
  sz[R_LSTOP] = sizeof(uint32_t) * lpix;
  const size_t ipix = p->loss_kind == 1 ? (size_t)pix * p->L * p->K : 0;
  sz[R_UPROP] = sizeof(float2) * ipix;
  sz[R_INTEN] = sz[R_DMU] = sz[R_DEXX] = sz[R_DEXY] = sz[R_DLDI] = sizeof(float) * ipix;
  sz[R_LOSS2] = p->loss_kind == 1 ? sizeof(float) * (size_t)loss_partial_elems(p->B * p->L * p->K, p->H, p->W) : 0;
  const bool po = d.phase_only != 0;
  const size_t fpix = po ? (size_t)pix * p->L : 0;         // hologram elements
  sz[R_PO_P] = sz[R_PO_GP] = sizeof(float2) * fpix;
  sz[R_PO_V] = sz[R_PO_GV] = sizeof(float2) * fpix * p->K;
  sz[R_PO_D] = sizeof(float) * fpix * p->K * 6;             // 3 SSIM derivative maps x (re, im)
  sz[R_PO_PART] = po ? sizeof(float) * (size_t)loss_partial_elems(2 * p->B * p->L * p->K, p->H, p->W) : 0;
  sz[R_DET_RID] = sz[R_DET_INV] = p->deterministic ? sizeof(uint32_t) * cap : 0;
  sz[R_DET_GRAD] = p->deterministic ? sizeof(float) * cap * p->g2 : 0;
  size_t o = 0;
  for (int r = 0; r < R_NUM; ++r) {
    p->off[r] = o;
    p->bytes[r] = sz[r];
    o += align256(sz[r]);
  }
  p->ws_bytes = o;
  *out = p;
  return CHRF_OK;
}

// Frees nothing on the device itself (see chrf_ctx::retired_mem), so a plan
// may be destroyed while another stream is being captured.
void chrf_plan_destroy(chrf_plan* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lock(p->ctx->mu);
    if (p->hp_dev) p->ctx->retired_mem.push_back(p->hp_dev);
    for (auto& r : p->trec) {
      p->ctx->retired_events.push_back(r.a);
      p->ctx->retired_events.push_back(r.b);
    }
    for (auto e : p->ev_pool) p->ctx->retired_events.push_back(e);
  }
  delete p;
}

size_t chrf_plan_workspace_bytes(const chrf_plan* p) { return p ? p->ws_bytes : 0; }

chrf_status chrf_plan_region(const chrf_plan* p, int region, size_t* offset, size_t* bytes) {
  if (!p || !offset || !bytes) return fail(CHRF_EINVAL, "chrf_plan_region: NULL argument");
  int r;
  switch (region) {
    case CHRF_REGION_PAIR_KEYS: r = p->psort_alt ? R_PKEY_ALT : R_PKEY; break;
    case CHRF_REGION_PAIR_VALUES: r = p->psort_alt ? R_PVAL_ALT : R_PVAL; break;
    case CHRF_REGION_TILE_RANGES: r = R_RANGES; break;
    case CHRF_REGION_STATUS: r = R_STATUS; break;
    case CHRF_REGION_T_FINAL: r = R_TFINAL; break;
    case CHRF_REGION_LAST: r = R_LAST; break;
    case CHRF_REGION_FIELD: r = R_FIELD; break;
    case CHRF_REGION_GRAD_FIELD: r = R_GRAD_FIELD; break;
    case CHRF_REGION_LAYER_FIELDS: r = R_LFIELD; break;
    case CHRF_REGION_LAYER_T_FINAL: r = R_LTFINAL; break;
    case CHRF_REGION_LAYER_STOP: r = R_LSTOP; break;
    case CHRF_REGION_LAYER_GRAD: r = R_LGRAD; break;
    case CHRF_REGION_LOSS_PARTIAL: r = R_LOSS_PARTIAL; break;
    default: return fail(CHRF_EINVAL, "chrf_plan_region: unknown region");
  }
  *offset = p->off[r];
  *bytes = p->bytes[r];
  return CHRF_OK;
}

static chrf_status check_gaussians(const chrf_plan* p, const chrf_gaussians* g) {
  if (!g) return fail(CHRF_EINVAL, "gaussians is NULL");
  if (g->n < 0 || g->n > p->N) return fail(CHRF_EINVAL, "gaussians: n exceeds the plan's max_gaussians");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity || !g->amp || !g->phase))
    return fail(CHRF_EINVAL, "gaussians: NULL array");
  if (p->layered && g->n > 0 && !g->logits) return fail(CHRF_EINVAL, "gaussians: a layered plan needs logits");
  return CHRF_OK;
}

static chrf_status asm_forward(chrf_plan* plan, const float2* field, void* ws, float* prop_out, float* intensity_out,
                               const float* target, hipStream_t s) {
  const AsmGeom g = geom(plan);
  float2* x1 = at<float2>(plan, ws, R_X1);
  float2* y = at<float2>(plan, ws, R_Y);
  RUN("rows_forward", launch_rows_forward(field, x1, g, plan->frow, s));
  RUN("cols_forward", launch_cols_forward(x1, y, g, plan->fcol, plan->cols_per_block, s));
  const double numel = (double)plan->B * plan->L * plan->K * plan->H * plan->W;
  RUN("rows_inverse", launch_rows_inverse(y, g, plan->frow, reinterpret_cast<float2*>(prop_out), intensity_out,
                                          target, at<float>(plan, ws, R_LOSS_PARTIAL), (float)(2.0 / numel),
                                          target != nullptr, s));
  return CHRF_OK;
}

chrf_status chrf_forward(chrf_plan* plan, const chrf_gaussians* g, const chrf_camera* cams, void* ws,
                         float* field_out, float* prop_out, float* intensity_out, const float* target,
                         const uint8_t* masks, float* loss_out, void* hip_stream) {
  if (!plan || !cams || !ws) return fail(CHRF_EINVAL, "chrf_forward: NULL plan, cameras or workspace");
  chrf_status st = check_gaussians(plan, g);
  if (st != CHRF_OK) return st;
  if (target && !loss_out) return fail(CHRF_EINVAL, "chrf_forward: target needs loss_out");
  hipStream_t s = (hipStream_t)hip_stream;
  plan->fused_ready = false;
  plan->paper_ready = false;
  const int Nst = std::max(plan->N, 1);
  const int64_t BN = (int64_t)plan->B * Nst;
  float2* field = field_out ? reinterpret_cast<float2*>(field_out) : at<float2>(plan, ws, R_FIELD);
  uint32_t* status = at<uint32_t>(plan, ws, R_STATUS);
  uint64_t* total = reinterpret_cast<uint64_t*>(status);

  uint2* ranges = at<uint2>(plan, ws, R_RANGES);
  float* grad2d = at<float>(plan, ws, R_GRAD2D);
  ProjArgs pa{};
  pa.means = g->means;
  pa.log_scales = g->log_scales;
  pa.quats = g->quats;
  pa.opacity = g->opacity;
  pa.cams = reinterpret_cast<const Cam*>(cams);
  pa.n = g->n;
  pa.n_stride = Nst;
  pa.n_views = plan->B;
  pa.width = plan->W;
  pa.height = plan->H;
  pa.tile_w = plan->d.tile_w;
  pa.tile_h = plan->d.tile_h;
  pa.tiles_x = plan->tiles_x;
  pa.tiles_y = plan->tiles_y;
  pa.k_sigma = plan->d.k_sigma;
  pa.alpha_min = plan->d.alpha_min;
  pa.rec_g0 = at<float4>(plan, ws, R_G0);
  pa.rec_g1 = at<float4>(plan, ws, R_G1);
  pa.rec_rect = at<int4>(plan, ws, R_RECT);
  pa.sort_key = at<uint64_t>(plan, ws, R_GKEY);
  pa.sort_val = at<uint32_t>(plan, ws, R_GVAL);
  pa.count = at<uint32_t>(plan, ws, R_GCOUNT);
  // a training forward (a target is given) also zeroes the 2D gradient rows
  // that the backward accumulates into, which spares the backward a clear
  pa.grad2d = target ? grad2d : nullptr;
  pa.grad2d_stride = plan->g2;
  pa.amp = g->amp;
  pa.phase = g->phase;
  pa.v = at<float2>(plan, ws, R_V);
  pa.n_lambda = plan->L;
  pa.clear_a = status;
  pa.n_clear_a = 8;
  pa.clear_b = reinterpret_cast<uint32_t*>(ranges);
  pa.n_clear_b = (int64_t)2 * plan->B * plan->n_tiles;
  RUN("project", launch_project(pa, s));
  plan->grad2d_zeroed = target != nullptr;

  bool galt = false;
  RUN("sort_gaussians", radix_sort_u64(at<uint64_t>(plan, ws, R_GKEY), at<uint64_t>(plan, ws, R_GKEY_ALT),
                                       at<uint32_t>(plan, ws, R_GVAL), at<uint32_t>(plan, ws, R_GVAL_ALT), BN,
                                       nullptr, 0, plan->gsort_bits, at<uint32_t>(plan, ws, R_HIST),
                                       at<uint32_t>(plan, ws, R_SCAN_TMP), status + 3, &galt, s));
  const uint32_t* gval = at<uint32_t>(plan, ws, galt ? R_GVAL_ALT : R_GVAL);
  RUN("count_pairs", launch_count_pairs(gval, at<uint32_t>(plan, ws, R_GCOUNT), at<float4>(plan, ws, R_G0),
                                        at<float4>(plan, ws, R_G1), at<int4>(plan, ws, R_RECT), BN, plan->d.tile_w,
                                        plan->d.tile_h, at<uint32_t>(plan, ws, R_CNT_SORTED), s));
  RUN("scan_counts", launch_scan_u64_from_u32(at<uint32_t>(plan, ws, R_CNT_SORTED), at<uint64_t>(plan, ws, R_OFFSETS),
                                              BN, at<uint64_t>(plan, ws, R_SCAN_TMP), total, s));
  RUN("emit_pairs", launch_emit_pairs(gval, at<uint64_t>(plan, ws, R_OFFSETS), at<uint32_t>(plan, ws, R_CNT_SORTED),
                                      at<float4>(plan, ws, R_G0), at<float4>(plan, ws, R_G1),
                                      at<int4>(plan, ws, R_RECT), BN, Nst, plan->d.tile_w, plan->d.tile_h,
                                      plan->tiles_x, plan->psort_bits, at<uint32_t>(plan, ws, R_PKEY),
                                      at<uint32_t>(plan, ws, R_PVAL), plan->cap, total, status + 2,
                                      plan->deterministic ? at<uint32_t>(plan, ws, R_DET_RID) : nullptr, s));
  bool palt = false;
  RUN("sort_pairs", radix_sort_u32(at<uint32_t>(plan, ws, R_PKEY), at<uint32_t>(plan, ws, R_PKEY_ALT),
                                   at<uint32_t>(plan, ws, R_PVAL), at<uint32_t>(plan, ws, R_PVAL_ALT), plan->cap,
                                   total, 0, plan->psort_bits, at<uint32_t>(plan, ws, R_HIST),
                                   at<uint32_t>(plan, ws, R_SCAN_TMP), status + 3, &palt, s));
  const uint32_t* pkey = at<uint32_t>(plan, ws, palt ? R_PKEY_ALT : R_PKEY);
  const uint32_t* pval = at<uint32_t>(plan, ws, palt ? R_PVAL_ALT : R_PVAL);
  if (plan->deterministic)   // the sorted values (emission slots) become record ids
    RUN("det_gather", launch_det_gather(const_cast<uint32_t*>(pval), at<uint32_t>(plan, ws, R_DET_RID),
                                        at<uint32_t>(plan, ws, R_DET_INV), total, plan->cap, s));
  RUN("tile_ranges", launch_tile_ranges(pkey, plan->psort_bits, plan->n_tiles, total, plan->cap, ranges, s));
  RUN("tile_order", launch_tile_order(ranges, plan->B * plan->n_tiles, at<uint32_t>(plan, ws, R_TILE_ORDER), s));

  RasterArgs ra{};
  ra.rec_g0 = at<float4>(plan, ws, R_G0);
  ra.rec_g1 = at<float4>(plan, ws, R_G1);
  ra.rec_rect = at<int4>(plan, ws, R_RECT);
  ra.v = at<float2>(plan, ws, R_V);
  ra.pair_val = pval;
  ra.ranges = ranges;
  ra.tile_order = at<uint32_t>(plan, ws, R_TILE_ORDER);
  ra.n_stride = Nst;
  ra.n_lambda = plan->L;
  ra.width = plan->W;
  ra.height = plan->H;
  ra.tile_w = plan->d.tile_w;
  ra.tile_h = plan->d.tile_h;
  ra.tiles_x = plan->tiles_x;
  ra.tiles_y = plan->tiles_y;
  ra.n_views = plan->B;
  ra.k_sigma = plan->d.k_sigma;
  ra.alpha_min = plan->d.alpha_min;
  ra.alpha_max = plan->d.alpha_max;
  ra.t_min = plan->d.t_min;
  ra.last = at<uint32_t>(plan, ws, R_LAST);
  if (plan->layered) {
    const AsmGeom geo = geom(plan);
    uint8_t* layer_of = at<uint8_t>(plan, ws, R_LAYER_OF);
    float2* lfield = at<float2>(plan, ws, R_LFIELD);
    RUN("assign_layers", launch_assign_layers(g->logits, g->n, plan->K, kSteTau, layer_of, s));
    ra.layer_of = layer_of;
    ra.n_layers = plan->K;
    ra.layer_stop = at<uint32_t>(plan, ws, R_LSTOP);
    ra.field = lfield;
    ra.t_final = at<float>(plan, ws, R_LTFINAL);
    RUN("raster_layers_forward", launch_raster_layers_forward(ra, s));
    // forward recording P = sum_l ASM(U_l; +Z_l): the adjoint of the inverse
    // propagation the plan's transfer functions describe
    float2* y = at<float2>(plan, ws, R_Y);
    float2* x1 = at<float2>(plan, ws, R_X1);
    RUN("record_rows_in", launch_rows_adjoint_in(nullptr, nullptr, lfield, y, geo, plan->frow, s));
    RUN("record_cols", launch_cols_adjoint(y, x1, geo, plan->fcol, plan->cols_per_block, s));
    RUN("record_rows_out", launch_rows_adjoint_out(x1, nullptr, field, geo, plan->frow, s));
  } else {
    ra.field = field;
    ra.t_final = at<float>(plan, ws, R_TFINAL);
    RUN("raster_forward", launch_raster_forward(ra, s));
  }

  if (target && plan->loss_kind == 1) {
    // unfused: keep u and I for the loss and its backward
    float2* u = prop_out ? reinterpret_cast<float2*>(prop_out) : at<float2>(plan, ws, R_UPROP);
    float* I = intensity_out ? intensity_out : at<float>(plan, ws, R_INTEN);
    st = asm_forward(plan, field, ws, reinterpret_cast<float*>(u), I, nullptr, s);
    if (st != CHRF_OK) return st;
    const int n_img = plan->B * plan->L * plan->K;
    RUN("loss_forward", launch_paper_loss_forward(I, target, masks, n_img, plan->L * plan->K, plan->K, plan->H,
                                                  plan->W, plan->d.ssim_weight, at<float>(plan, ws, R_DMU),
                                                  at<float>(plan, ws, R_DEXX), at<float>(plan, ws, R_DEXY),
                                                  at<float>(plan, ws, R_LOSS2), loss_out, s));
    plan->paper_ready = true;
    plan->saved_prop = u;
    plan->saved_inten = I;
    plan->saved_target = target;
    plan->saved_masks = masks;
    return CHRF_OK;
  }
  st = asm_forward(plan, field, ws, prop_out, intensity_out, target, s);
  if (st != CHRF_OK) return st;
  if (target) {
    const double numel = (double)plan->B * plan->L * plan->K * plan->H * plan->W;
    RUN("reduce_loss", launch_reduce_loss(at<float>(plan, ws, R_LOSS_PARTIAL), (int64_t)plan->B * plan->L * plan->K * plan->H,
                                          (float)(1.0 / numel), loss_out, s));
    plan->fused_ready = true;
  }
  return CHRF_OK;
}

chrf_status chrf_backward(chrf_plan* plan, const chrf_gaussians* g, const chrf_camera* cams, void* ws,
                          const float* dL_dI, const float* prop, const float* dL_dprop, const float* dL_dfield,
                          const float* grad_scale, const chrf_grads* out, void* hip_stream) {
  if (!plan || !cams || !ws || !out) return fail(CHRF_EINVAL, "chrf_backward: NULL plan, cameras, workspace or grads");
  chrf_status st = check_gaussians(plan, g);
  if (st != CHRF_OK) return st;
  if (g->n > 0 && (!out->means || !out->log_scales || !out->quats || !out->opacity || !out->amp || !out->phase))
    return fail(CHRF_EINVAL, "chrf_backward: NULL gradient array");
  if (dL_dI && !prop) return fail(CHRF_EINVAL, "chrf_backward: dL_dI needs the saved prop");
  hipStream_t s = (hipStream_t)hip_stream;
  const int Nst = std::max(plan->N, 1);
  const AsmGeom geo = geom(plan);
  float2* y = at<float2>(plan, ws, R_Y);
  float2* x1 = at<float2>(plan, ws, R_X1);
  if (!dL_dI && !dL_dprop && plan->paper_ready) {
    // gradient of the paper's loss w.r.t. the intensities of the last forward
    float* dldi = at<float>(plan, ws, R_DLDI);
    RUN("loss_backward", launch_paper_loss_backward(plan->saved_inten, plan->saved_target, plan->saved_masks,
                                                    plan->B * plan->L * plan->K, plan->L * plan->K, plan->K,
                                                    plan->H, plan->W, plan->d.ssim_weight,
                                                    at<float>(plan, ws, R_DMU), at<float>(plan, ws, R_DEXX),
                                                    at<float>(plan, ws, R_DEXY), nullptr, dldi, s));
    dL_dI = dldi;
    prop = reinterpret_cast<const float*>(plan->saved_prop);
  }
  const bool have_prop_grad = dL_dI || dL_dprop;
  if (!have_prop_grad && !plan->fused_ready && !dL_dfield)
    return fail(CHRF_EINVAL, "chrf_backward: no incoming gradient (no dL_dI/dL_dprop/dL_dfield and no fused loss)");
  const float2* grad_field = reinterpret_cast<const float2*>(dL_dfield);
  if (have_prop_grad || plan->fused_ready) {
    if (have_prop_grad)  // (the fused spectra of an MSE forward are used only when no gradient is passed)
      RUN("rows_adjoint_in", launch_rows_adjoint_in(reinterpret_cast<const float2*>(prop), dL_dI,
                                                    reinterpret_cast<const float2*>(dL_dprop), y, geo, plan->frow, s));
    RUN("cols_adjoint", launch_cols_adjoint(y, x1, geo, plan->fcol, plan->cols_per_block, s));
    float2* gf = at<float2>(plan, ws, R_GRAD_FIELD);
    RUN("rows_adjoint_out", launch_rows_adjoint_out(x1, reinterpret_cast<const float2*>(dL_dfield), gf, geo,
                                                    plan->frow, s));
    grad_field = gf;
  }
  if (plan->layered) {
    // dL/dU_l = ASM(dL/dP; -Z_l): the adjoint of the recording
    const double numel = (double)plan->B * plan->L * plan->K * plan->H * plan->W;
    float2* lgrad = at<float2>(plan, ws, R_LGRAD);
    RUN("layer_grad_rows", launch_rows_forward(grad_field, x1, geo, plan->frow, s));
    RUN("layer_grad_cols", launch_cols_forward(x1, y, geo, plan->fcol, plan->cols_per_block, s));
    RUN("layer_grad_rows_inv", launch_rows_inverse(y, geo, plan->frow, lgrad, nullptr, nullptr,
                                                   at<float>(plan, ws, R_LOSS_PARTIAL), (float)(2.0 / numel),
                                                   false, s));
    plan->fused_ready = false;   // Y now holds the layer gradients' spectra
    grad_field = lgrad;
  }
  float* grad2d = at<float>(plan, ws, R_GRAD2D);
  if (!plan->grad2d_zeroed) RUN("grad2d_clear", launch_fill_f32(grad2d, 0.f, (int64_t)plan->B * Nst * plan->g2, s));
  plan->grad2d_zeroed = false;   // this backward accumulates into the rows
  size_t o, b;
  chrf_plan_region(plan, CHRF_REGION_PAIR_VALUES, &o, &b);
  RasterArgs ra{};
  ra.rec_g0 = at<float4>(plan, ws, R_G0);
  ra.rec_g1 = at<float4>(plan, ws, R_G1);
  ra.rec_rect = at<int4>(plan, ws, R_RECT);
  ra.v = at<float2>(plan, ws, R_V);
  ra.pair_val = reinterpret_cast<const uint32_t*>(static_cast<char*>(ws) + o);
  ra.ranges = at<uint2>(plan, ws, R_RANGES);
  ra.tile_order = at<uint32_t>(plan, ws, R_TILE_ORDER);
  ra.n_stride = Nst;
  ra.n_lambda = plan->L;
  ra.width = plan->W;
  ra.height = plan->H;
  ra.tile_w = plan->d.tile_w;
  ra.tile_h = plan->d.tile_h;
  ra.tiles_x = plan->tiles_x;
  ra.tiles_y = plan->tiles_y;
  ra.n_views = plan->B;
  ra.k_sigma = plan->d.k_sigma;
  ra.alpha_min = plan->d.alpha_min;
  ra.alpha_max = plan->d.alpha_max;
  ra.t_min = plan->d.t_min;
  ra.t_final = at<float>(plan, ws, R_TFINAL);
  ra.last = at<uint32_t>(plan, ws, R_LAST);
  ra.grad_field = grad_field;
  ra.grad_scale = grad_scale;
  ra.grad2d = grad2d;
  ra.g2stride = plan->g2;
  float* pair_grad = plan->deterministic ? at<float>(plan, ws, R_DET_GRAD) : nullptr;
  if (pair_grad) {
    RUN("pair_grad_clear", launch_fill_f32(pair_grad, 0.f, plan->cap * plan->g2, s));
    ra.pair_grad = pair_grad;
  }
  if (plan->layered) {
    ra.layer_of = at<uint8_t>(plan, ws, R_LAYER_OF);
    ra.n_layers = plan->K;
    ra.layer_stop = at<uint32_t>(plan, ws, R_LSTOP);
    ra.t_final = at<float>(plan, ws, R_LTFINAL);
    RUN("raster_layers_backward", launch_raster_layers_backward(ra, s));
  } else {
    RUN("raster_backward", launch_raster_backward(ra, s));
  }
  if (pair_grad)
    RUN("det_reduce", launch_det_reduce(at<uint32_t>(plan, ws, plan->gsort_alt ? R_GVAL_ALT : R_GVAL),
                                        at<uint64_t>(plan, ws, R_OFFSETS), at<uint32_t>(plan, ws, R_CNT_SORTED),
                                        at<uint32_t>(plan, ws, R_DET_INV), pair_grad, (int64_t)plan->B * Nst,
                                        plan->g2, plan->cap, grad2d, s));
  RUN("project_backward",
      launch_project_backward(g->means, g->log_scales, g->quats, g->amp, g->phase, reinterpret_cast<const Cam*>(cams),
                              g->n, Nst, plan->B, plan->L, at<uint32_t>(plan, ws, R_GCOUNT), grad2d, plan->g2,
                              out->means, out->log_scales, out->quats, out->opacity, out->amp, out->phase, s));
  if (plan->layered && out->logits)
    RUN("logits_backward", launch_logits_backward(g->logits, grad2d, plan->g2, 6 + 2 * plan->L,
                                                  at<uint32_t>(plan, ws, R_GCOUNT), g->n, Nst, plan->B, plan->K,
                                                  kSteTau, out->logits, s));
  return CHRF_OK;
}

chrf_status chrf_propagate(chrf_plan* plan, const float* field, void* ws, float* prop_out, float* intensity_out,
                           void* hip_stream) {
  if (!plan || !field || !ws) return fail(CHRF_EINVAL, "chrf_propagate: NULL argument");
  plan->fused_ready = false;
  plan->paper_ready = false;
  return asm_forward(plan, reinterpret_cast<const float2*>(field), ws, prop_out, intensity_out, nullptr,
                     (hipStream_t)hip_stream);
}

chrf_status chrf_propagate_adjoint(chrf_plan* plan, const float* grad_prop, void* ws, float* grad_field,
                                   void* hip_stream) {
  if (!plan || !grad_prop || !ws || !grad_field) return fail(CHRF_EINVAL, "chrf_propagate_adjoint: NULL argument");
  hipStream_t s = (hipStream_t)hip_stream;
  const AsmGeom geo = geom(plan);
  float2* y = at<float2>(plan, ws, R_Y);
  float2* x1 = at<float2>(plan, ws, R_X1);
  RUN("rows_adjoint_in", launch_rows_adjoint_in(nullptr, nullptr, reinterpret_cast<const float2*>(grad_prop), y, geo,
                                                plan->frow, s));
  RUN("cols_adjoint", launch_cols_adjoint(y, x1, geo, plan->fcol, plan->cols_per_block, s));
  RUN("rows_adjoint_out", launch_rows_adjoint_out(x1, nullptr, reinterpret_cast<float2*>(grad_field), geo,
                                                  plan->frow, s));
  return CHRF_OK;
}

chrf_status chrf_phase_only_step(chrf_plan* plan, const float* targets, const float* phi, void* ws, float* loss_out,
                                 float* dphi, void* hip_stream) {
  if (!plan || !targets || !phi || !ws || !loss_out || !dphi)
    return fail(CHRF_EINVAL, "chrf_phase_only_step: NULL argument");
  if (!plan->d.phase_only) return fail(CHRF_EINVAL, "chrf_phase_only_step: plan was not created with phase_only");
  hipStream_t s = (hipStream_t)hip_stream;
  plan->fused_ready = false;
  plan->paper_ready = false;
  const AsmGeom geo = geom(plan);
  const int64_t n = (int64_t)plan->B * plan->L * plan->H * plan->W;
  const int n_img = plan->B * plan->L * plan->K;
  float2* P = at<float2>(plan, ws, R_PO_P);
  float2* V = at<float2>(plan, ws, R_PO_V);
  float2* GV = at<float2>(plan, ws, R_PO_GV);
  float2* GP = at<float2>(plan, ws, R_PO_GP);
  const float2* U = reinterpret_cast<const float2*>(targets);
  RUN("phase_field", launch_phase_field(phi, n, P, s));
  chrf_status st = asm_forward(plan, P, ws, reinterpret_cast<float*>(V), nullptr, nullptr, s);
  if (st != CHRF_OK) return st;
  RUN("field_loss_forward", launch_field_loss_forward(V, U, n_img, plan->H, plan->W, plan->d.ssim_weight,
                                                      at<float>(plan, ws, R_PO_D), at<float>(plan, ws, R_PO_PART),
                                                      loss_out, s));
  RUN("field_loss_backward", launch_field_loss_backward(V, U, n_img, plan->H, plan->W, plan->d.ssim_weight,
                                                        at<float>(plan, ws, R_PO_D), GV, s));
  float2* y = at<float2>(plan, ws, R_Y);
  float2* x1 = at<float2>(plan, ws, R_X1);
  RUN("rows_adjoint_in", launch_rows_adjoint_in(nullptr, nullptr, GV, y, geo, plan->frow, s));
  RUN("cols_adjoint", launch_cols_adjoint(y, x1, geo, plan->fcol, plan->cols_per_block, s));
  RUN("rows_adjoint_out", launch_rows_adjoint_out(x1, nullptr, GP, geo, plan->frow, s));
  RUN("phase_grad", launch_phase_grad(GP, phi, n, dphi, s));
  return CHRF_OK;
}

chrf_status chrf_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                           float beta2, float eps, int32_t step, void* hip_stream) {
  if (n < 0 || (n > 0 && (!param || !grad || !m || !v))) return fail(CHRF_EINVAL, "chrf_adam_step: bad argument");
  if (step < 1 || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(CHRF_EINVAL, "chrf_adam_step: step must be >= 1, betas in [0, 1), eps > 0");
  HIP_TRY(launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, step, (hipStream_t)hip_stream));
  return CHRF_OK;
}

chrf_status chrf_adan_step(float* param, const float* grad, float* grad_prev, float* m, float* v, float* nm,
                           int64_t n, float lr, float beta1, float beta2, float beta3, float eps, float weight_decay,
                           int32_t step, void* hip_stream) {
  if (n < 0 || (n > 0 && (!param || !grad || !grad_prev || !m || !v || !nm)))
    return fail(CHRF_EINVAL, "chrf_adan_step: bad argument");
  const bool betas_ok = beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && beta3 >= 0 && beta3 < 1;
  if (step < 1 || !betas_ok || !(eps > 0) || !(weight_decay >= 0))
    return fail(CHRF_EINVAL, "chrf_adan_step: step must be >= 1, betas in [0, 1), eps > 0, weight_decay >= 0");
  HIP_TRY(launch_adan(param, grad, grad_prev, m, v, nm, n, lr, beta1, beta2, beta3, eps, weight_decay, step,
                      (hipStream_t)hip_stream));
  return CHRF_OK;
}

chrf_status chrf_densify_stats(chrf_plan* plan, void* ws, int32_t n, float* grad_accum, float* grad_count,
                               void* hip_stream) {
  if (!plan || !ws || (n > 0 && (!grad_accum || !grad_count))) return fail(CHRF_EINVAL, "chrf_densify_stats: NULL argument");
  if (n < 0 || n > plan->N) return fail(CHRF_EINVAL, "chrf_densify_stats: n exceeds the plan's max_gaussians");
  HIP_TRY(launch_densify_stats(at<float>(plan, ws, R_GRAD2D), plan->g2, at<uint32_t>(plan, ws, R_GCOUNT), n,
                               std::max(plan->N, 1), plan->B, grad_accum, grad_count, (hipStream_t)hip_stream));
  return CHRF_OK;
}

struct DensifyScratch {
  size_t counts, offsets, tmp, bytes;
};

static DensifyScratch densify_scratch(int64_t n) {
  DensifyScratch d;
  const int64_t m = std::max<int64_t>(n, 1);
  d.counts = 0;
  d.offsets = align256(sizeof(uint32_t) * m);
  d.tmp = d.offsets + align256(sizeof(uint64_t) * m);
  d.bytes = d.tmp + align256(sizeof(uint64_t) * (scan_tmp_elems(m) + 16));
  return d;
}

size_t chrf_densify_workspace_bytes(int64_t n) { return n < 0 ? 0 : densify_scratch(n).bytes; }


chrf_status chrf_densify(const chrf_densify_desc* d, void* scratch, int64_t capacity, int32_t* src, int32_t* kind,
                         float* means_out, float* log_scales_out, float* phase_out, int64_t* n_out,
                         void* hip_stream) {
  if (!d || !scratch || !n_out) return fail(CHRF_EINVAL, "chrf_densify: NULL argument");
  if (d->n < 0 || d->n_lambda < 1 || d->n_lambda > kMaxLambda || capacity < 0)
    return fail(CHRF_EINVAL, "chrf_densify: bad sizes");
  if (d->n > 0 && (!d->means || !d->log_scales || !d->quats || !d->opacity || !d->phase || !d->grad_accum ||
                   !d->grad_count || !d->xi || !d->zeta))
    return fail(CHRF_EINVAL, "chrf_densify: NULL input array");
  if (capacity > 0 && (!src || !kind || !means_out || !log_scales_out || !phase_out))
    return fail(CHRF_EINVAL, "chrf_densify: NULL output array");
  DensifyArgs a{};
  a.n = d->n;
  a.n_lambda = d->n_lambda;
  a.means = d->means;
  a.log_scales = d->log_scales;
  a.quats = d->quats;
  a.opacity = d->opacity;
  a.phase = d->phase;
  a.grad_accum = d->grad_accum;
  a.grad_count = d->grad_count;
  a.xi = d->xi;
  a.zeta = d->zeta;
  a.tau_grad = d->tau_grad;
  a.sigma_split = d->sigma_split;
  a.sigma_prune = d->sigma_prune;
  a.min_opacity = d->min_opacity;
  a.phase_sigma = d->phase_sigma;
  a.shrink = d->shrink;
  a.capacity = capacity;
  a.src = src;
  a.kind = kind;
  a.means_out = means_out;
  a.log_scales_out = log_scales_out;
  a.phase_out = phase_out;
  const DensifyScratch ds = densify_scratch(d->n);
  char* base = static_cast<char*>(scratch);
  HIP_TRY(launch_densify(a, reinterpret_cast<uint32_t*>(base + ds.counts), reinterpret_cast<uint64_t*>(base + ds.offsets),
                         reinterpret_cast<uint64_t*>(base + ds.tmp), reinterpret_cast<uint64_t*>(n_out),
                         (hipStream_t)hip_stream));
  return CHRF_OK;
}

chrf_status chrf_densify_noalloc(const chrf_densify_desc* d, int64_t capacity, int32_t* src, int32_t* kind,
                                 float* means_out, float* log_scales_out, float* phase_out, int64_t* n_out,
                                 void* hip_stream) {
  if (!d) return fail(CHRF_EINVAL, "chrf_densify_noalloc: NULL argument");
  if (d->n > kNoallocMaxN)
    return fail(CHRF_EINVAL, "chrf_densify_noalloc: n = " + std::to_string(d->n) + " exceeds the maximum " +
                                 std::to_string(kNoallocMaxN) + " of the library's scratch array");
  int device = 0;
  if (hip_stream)
    HIP_TRY(hipStreamGetDevice((hipStream_t)hip_stream, &device));
  else
    HIP_TRY(hipGetDevice(&device));
  void* ptr = nullptr;
  const chrf_status st = noalloc_scratch(device, &ptr);
  if (st != CHRF_OK) return st;
  return chrf_densify(d, ptr, capacity, src, kind, means_out, log_scales_out, phase_out, n_out, hip_stream);
}

chrf_status chrf_gather_rows(const float* in, int64_t row, const int32_t* src, const int32_t* kind,
                             const int64_t* n_out, int64_t capacity, int32_t zero_new, float* out,
                             void* hip_stream) {
  if (row < 1 || capacity < 0) return fail(CHRF_EINVAL, "chrf_gather_rows: bad sizes");
  if (capacity > 0 && (!in || !src || !kind || !n_out || !out)) return fail(CHRF_EINVAL, "chrf_gather_rows: NULL argument");
  HIP_TRY(launch_gather_rows(in, row, src, kind, reinterpret_cast<const uint64_t*>(n_out), capacity, zero_new,
                             out, (hipStream_t)hip_stream));
  return CHRF_OK;
}

chrf_status chrf_read_status(chrf_plan* plan, void* ws, int64_t* pairs_needed, void* hip_stream) {
  if (!plan || !ws) return fail(CHRF_EINVAL, "chrf_read_status: NULL argument");
  uint32_t h[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(h, at<uint32_t>(plan, ws, R_STATUS), sizeof(h), hipMemcpyDeviceToHost,
                         (hipStream_t)hip_stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
  const uint64_t total = (uint64_t)h[0] | ((uint64_t)h[1] << 32);
  if (pairs_needed) *pairs_needed = (int64_t)total;
  if (h[3] != 0) return fail(CHRF_EHIP, "radix sort: a look-back wait gave up; the pair lists are not valid");
  if (h[2] != 0 || total > (uint64_t)plan->cap)
    return fail(CHRF_ECAPACITY, "pair list needs " + std::to_string(total) + " entries, capacity " +
                                    std::to_string(plan->cap));
  return CHRF_OK;
}

chrf_status chrf_timing_enable(chrf_plan* plan, int enable) {
  if (!plan) return fail(CHRF_EINVAL, "chrf_timing_enable: NULL plan");
  plan->timing = enable != 0;
  return CHRF_OK;
}

chrf_status chrf_timing_report(chrf_plan* plan, char* buf, size_t size) {
  if (!plan || !buf || size == 0) return fail(CHRF_EINVAL, "chrf_timing_report: bad argument");
  std::map<std::string, std::pair<int, double>> acc;
  std::vector<std::string> order;
  for (auto& r : plan->trec) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    if (!acc.count(r.name)) order.push_back(r.name);
    acc[r.name].first += 1;
    acc[r.name].second += ms;
    plan->ev_pool.push_back(r.a);
    plan->ev_pool.push_back(r.b);
  }
  plan->trec.clear();
  std::string outs;
  for (auto& n : order) {
    char line[256];
    snprintf(line, sizeof(line), "%s %d %.6f\n", n.c_str(), acc[n].first, acc[n].second);
    outs += line;
  }
  strncpy(buf, outs.c_str(), size - 1);
  buf[size - 1] = 0;
  return CHRF_OK;
}

}  // extern "C"
