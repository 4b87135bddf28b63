// Tile binning: device-wide scans, a stable LSD radix sort, pair emission and
// tile ranges (Algorithm 2: DuplicateWithDepthKeys, SortByKeys,
// IdentifyTileRanges).
//
// Ordering.  Visible Gaussians of every view are first sorted by the key
// (view, depth bits); the pairs (view * tiles + tile, Gaussian) are then
// emitted in that order and stably sorted by their 32-bit tile key.  The
// result equals a sort by (view, tile, depth, Gaussian index): the index
// tie-break comes from the stability of both sorts, since the first sort
// starts from index order.  Depths are positive floats, whose bit patterns
// order like their values.
//
// The radix sort is LSD with 8-bit digits.  Long sorts count per-block digit
// histograms of the keys in their current order each pass, scan them over
// (digit, block) and scatter stably through an LDS reorder; short sorts use
// single-sweep passes with decoupled look-back (below).  (The per-block split of a pass depends on the
// permutation the previous pass produced, so histograms of later passes
// cannot be taken from the input order.)  Ranks inside a
// block come from wave ballots: a lane's rank among equal digits is the
// popcount of the lower lanes whose 8 digit bits all match, plus the counts of
// earlier waves and earlier rounds held in LDS.  Counts that are only known on
// the device (the number of pairs) are read by every block, so the launch
// grid can be sized by capacity and the sequence needs no host round trip.
#include <algorithm>

#include "internal.h"

namespace chrf {

// ----------------------------------------------------------------- scans ---
template <typename T>
__device__ inline T block_exclusive_scan(T v, T* lds_warp, T* total) {
  // lds_warp holds kScanThreads / 64 entries
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds_warp[wave] = x;
  __syncthreads();
  T wbase = 0, tot = 0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) {
    T c = lds_warp[w];
    if (w < wave) wbase += c;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const TIn* __restrict__ in, int64_t n,
                                                              TOut* __restrict__ block_sums) {
  __shared__ TOut lw[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TOut s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += (TOut)in[base + i];
  TOut tot;
  block_exclusive_scan<TOut>(s, lw, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the block sums in place; sums[nb] = total
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_top(T* sums, int64_t nb, T* total) {
  __shared__ T lw[1024 / 64];
  T carry = 0;
  for (int64_t base = 0; base < nb; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    T v = i < nb ? sums[i] : 0;
    T tot;
    T ex = block_exclusive_scan<T>(v, lw, &tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const TIn* __restrict__ in, TOut* __restrict__ out,
                                                            int64_t n, const TOut* __restrict__ block_off) {
  __shared__ TOut lw[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TIn v[kScanItems];
  TOut s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += (TOut)v[i];
  }
  TOut tot;
  TOut run = block_exclusive_scan<TOut>(s, lw, &tot) + block_off[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += (TOut)v[i];
  }
}

// Down-sweep that forms its block offset itself, the sum of the block sums
// before it (a block reduction over at most kScanFuseBlocks values), instead
// of a separate single-block scan of the block sums; the last block also
// writes the total.
constexpr int kScanFuseBlocks = 1024;

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kScanThreads) void k_scan_down_fused(const TIn* __restrict__ in, TOut* __restrict__ out,
                                                                  int64_t n, const TOut* __restrict__ block_sums,
                                                                  TOut* total) {
  __shared__ TOut lw[kScanThreads / 64];
  TOut pre = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kScanThreads) pre += block_sums[b];
  TOut off;
  block_exclusive_scan<TOut>(pre, lw, &off);   // off: the sum over all threads
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TIn v[kScanItems];
  TOut s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += (TOut)v[i];
  }
  TOut tot;
  TOut run = block_exclusive_scan<TOut>(s, lw, &tot) + off;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += (TOut)v[i];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <typename T>
__global__ void k_zero_one(T* p) {
  *p = 0;
}

template <typename TIn, typename TOut>
static hipError_t scan_impl(const TIn* in, TOut* out, int64_t n, TOut* tmp, TOut* total, hipStream_t s) {
  if (n <= 0) {   // a kernel, not a memset, so that the sequence stays capturable
    if (total) k_zero_one<TOut><<<1, 1, 0, s>>>(total);
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  k_scan_reduce<TIn, TOut><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, tmp);
  if (nb <= kScanFuseBlocks) {
    k_scan_down_fused<TIn, TOut><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, tmp, total);
  } else {
    k_scan_top<TOut><<<1, 1024, 0, s>>>(tmp, nb, total);
    k_scan_down<TIn, TOut><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, tmp);
  }
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s) {
  return scan_impl<uint32_t, uint32_t>(in, out, n, tmp, (uint32_t*)nullptr, s);
}
hipError_t launch_scan_u64_from_u32(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* tmp, uint64_t* total,
                                    hipStream_t s) {
  return scan_impl<uint32_t, uint64_t>(in, out, n, tmp, total, s);
}

// ----------------------------------------------------------- radix sort ---
__device__ inline int64_t live_count(int64_t n_max, const uint64_t* n_dev) {
  if (!n_dev) return n_max;
  const uint64_t v = *n_dev;
  return v < (uint64_t)n_max ? (int64_t)v : n_max;
}

// Digit histogram of one pass per block: hist[digit * nblocks + block].
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K* __restrict__ keys, int64_t n_max,
                                                             const uint64_t* n_dev, int shift, uint32_t mask,
                                                             uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = live_count(n_max, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base < n) {
    // each thread counts kSortItems consecutive keys and adds every run of
    // equal digits with one atomic: sorted-by-depth pairs carry long runs in
    // their high tile digits, which would otherwise pile atomics on one counter
    const int64_t t0 = base + (int64_t)threadIdx.x * kSortItems;
    K k[kSortItems];
    if constexpr (sizeof(K) == 4) {
      if (t0 + kSortItems <= n) {
#pragma unroll
        for (int i = 0; i < kSortItems; i += 4) {
          const uint4 v = *reinterpret_cast<const uint4*>(keys + t0 + i);
          k[i] = v.x;
          k[i + 1] = v.y;
          k[i + 2] = v.z;
          k[i + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) k[i] = t0 + i < n ? keys[t0 + i] : K(0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < kSortItems; ++i) k[i] = t0 + i < n ? keys[t0 + i] : K(0);
    }
    uint32_t run_d = 0, run_c = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      if (t0 + i >= n) break;
      const uint32_t d = (uint32_t)(k[i] >> shift) & mask;
      if (run_c != 0 && d != run_d) {
        atomicAdd(&cnt[run_d], run_c);
        run_c = 0;
      }
      run_d = d;
      ++run_c;
    }
    if (run_c != 0) atomicAdd(&cnt[run_d], run_c);
  }
  __syncthreads();
  if (threadIdx.x <= mask) hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one pass.  Each wave ranks a contiguous quarter of the
// block's 16 x 256 keys, 64 at a time in order, against its own running
// digit counts in LDS (wave ballots group equal digits; no workgroup barrier
// while ranking), then the waves' counts give each wave's start within every
// digit.  The keys are placed in LDS in block-local digit order and written
// out in that order: the keys of one digit leave the block as one contiguous
// run, so the stores are coalesced instead of one scattered 4-byte store per
// key.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const K* __restrict__ keys_in,
                                                                const uint32_t* __restrict__ vals_in,
                                                                K* __restrict__ keys_out,
                                                                uint32_t* __restrict__ vals_out, int64_t n_max,
                                                                const uint64_t* n_dev, int shift, uint32_t mask,
                                                                const uint32_t* __restrict__ offsets, int nblocks) {
  constexpr int NW = kSortThreads / 64;
  constexpr int kWaveKeys = kSortItems * 64;   // keys ranked by one wave
  __shared__ uint32_t wcnt[NW][256];           // per wave: running digit counts, then its start in each digit
  __shared__ uint32_t goff[256];
  __shared__ uint32_t lstart[256];
  __shared__ uint32_t wsum[NW];
  __shared__ K skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = live_count(n_max, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= n) return;   // uniform per block
#pragma unroll
  for (int i = lane; i < 256; i += 64) wcnt[wave][i] = 0;   // read back only by this wave until the barrier
  goff[tid] = tid <= (int)mask ? offsets[(int64_t)tid * nblocks + blockIdx.x] : 0u;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  K key[kSortItems];
  uint32_t val[kSortItems], dig[kSortItems], rank[kSortItems];
  const int64_t wbase = base + (int64_t)wave * kWaveKeys;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = wbase + r * 64 + lane;
    const bool valid = idx < n;
    key[r] = 0;
    val[r] = 0;
    dig[r] = 0;
    if (valid) {
      key[r] = keys_in[idx];
      val[r] = vals_in[idx];
      dig[r] = (uint32_t)(key[r] >> shift) & mask;
    }
    const uint32_t d = dig[r];
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      if ((mask >> bit) == 0u) break;   // uniform: no digit has this bit
      const bool on = (d >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t lower = __popcll(peers & lt_mask);
    // every lane reads the count before the group's first lane updates it
    // (one wave's LDS operations complete in program order)
    const uint32_t before = wcnt[wave][d];
    rank[r] = valid ? before + lower : ~0u;   // rank among this wave's keys of digit d so far
    if (valid && lower == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // digit tid: each wave's start among the block's keys of that digit
  uint32_t total = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t c = wcnt[w][tid];
    wcnt[w][tid] = total;
    total += c;
  }
  uint32_t tot;
  lstart[tid] = block_exclusive_scan<uint32_t>(total, wsum, &tot);   // block-local start of every digit
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (rank[r] != ~0u) {
      const uint32_t p = lstart[dig[r]] + wcnt[wave][dig[r]] + rank[r];
      skey[p] = key[r];
      sval[p] = val[r];
    }
  }
  __syncthreads();
  const int nv = (int)(n - base < kSortTile ? n - base : kSortTile);
  for (int i = tid; i < nv; i += kSortThreads) {
    const K k = skey[i];
    const uint32_t d = (uint32_t)(k >> shift) & mask;
    const uint32_t pos = goff[d] + (uint32_t)i - lstart[d];
    if (pos < (uint64_t)n) {   // always true for consistent offsets; keeps every write in bounds
      keys_out[pos] = k;
      vals_out[pos] = sval[i];
    }
  }
}

// ------------------------------------------------- single-sweep passes ---
// The per-pass histogram and scan kernels above cost two extra sweeps and
// four launches per pass, which dominate short sorts (the per-view depth
// sort of 10^5 Gaussians).  A single-sweep pass instead takes each block's
// digit offsets from the blocks before it by decoupled look-back: blocks
// draw partition numbers from a counter in launch order, publish their
// per-digit counts, and add up the counts of earlier partitions until one
// that already holds its inclusive prefix.  The global digit totals of every
// pass do not depend on the order of the keys, so one counting sweep over
// the input serves all passes.
//
// Status word of (partition, digit): bits 30-31 a flag (0: not published,
// 1: this partition's count only, 2: inclusive prefix through this
// partition), bits 0-29 the value.  Needs fewer than 2^30 keys.
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1u;
constexpr int kLookbackPolls = 1 << 22;   // a wait that never ends sets the error word and stops
constexpr int kCountBlocks = 1024;
constexpr int kSweepMaxKeys = 1 << 19;      // sorts of up to 512 Ki keys take single sweeps
constexpr int kSweepItems = 4;              // keys per thread of a sweep partition
constexpr int kSweepTile = kSortThreads * kSweepItems;

__device__ inline uint32_t load_status(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_status(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Global digit counts of every pass: counts[pass][digit].
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_digit_counts(const K* __restrict__ keys, int64_t n_max,
                                                               const uint64_t* n_dev, int begin_bit, int npasses,
                                                               uint32_t* __restrict__ counts) {
  __shared__ uint32_t c[kMaxSortPasses][256];
  for (int p = 0; p < npasses; ++p) c[p][threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = live_count(n_max, n_dev);
  for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSortThreads) {
    const K k = keys[i];
    for (int p = 0; p < npasses; ++p) atomicAdd(&c[p][(uint32_t)(k >> (begin_bit + 8 * p)) & 255u], 1u);
  }
  __syncthreads();
  for (int p = 0; p < npasses; ++p) {
    const uint32_t v = c[p][threadIdx.x];
    if (v) atomicAdd(&counts[p * 256 + threadIdx.x], v);
  }
}

// One pass: count the partition's digits and publish them at once (so that
// later partitions rarely wait), look back for the digit offsets, rank the
// keys (as k_radix_scatter), then write through the LDS reorder.
template <typename K, int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_onesweep(const K* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           K* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                           int64_t n_max, const uint64_t* n_dev, int shift,
                                                           const uint32_t* __restrict__ counts, uint32_t* status,
                                                           uint32_t* ticket, uint32_t* error) {
  constexpr int NW = kSortThreads / 64;
  __shared__ uint32_t hcnt[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[NW][256];
  __shared__ uint32_t goff[256];
  __shared__ uint32_t lstart[256];
  __shared__ uint32_t wsum[NW];
  __shared__ uint32_t s_part;
  constexpr int TILE = kSortThreads * ITEMS;
  __shared__ K skey[TILE];
  __shared__ uint32_t sval[TILE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_part = atomicAdd(ticket, 1u);
  hcnt[tid] = 0;
  run[tid] = 0;
  for (int w = 0; w < NW; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint32_t part = s_part;
  const int64_t n = live_count(n_max, n_dev);
  const int64_t base = (int64_t)part * TILE;
  if (base >= n) return;   // uniform per block; later partitions are empty too, so nobody waits on this one
  K key[ITEMS];
  uint32_t val[ITEMS], dig[ITEMS], rank[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t idx = base + (int64_t)r * kSortThreads + tid;
    key[r] = 0;
    val[r] = 0;
    dig[r] = 0;
    if (idx < n) {
      key[r] = keys_in[idx];
      val[r] = vals_in[idx];
      dig[r] = (uint32_t)(key[r] >> shift) & 255u;
      atomicAdd(&hcnt[dig[r]], 1u);
    }
  }
  __syncthreads();
  // publish this partition's count of digit tid, then look back
  const uint32_t mine = hcnt[tid];
  uint32_t* my = status + (size_t)part * 256 + tid;
  store_status(my, (part == 0 ? kFlagInc : kFlagAgg) | mine);
  uint32_t excl = 0;
  if (part > 0) {
    int64_t k = (int64_t)part - 1;
    int polls = 0;
    while (true) {
      const uint32_t w = load_status(status + (size_t)k * 256 + tid);
      const uint32_t f = w & ~kValMask;
      if (f == 0u) {
        if (++polls > kLookbackPolls) {
          store_status(error, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += w & kValMask;
      if (f == kFlagInc) break;
      --k;   // partition 0 always publishes an inclusive value, so k stays >= 0
    }
    store_status(my, kFlagInc | (excl + mine));
  }
  uint32_t tot;
  goff[tid] = block_exclusive_scan<uint32_t>(counts[tid], wsum, &tot) + excl;
  lstart[tid] = block_exclusive_scan<uint32_t>(mine, wsum, &tot);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const bool valid = base + (int64_t)r * kSortThreads + tid < n;
    const uint32_t d = dig[r];
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t lower = __popcll(peers & lt_mask);
    if (valid && lower == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wcnt[w][d];
    rank[r] = valid ? run[d] + before + lower : ~0u;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < NW; ++w) {
      add += wcnt[w][tid];
      wcnt[w][tid] = 0;
    }
    run[tid] += add;
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    if (rank[r] != ~0u) {
      const uint32_t p = lstart[dig[r]] + rank[r];
      skey[p] = key[r];
      sval[p] = val[r];
    }
  }
  __syncthreads();
  const int nv = (int)(n - base < TILE ? n - base : TILE);
  for (int i = tid; i < nv; i += kSortThreads) {
    const K k = skey[i];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const uint32_t pos = goff[d] + (uint32_t)i - lstart[d];
    if (pos < (uint64_t)n) {   // always true for consistent offsets; keeps every write in bounds
      keys_out[pos] = k;
      vals_out[pos] = sval[i];
    }
  }
}

// Workspace of a sort of up to n_max keys, in 32-bit words: the three-kernel
// passes use 256 * nblocks words of histogram; single sweeps use, per pass,
// the (partition, digit) status words, the digit counts and a partition
// counter.
int64_t radix_hist_elems(int64_t n_max) {
  const int64_t nb = std::max<int64_t>((n_max + kSortTile - 1) / kSortTile, 1);
  int64_t words = 256 * nb;
  if (n_max <= kSweepMaxKeys) {
    const int64_t parts = std::max<int64_t>((n_max + kSweepTile - 1) / kSweepTile, 1);
    words = std::max<int64_t>(words, (int64_t)kMaxSortPasses * (256 * parts + 256 + 1));
  }
  return words;
}

template <typename K>
static hipError_t radix_sort_impl(K* keys, K* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t n_max,
                                  const uint64_t* n_dev, int begin_bit, int end_bit, uint32_t* hist,
                                  uint32_t* scan_tmp, uint32_t* error, bool* result_in_alt, hipStream_t s) {
  *result_in_alt = false;
  if (n_max <= 0) return hipSuccess;
  // single sweeps pay off for short sorts, where the launches of the
  // histogram and scan kernels dominate; long ones keep the three-kernel pass
  const bool sweep = n_max <= kSweepMaxKeys;
  const int nblocks = (int)((n_max + (sweep ? kSweepTile : kSortTile) - 1) / (sweep ? kSweepTile : kSortTile));
  const int npasses = (end_bit - begin_bit + 7) / 8;
  if (npasses <= 0) return hipSuccess;
  if (npasses > kMaxSortPasses) return hipErrorInvalidValue;
  K* kin = keys;
  K* kout = keys_alt;
  uint32_t* vin = vals;
  uint32_t* vout = vals_alt;
  hipError_t e = hipSuccess;
  uint32_t* status = hist;
  uint32_t* counts = hist + (size_t)npasses * 256 * nblocks;
  uint32_t* tickets = counts + (size_t)npasses * 256;
  if (sweep) {
    e = launch_fill_u32(hist, 0u, (int64_t)npasses * (256 * (int64_t)nblocks + 256) + npasses, s);
    if (e != hipSuccess) return e;
    const int cb = nblocks < kCountBlocks ? nblocks : kCountBlocks;
    k_digit_counts<K><<<cb, kSortThreads, 0, s>>>(kin, n_max, n_dev, begin_bit, npasses, counts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // The three-kernel passes split the key bits evenly (13 bits: 7 + 6), so
  // that each block's keys of one digit leave it in longer runs; single
  // sweeps take 8-bit digits.
  int shift = begin_bit;
  for (int pass = 0; pass < npasses; ++pass) {
    const int bits = end_bit - begin_bit;
    const int width = sweep ? 8 : bits / npasses + (pass < bits % npasses ? 1 : 0);
    const uint32_t mask = (1u << width) - 1u;
    if (sweep) {
      k_onesweep<K, kSweepItems><<<nblocks, kSortThreads, 0, s>>>(kin, vin, kout, vout, n_max, n_dev, shift,
                                                                  counts + pass * 256,
                                                                  status + (size_t)pass * 256 * nblocks,
                                                                  tickets + pass, error);
    } else {
      k_radix_hist<K><<<nblocks, kSortThreads, 0, s>>>(kin, n_max, n_dev, shift, mask, hist, nblocks);
      e = launch_scan_u32(hist, hist, (int64_t)(mask + 1) * nblocks, scan_tmp, s);
      if (e != hipSuccess) return e;
      k_radix_scatter<K><<<nblocks, kSortThreads, 0, s>>>(kin, vin, kout, vout, n_max, n_dev, shift, mask, hist,
                                                          nblocks);
    }
    shift += width;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    K* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
    *result_in_alt = !*result_in_alt;
  }
  return hipGetLastError();
}

hipError_t radix_sort_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t n_max,
                          const uint64_t* n_dev, int begin_bit, int end_bit, uint32_t* hist, uint32_t* scan_tmp,
                          uint32_t* error, bool* result_in_alt, hipStream_t s) {
  return radix_sort_impl<uint64_t>(keys, keys_alt, vals, vals_alt, n_max, n_dev, begin_bit, end_bit, hist,
                                   scan_tmp, error, result_in_alt, s);
}
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t n_max,
                          const uint64_t* n_dev, int begin_bit, int end_bit, uint32_t* hist, uint32_t* scan_tmp,
                          uint32_t* error, bool* result_in_alt, hipStream_t s) {
  return radix_sort_impl<uint32_t>(keys, keys_alt, vals, vals_alt, n_max, n_dev, begin_bit, end_bit, hist,
                                   scan_tmp, error, result_in_alt, s);
}

// -------------------------------------------------------- pair emission ---
// Which tiles of its support rectangle a Gaussian is binned to.  A pixel is
// supported only where power = (A dx^2 + C dy^2) / 2 + B dx dy <= pmax
// (dx, dy: pixel centre - mu; pmax = min(k^2/2, ln(o / alpha_min)), set by
// the projection).  For one tile row, whose pixel centres span dy in
// [y0, y1], the centres dx of that band inside the ellipse power <= pm form
// one interval (the projection of a convex set): its right end is the
// largest root dx of power(dx, dy) = pm over dy in the band, a concave
// function of dy that peaks at the ellipse's rightmost point dy = -B xr / C
// (xr = sqrt(2 pm C / D), D = AC - B^2), so it is attained at that dy
// clamped to the band; the left end likewise.  The row keeps the tiles that
// the interval's pixel columns touch.  pm exceeds pmax by a margin that
// covers the rounding of the per-pixel power (1e-4 plus 4e-6 times the
// form's size over the rectangle) and of this computation (1e-3 |pmax|), so
// no tile holding a supported pixel is dropped.  The result decides the
// tile lists, so it is one fixed single-precision recipe (no contraction,
// IEEE division and square root; D from exact double products rounded once)
// that the CPU reference reproduces bit for bit.
struct SpanGeom {
  float mx, my, A, B, D, t, ymax, ytip;
  int c0, c1, r0, r1;
  bool none, full;   // no tile at all / every tile of the rectangle
};

__device__ inline SpanGeom span_geom(const float4& g0, const float4& g1, const int4& rc) {
#pragma clang fp contract(off)
  SpanGeom s;
  s.mx = g0.x;
  s.my = g0.y;
  s.A = g0.z;
  s.B = g0.w;
  const float C = g1.x, P = g1.z;
  s.c0 = rc.x;
  s.c1 = rc.x + rc.y;
  s.r0 = rc.z;
  s.r1 = rc.z + rc.w;
  const float x0 = ((float)s.c0 + 0.5f) - s.mx, x1 = ((float)s.c1 + 0.5f) - s.mx;
  const float y0 = ((float)s.r0 + 0.5f) - s.my, y1 = ((float)s.r1 + 0.5f) - s.my;
  const float xm = fmaxf(-x0, x1), ym = fmaxf(-y0, y1);   // largest |dx|, |dy| over the rectangle
  const float mag = 0.5f * ((s.A * xm) * xm + (C * ym) * ym) + (fabsf(s.B) * xm) * ym;
  const float pm = P + ((1e-4f + 1e-3f * fabsf(P)) + 4e-6f * mag);
  s.D = (float)((double)s.A * (double)C - (double)s.B * (double)s.B);
  const float w = (2.0f * pm) / s.D;
  s.t = (2.0f * pm) * s.A;
  s.ymax = __builtin_sqrtf(w * s.A);   // the ellipse's half-height
  const float xr = __builtin_sqrtf(w * C);
  s.ytip = -(s.B * xr) / C;             // dy of its rightmost point
  s.none = !(pm > 0.0f);
  s.full = !s.none && !(s.D > 0.0f && s.A > 0.0f && C > 0.0f && __builtin_isfinite(s.t) &&
                        __builtin_isfinite(s.ymax) && __builtin_isfinite(s.ytip));
  return s;
}

// Pixel columns [*clo, *chi] of tile row ty that the ellipse reaches; returns
// the number of tiles they touch (0: none, *clo > *chi).
__device__ inline int row_span(const SpanGeom& s, int ty, int tile_w, int tile_h, int* clo, int* chi) {
#pragma clang fp contract(off)
  int lo = s.c0, hi = s.c1;
  if (s.none) {
    hi = lo - 1;
  } else if (!s.full) {
    const int ylo = max(ty * tile_h, s.r0), yhi = min(ty * tile_h + tile_h - 1, s.r1);
    const float y0 = ((float)ylo + 0.5f) - s.my, y1 = ((float)yhi + 0.5f) - s.my;
    const float a = fmaxf(y0, -s.ymax), b = fminf(y1, s.ymax);
    if (!(a <= b)) {
      hi = lo - 1;                       // the band misses the ellipse
    } else {
      const float dr = fminf(fmaxf(s.ytip, a), b), dl = fminf(fmaxf(-s.ytip, a), b);
      const float sr = __builtin_sqrtf(fmaxf(s.t - (s.D * dr) * dr, 0.0f));
      const float sl = __builtin_sqrtf(fmaxf(s.t - (s.D * dl) * dl, 0.0f));
      const float xh = (s.mx + (sr - s.B * dr) / s.A) - 0.5f;
      const float xl = (s.mx + (-sl - s.B * dl) / s.A) - 0.5f;
      if (xl == xl && xh == xh) {       // a NaN keeps the whole row
        const float cl = (float)s.c0 - 1.0f, ch = (float)s.c1 + 1.0f;
        lo = max((int)ceilf(fminf(fmaxf(xl, cl), ch)), s.c0);
        hi = min((int)floorf(fminf(fmaxf(xh, cl), ch)), s.c1);
      }
    }
  }
  *clo = lo;
  *chi = hi;
  return lo <= hi ? hi / tile_w - lo / tile_w + 1 : 0;
}

// A team of consecutive lanes per sorted (view, Gaussian) entry i; lane r
// takes the tile rows r, r + team, ... of its rectangle.  Counting, which
// only sums, takes teams of 8; emission, which writes the rows' tiles, 16.
constexpr int kCountTeam = 8;
constexpr int kEmitTeam = 16;

template <int TEAM>
__device__ inline int team_sum(int v) {
#pragma unroll
  for (int m = TEAM / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, TEAM);
  return v;
}

__global__ __launch_bounds__(256) void k_count_pairs(const uint32_t* __restrict__ sorted_val,
                                                     const uint32_t* __restrict__ count,
                                                     const float4* __restrict__ rec_g0,
                                                     const float4* __restrict__ rec_g1,
                                                     const int4* __restrict__ rect, int64_t n, int tile_w, int tile_h,
                                                     uint32_t* __restrict__ cnt_sorted) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kCountTeam;
  const int lane = threadIdx.x % kCountTeam;
  const bool live = i < n;
  const uint32_t rid = live ? sorted_val[i] : 0u;
  int kept = 0;
  if (live && count[rid] > 0) {          // visible, with a non-empty rectangle
    const SpanGeom g = span_geom(rec_g0[rid], rec_g1[rid], rect[rid]);
    const int ty1 = g.r1 / tile_h;
    for (int ty = g.r0 / tile_h + lane; ty <= ty1; ty += kCountTeam) {
      int lo, hi;
      kept += row_span(g, ty, tile_w, tile_h, &lo, &hi);
    }
  }
  kept = team_sum<kCountTeam>(kept);
  if (live && lane == 0) cnt_sorted[i] = (uint32_t)kept;
}

hipError_t launch_count_pairs(const uint32_t* sorted_val, const uint32_t* count, const float4* rec_g0,
                              const float4* rec_g1, const int4* rect, int64_t n, int tile_w, int tile_h,
                              uint32_t* cnt_sorted, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t threads = n * kCountTeam;
  k_count_pairs<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(sorted_val, count, rec_g0, rec_g1, rect, n, tile_w,
                                                                   tile_h, cnt_sorted);
  return hipGetLastError();
}

// Emission: the team computes the spans of kEmitTeam tile rows at once (lane
// r: row base + r) and scans their tile counts; the rows' ends and first
// keys go to LDS, and the team then writes the chunk's pairs as one flat run,
// consecutive lanes on consecutive slots, each lane finding its row by a
// binary search over the ends.  Pairs past the capacity are dropped and
// flagged, so every write stays in bounds.
__global__ __launch_bounds__(256) void k_emit_pairs(const uint32_t* __restrict__ sorted_val,
                                                    const uint64_t* __restrict__ offsets,
                                                    const uint32_t* __restrict__ cnt_sorted,
                                                    const float4* __restrict__ rec_g0,
                                                    const float4* __restrict__ rec_g1,
                                                    const int4* __restrict__ rect, int64_t n, int n_stride,
                                                    int tile_w, int tile_h, int tiles_x, int tile_bits,
                                                    uint32_t* __restrict__ pair_key, uint32_t* __restrict__ pair_val,
                                                    int64_t capacity, const uint64_t* total, uint32_t* status,
                                                    uint32_t* __restrict__ det_rid) {
  __shared__ int s_end[256 / kEmitTeam][kEmitTeam];
  __shared__ uint32_t s_key[256 / kEmitTeam][kEmitTeam];
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kEmitTeam;
  const int lane = threadIdx.x % kEmitTeam, team = threadIdx.x / kEmitTeam;
  if (i == 0 && lane == 0 && *total > (uint64_t)capacity) status[0] = 1u;
  if (i >= n || cnt_sorted[i] == 0) return;   // whole teams leave together
  const uint32_t rid = sorted_val[i];
  uint64_t out = offsets[i];
  const SpanGeom g = span_geom(rec_g0[rid], rec_g1[rid], rect[rid]);
  // key = view << tile_bits | tile.  The list arrives view-major (the
  // Gaussians are sorted by (view, depth)), so a stable sort by the low
  // tile_bits bits (or by any more low bits) keeps each (view, tile) run
  // contiguous and in depth order: runs that share those bits belong to
  // different views and stay in view order.
  const uint32_t vkey = (rid / (uint32_t)n_stride) << tile_bits;
  const int ty0 = g.r0 / tile_h, ty1 = g.r1 / tile_h;
  for (int base = ty0; base <= ty1; base += kEmitTeam) {
    const int ty = base + lane;
    int lo = 0, hi = -1, nt = 0;
    if (ty <= ty1) nt = row_span(g, ty, tile_w, tile_h, &lo, &hi);
    int end = nt;   // inclusive scan of the rows' tile counts
#pragma unroll
    for (int d = 1; d < kEmitTeam; d <<= 1) {
      const int v = __shfl_up(end, d, kEmitTeam);
      if (lane >= d) end += v;
    }
    const int tot = __shfl(end, kEmitTeam - 1, kEmitTeam);
    // pair j of the chunk in row r has key s_key[r] + j (vkey + tile equals
    // vkey | tile; the offset by the row's first j may wrap, the sum does not)
    s_end[team][lane] = end;
    s_key[team][lane] = vkey + (uint32_t)(ty * tiles_x + lo / tile_w - (end - nt));
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < tot; j += kEmitTeam) {
      int r = 0;   // first row whose end exceeds j
#pragma unroll
      for (int step = kEmitTeam / 2; step >= 1; step >>= 1)
        if (s_end[team][r + step - 1] <= j) r += step;
      const uint64_t slot = out + (uint64_t)j;
      if (slot < (uint64_t)capacity) {
        pair_key[slot] = s_key[team][r] + (uint32_t)j;
        if (det_rid) {
          // deterministic mode: the sort carries the emission slot, the record id waits aside
          pair_val[slot] = (uint32_t)slot;
          det_rid[slot] = rid;
        } else {
          pair_val[slot] = rid;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    out += (uint64_t)tot;
  }
}

hipError_t launch_emit_pairs(const uint32_t* sorted_val, const uint64_t* offsets, const uint32_t* cnt_sorted,
                             const float4* rec_g0, const float4* rec_g1, const int4* rect, int64_t n, int n_stride,
                             int tile_w, int tile_h, int tiles_x, int tile_bits, uint32_t* pair_key,
                             uint32_t* pair_val, int64_t capacity, const uint64_t* total, uint32_t* status,
                             uint32_t* det_rid, hipStream_t s) {
  if (n <= 0 || capacity <= 0) return hipSuccess;
  const int64_t threads = n * kEmitTeam;
  k_emit_pairs<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(sorted_val, offsets, cnt_sorted, rec_g0, rec_g1,
                                                                  rect, n, n_stride, tile_w, tile_h, tiles_x,
                                                                  tile_bits, pair_key, pair_val, capacity, total,
                                                                  status, det_rid);
  return hipGetLastError();
}

// Deterministic mode, after the pair sort: the sorted values are emission
// slots u.  Record where each slot went (inv[u] = sorted position) and
// replace the slot by its record id, so the raster reads the usual list.
__global__ __launch_bounds__(256) void k_det_gather(uint32_t* __restrict__ pair_val,
                                                    const uint32_t* __restrict__ det_rid, uint32_t* __restrict__ inv,
                                                    const uint64_t* total, int64_t capacity) {
  const uint64_t live = min(*total, (uint64_t)capacity);
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < live; j += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = pair_val[j];
    inv[u] = (uint32_t)j;
    pair_val[j] = det_rid[u];
  }
}

hipError_t launch_det_gather(uint32_t* pair_val, const uint32_t* det_rid, uint32_t* inv, const uint64_t* total,
                             int64_t capacity, hipStream_t s) {
  if (capacity <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((capacity + 255) / 256, 4096);
  k_det_gather<<<(unsigned)blocks, 256, 0, s>>>(pair_val, det_rid, inv, total, capacity);
  return hipGetLastError();
}

// Deterministic mode, after the raster backward wrote one gradient row per
// sorted pair: each (view, Gaussian) row of grad2d is the sum of its pairs'
// rows taken in emission order (the order of its tiles), with plain stores.
__global__ __launch_bounds__(256) void k_det_reduce(const uint32_t* __restrict__ sorted_val,
                                                    const uint64_t* __restrict__ offsets,
                                                    const uint32_t* __restrict__ cnt_sorted,
                                                    const uint32_t* __restrict__ inv,
                                                    const float* __restrict__ pair_grad, int64_t n, int g2,
                                                    int64_t capacity, float* __restrict__ grad2d) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / g2;
  const int c = (int)(t - i * g2);
  if (i >= n) return;
  const uint32_t cnt = cnt_sorted[i];
  if (cnt == 0) return;
  const uint64_t base = offsets[i];
  if (base >= (uint64_t)capacity) return;
  const uint64_t end = min(base + cnt, (uint64_t)capacity);
  float sum = 0.f;
  for (uint64_t u = base; u < end; ++u) sum += pair_grad[(size_t)inv[u] * g2 + c];
  grad2d[(size_t)sorted_val[i] * g2 + c] = sum;
}

hipError_t launch_det_reduce(const uint32_t* sorted_val, const uint64_t* offsets, const uint32_t* cnt_sorted,
                             const uint32_t* inv, const float* pair_grad, int64_t n, int g2, int64_t capacity,
                             float* grad2d, hipStream_t s) {
  if (n <= 0 || capacity <= 0) return hipSuccess;
  const int64_t threads = n * g2;
  k_det_reduce<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(sorted_val, offsets, cnt_sorted, inv, pair_grad, n,
                                                                  g2, capacity, grad2d);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, value, n);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, value, n);
  return hipGetLastError();
}

// Tile ranges from the sorted pair keys: [first, one past last) of every
// tile present.  Each thread takes four consecutive keys with one 16-byte
// load (plus the keys just before and after them), in a grid-stride loop.
constexpr int kRangeKeys = 4;
constexpr int kRangeMaxBlocks = 2048;

// [start, end) of every (view, tile) run of the sorted list; a key
// view << tile_bits | tile is the run view * n_tiles + tile.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ key, int tile_bits, uint32_t n_tiles,
                                                     const uint64_t* total, int64_t capacity,
                                                     uint2* __restrict__ ranges) {
  const uint64_t t = *total;
  const int64_t n = t < (uint64_t)capacity ? (int64_t)t : capacity;
  const uint32_t tmask = (1u << tile_bits) - 1u;
  auto run_of = [&](uint32_t k) { return (k >> tile_bits) * n_tiles + (k & tmask); };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kRangeKeys;
  for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeKeys; i0 < n; i0 += stride) {
    uint32_t k[kRangeKeys];
    if (i0 + kRangeKeys <= n) {
      const uint4 v = *reinterpret_cast<const uint4*>(key + i0);
      k[0] = v.x;
      k[1] = v.y;
      k[2] = v.z;
      k[3] = v.w;
    } else {
#pragma unroll
      for (int e = 0; e < kRangeKeys; ++e) k[e] = i0 + e < n ? key[i0 + e] : 0u;
    }
    const bool has_prev = i0 > 0, has_next = i0 + kRangeKeys < n;
    const uint32_t prev = has_prev ? key[i0 - 1] : 0u;
    const uint32_t next = has_next ? key[i0 + kRangeKeys] : 0u;
#pragma unroll
    for (int e = 0; e < kRangeKeys; ++e) {
      const int64_t i = i0 + e;
      if (i >= n) break;
      const bool first = e == 0 ? !has_prev || prev != k[0] : k[e - 1] != k[e];
      const bool last = i + 1 == n || (e + 1 < kRangeKeys ? k[e + 1] != k[e] : next != k[e]);
      if (first) ranges[run_of(k[e])].x = (uint32_t)i;
      if (last) ranges[run_of(k[e])].y = (uint32_t)(i + 1);
    }
  }
}

hipError_t launch_tile_ranges(const uint32_t* pair_key, int tile_bits, int n_tiles, const uint64_t* total,
                              int64_t capacity, uint2* ranges, hipStream_t s) {
  if (capacity <= 0) return hipSuccess;
  const int64_t per_block = 256 * kRangeKeys;
  const int64_t blocks = std::min<int64_t>((capacity + per_block - 1) / per_block, kRangeMaxBlocks);
  k_tile_ranges<<<(unsigned)blocks, 256, 0, s>>>(pair_key, tile_bits, (uint32_t)n_tiles, total, capacity, ranges);
  return hipGetLastError();
}

// One workgroup: histogram of the (view, tile) items over 256 buckets of
// descending list length (8 per octave of length + 1), exclusive scan, then
// each item takes the next slot of its bucket.
__global__ __launch_bounds__(1024) void k_tile_order(const uint2* __restrict__ ranges, int n,
                                                     uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[256];
  if (threadIdx.x < 256) cnt[threadIdx.x] = 0;
  __syncthreads();
  auto bucket = [&](int i) {
    const uint2 r = ranges[i];
    const uint32_t len = (r.y > r.x ? r.y - r.x : 0u) + 1u;
    const int msb = 31 - __clz(len);
    const int frac = msb >= 3 ? (int)((len >> (msb - 3)) & 7u) : (int)((len << (3 - msb)) & 7u);
    return 255 - min(255, msb * 8 + frac);
  };
  for (int i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&cnt[bucket(i)], 1u);
  __syncthreads();
  // exclusive scan of the 256 counts: four waves scan 64 each, then add the
  // totals of the waves before them
  __shared__ uint32_t wave_tot[4];
  uint32_t c = 0, incl = 0;
  if (threadIdx.x < 256) {
    c = cnt[threadIdx.x];
    incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off, 64);
      if ((int)(threadIdx.x & 63) >= off) incl += t;
    }
    if ((threadIdx.x & 63) == 63) wave_tot[threadIdx.x >> 6] = incl;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    uint32_t before = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += wave_tot[w];
    cnt[threadIdx.x] = before + incl - c;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) order[atomicAdd(&cnt[bucket(i)], 1u)] = (uint32_t)i;
}

hipError_t launch_tile_order(const uint2* ranges, int n, uint32_t* order, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_tile_order<<<1, 1024, 0, s>>>(ranges, n, order);
  return hipGetLastError();
}

}  // namespace chrf
