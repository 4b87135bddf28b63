// Mixed-radix Stockham FFT building blocks for LDS-resident sequences.
//
// The propagation of Eqs. 14 and 16 is two passes of 1-D transforms over a
// zero-padded grid.  Each pass keeps one or a few sequences of length N in
// LDS and runs log_R(N) Stockham stages on them; every stage reads R elements
// per butterfly into registers, applies the inter-stage twiddles and a small
// radix-R DFT, and writes the outputs back in autosorted order, so that the
// result is in natural order with no bit-reversal pass.
//
// Small DFTs are written out for radix 2, 3, 4, 5, 8; radices 6, 9, 10, 12,
// 15, 16 are composed from them with compile-time twiddles.  Forward
// transforms use exp(-2 pi i k n / N), inverse ones exp(+2 pi i k n / N);
// neither is normalised here.
#pragma once
#include <hip/hip_runtime.h>

namespace chrf {

struct cpx {
  float x, y;
};

// Workgroup barrier ordering LDS accesses only.  The stage barriers of the
// transforms guard nothing but the LDS work buffer; unlike __syncthreads()
// this one does not first wait for the wave's global loads and stores still
// in flight (output stores, or copies into LDS for the next transform).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// The same for waves with copies into LDS (global_load_lds) in flight to a
// buffer that the barrier does not guard: an LDS fence would also wait for
// those copies, so the wave waits only for its own LDS operations (the
// memory clobber keeps the compiler from moving accesses across).  The
// caller waits for the copies itself before reading their buffer.
__device__ inline void lds_barrier_copies_in_flight() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__host__ __device__ inline cpx mk(float x, float y) { return cpx{x, y}; }
__host__ __device__ inline cpx operator+(cpx a, cpx b) { return cpx{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cpx operator-(cpx a, cpx b) { return cpx{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cpx operator*(cpx a, float s) { return cpx{a.x * s, a.y * s}; }
__host__ __device__ inline cpx cmul(cpx a, cpx b) { return cpx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline cpx cmulc(cpx a, cpx b) { return cpx{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a * conj(b)
__host__ __device__ inline cpx cconj(cpx a) { return cpx{a.x, -a.y}; }
// multiply by -i for the forward sign, +i for the inverse sign
template <bool INV> __host__ __device__ inline cpx rot(cpx a) {
  return INV ? cpx{-a.y, a.x} : cpx{a.y, -a.x};
}

// ---- compile-time twiddles: exp(-2 pi i m / R) as double, folded to float ----
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double ct_sin(double x) {   // |x| <= pi after reduction
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double ct_reduce(double x) {
  while (x > kPi) x -= 2 * kPi;
  while (x < -kPi) x += 2 * kPi;
  return x;
}
constexpr double ct_sin_r(double x) { return ct_sin(ct_reduce(x)); }
constexpr double ct_cos_r(double x) { return ct_sin(ct_reduce(x + kPi / 2)); }

template <int N>
struct TwidN {   // exp(-2 pi i m / N), m < N
  float c[N], s[N];
  constexpr TwidN() : c(), s() {
    for (int m = 0; m < N; ++m) {
      c[m] = float(ct_cos_r(2.0 * kPi * double(m) / double(N)));
      s[m] = float(ct_sin_r(2.0 * kPi * double(m) / double(N)));
    }
  }
};

template <int N, bool INV>
__host__ __device__ inline cpx ct_tw(int m) {   // m is a compile-time constant after unrolling
  constexpr TwidN<N> t{};
  return INV ? cpx{t.c[m % N], t.s[m % N]} : cpx{t.c[m % N], -t.s[m % N]};
}

// ---- small DFTs in registers ----
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  __host__ __device__ static inline void run(cpx* x) {
    cpx a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  }
};

template <bool INV> struct Dft<3, INV> {
  __host__ __device__ static inline void run(cpx* x) {
    const float s3 = 0.86602540378443864676f;
    cpx t = x[1] + x[2];
    cpx m = x[0] - t * 0.5f;
    cpx d = rot<INV>(x[1] - x[2]) * s3;
    x[0] = x[0] + t;
    x[1] = m + d;
    x[2] = m - d;
  }
};

template <bool INV> struct Dft<4, INV> {
  __host__ __device__ static inline void run(cpx* x) {
    cpx a = x[0] + x[2], b = x[0] - x[2];
    cpx c = x[1] + x[3], d = rot<INV>(x[1] - x[3]);
    x[0] = a + c;
    x[2] = a - c;
    x[1] = b + d;
    x[3] = b - d;
  }
};

template <bool INV> struct Dft<5, INV> {
  __host__ __device__ static inline void run(cpx* x) {
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
    cpx t1 = x[1] + x[4], t2 = x[2] + x[3];
    cpx d1 = x[1] - x[4], d2 = x[2] - x[3];
    cpx a1 = x[0] + t1 * c1 + t2 * c2;
    cpx a2 = x[0] + t1 * c2 + t2 * c1;
    cpx b1 = rot<INV>(d1 * s1 + d2 * s2);
    cpx b2 = rot<INV>(d1 * s2 - d2 * s1);
    x[0] = x[0] + t1 + t2;
    x[1] = a1 + b1;
    x[4] = a1 - b1;
    x[2] = a2 + b2;
    x[3] = a2 - b2;
  }
};

template <bool INV> struct Dft<8, INV> {
  __host__ __device__ static inline void run(cpx* x) {
    const float h = 0.70710678118654752440f;
    cpx e[4] = {x[0], x[2], x[4], x[6]};
    cpx o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // o[q] *= W8^q (forward W8 = (1 - i)/sqrt2)
    cpx o1 = (rot<INV>(o[1]) + o[1]) * h;          // (1 -+ i)/sqrt2 * o1
    cpx o2 = rot<INV>(o[2]);
    cpx o3 = (rot<INV>(o[3]) - o[3]) * h;          // (-1 -+ i)/sqrt2 * o3
    x[0] = e[0] + o[0];
    x[4] = e[0] - o[0];
    x[1] = e[1] + o1;
    x[5] = e[1] - o1;
    x[2] = e[2] + o2;
    x[6] = e[2] - o2;
    x[3] = e[3] + o3;
    x[7] = e[3] - o3;
  }
};

// R = R1 * R2:  n = n1 + R1 n2,  k = k2 + R2 k1
template <int R1, int R2, bool INV>
struct DftComp {
  __host__ __device__ static inline void run(cpx* x) {
    constexpr int R = R1 * R2;
    cpx y[R1][R2];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) y[n1][n2] = x[n1 + R1 * n2];
      Dft<R2, INV>::run(y[n1]);
#pragma unroll
      for (int k2 = 1; k2 < R2; ++k2)
        if (n1 > 0) y[n1][k2] = cmul(y[n1][k2], ct_tw<R, INV>(n1 * k2));
    }
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      cpx z[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) z[n1] = y[n1][k2];
      Dft<R1, INV>::run(z);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) x[k2 + R2 * k1] = z[k1];
    }
  }
};

template <bool INV> struct Dft<6, INV> : DftComp<2, 3, INV> {};
template <bool INV> struct Dft<9, INV> : DftComp<3, 3, INV> {};
template <bool INV> struct Dft<10, INV> : DftComp<2, 5, INV> {};
template <bool INV> struct Dft<12, INV> : DftComp<4, 3, INV> {};
template <bool INV> struct Dft<15, INV> : DftComp<3, 5, INV> {};
template <bool INV> struct Dft<16, INV> : DftComp<4, 4, INV> {};
template <bool INV> struct Dft<18, INV> : DftComp<2, 9, INV> {};
template <bool INV> struct Dft<20, INV> : DftComp<4, 5, INV> {};
template <bool INV> struct Dft<24, INV> : DftComp<8, 3, INV> {};

// Radices the planner may use, largest first.
constexpr int kRadices[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
constexpr int kMaxStages = 12;

// Factor n into supported radices (largest first).  Returns the stage count,
// or 0 if n has a prime factor other than 2, 3, 5.
__host__ inline int fft_plan_radices(int n, int* radices) {
  int count = 0;
  while (n > 1) {
    bool found = false;
    for (int r : kRadices) {
      if (n % r == 0) {
        if (count >= kMaxStages) return 0;
        radices[count++] = r;
        n /= r;
        found = true;
        break;
      }
    }
    if (!found) return 0;
  }
  return count;
}

// One Stockham stage on C interleaved sequences of length N, element (s, n)
// at src[n * C + s].  Butterfly b covers sequence s = b % C and index
// j = b / C; it reads src[(j + r N/R) C + s], r < R, applies w^{r k},
// k = j mod Ns, with w = exp(-+2 pi i / (Ns R)), and writes output q to
// dst[((j / Ns) Ns R + k + q Ns) C + s].  Ns is the product of the radices of
// the earlier stages; tw[m] = exp(-2 pi i m / N) for m < N.  Stages are out of
// place (src and dst alternate), so a thread only holds one butterfly.
template <int R, int NT, bool INV>
__device__ inline void stockham_stage(const cpx* __restrict__ src, cpx* __restrict__ dst, int N, int C, int logC,
                                      int Ns, const cpx* __restrict__ tw) {
  const int nb = N / R;
  const int total = nb * C;
  const int twstep = N / (Ns * R);
  for (int b = threadIdx.x; b < total; b += NT) {
    const int s = b & (C - 1);
    const int j = b >> logC;
    const int k = j % Ns;
    cpx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(j + r * nb) * C + s];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cpx w = tw[r * k * twstep];
        v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
      }
    }
    Dft<R, INV>::run(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[(base + q * Ns) * C + s] = v[q];
  }
  __syncthreads();
}

// All stages of one transform on data in buf0; returns the buffer (buf0 or
// buf1) that holds the result.  radices/nstages come from fft_plan_radices.
// The caller must have synchronised after writing buf0.
template <int NT, bool INV>
__device__ inline cpx* fft_lds(cpx* buf0, cpx* buf1, int N, int C, int logC, const int* radices, int nstages,
                               const cpx* __restrict__ tw) {
  int Ns = 1;
  cpx* src = buf0;
  cpx* dst = buf1;
  for (int st = 0; st < nstages; ++st) {
    const int R = radices[st];
    switch (R) {
#define CHRF_STAGE(RR) \
  case RR: stockham_stage<RR, NT, INV>(src, dst, N, C, logC, Ns, tw); break;
      CHRF_STAGE(16) CHRF_STAGE(15) CHRF_STAGE(12) CHRF_STAGE(10) CHRF_STAGE(9) CHRF_STAGE(8)
      CHRF_STAGE(6) CHRF_STAGE(5) CHRF_STAGE(4) CHRF_STAGE(3) CHRF_STAGE(2)
#undef CHRF_STAGE
      default: break;
    }
    Ns *= R;
    cpx* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// ---------------------------------------------------------------------------
// Compile-time three-stage transform for the tuned sizes.  C sequences of
// length N = R1 R2 R3 are interleaved as element (s, n) -> n * C + s.  A
// butterfly b = tid + i * NT of a stage with radix R covers sequence
// s = b % C and index j = b / C.
//   in : v1[i][r] = element (s, j + r N/R1) of the stage-1 butterfly b
//   out: v3[i][q] = element (s, j + q N/R3) of the stage-3 butterfly b
// Stage 1 reads its inputs from registers and stage 3 leaves its outputs in
// registers, so the caller loads from and stores to HBM directly; only the
// two inner exchanges go through LDS (lds_padded_size(C * N) values, in place).  A transform
// whose R1 equals the R3 of the previous one consumes that one's v3 as is.
// tw[m] = exp(-2 pi i m / N).
// ---------------------------------------------------------------------------
// LDS index with one padding slot per 32 complex values: the Stockham stages
// write with strides of R or R * C elements, which without padding would send
// every lane of a wave to the same few banks.
// The padding period is a parameter of the transform (2^PAD values per
// slot; PAD = 0: no padding): the column transforms take the layout with the
// fewest bank conflicts for their stride pattern.
template <int PAD = 5>
__host__ __device__ constexpr int lds_pad(int i) {
  if constexpr (PAD == 0)
    return i;
  else
    return i + (i >> PAD);
}
__host__ __device__ constexpr int lds_padded_size(int n, int pad = 5) { return n + (pad ? (n >> pad) : 0) + 1; }

// lds_pad(x + r S) from p0 = lds_pad(x): when the stride S is a multiple of
// the padding period the padding grows by exactly S / 2^PAD per step, so the
// address is p0 plus a compile-time offset (no per-access shift and add).
template <int S, int PAD = 5>
__device__ inline int strided_pad(int p0, int x, int r) {
  if constexpr (PAD == 0) {
    return p0 + r * S;
  } else if constexpr (S % (1 << PAD) == 0) {
    return p0 + r * (S + (S >> PAD));
  } else {
    return lds_pad<PAD>(x + r * S);
  }
}

template <int N, int C, int NT, int R1, int R2, int R3, bool INV, int PAD = 5>
struct Fft3 {
  static_assert(R1 * R2 * R3 == N, "radices must multiply to N");
  static constexpr int B1 = C * N / R1, B2 = C * N / R2, B3 = C * N / R3;
  static constexpr int M1 = (B1 + NT - 1) / NT, M2 = (B2 + NT - 1) / NT, M3 = (B3 + NT - 1) / NT;

  template <bool COPIES>
  __device__ static inline void stage_barrier() {
    if constexpr (COPIES)
      lds_barrier_copies_in_flight();
    else
      lds_barrier();
  }

  __device__ static inline cpx twid(const cpx* __restrict__ tw, int m) {
    const cpx w = tw[m];
    return INV ? cpx{w.x, -w.y} : w;
  }

  // Twiddle w^r applied to input r of a butterfly: TABLE reads every power
  // from the table (index arithmetic and a load, for LDS-resident tables of
  // VALU-bound callers); otherwise one table entry is raised by repeated
  // multiplication (error grows by about one rounding per power, < 1e-6 for
  // R <= 16), which keeps memory reads to one per stage.
  template <int R, bool TABLE>
  __device__ static inline void apply_twiddles(cpx (&v)[R], const cpx* __restrict__ tw, int step) {
    if constexpr (TABLE) {
      int m = step;
#pragma unroll
      for (int r = 1; r < R; ++r, m += step) v[r] = INV ? cmulc(v[r], tw[m]) : cmul(v[r], tw[m]);
    } else {
      apply_twiddle_powers(v, twid(tw, step));
    }
  }
  // The value is pinned where it is used: an early-loaded twiddle would
  // otherwise have all its powers formed early and kept live.
  __device__ static inline cpx pinned(cpx w) {
    asm volatile("" : "+v"(w.x), "+v"(w.y));
    return w;
  }
  // Makes the early twiddle loads complete here, before the hook starts
  // loads of its own: a later wait for them would also wait for those.
  template <int A, int B>
  __device__ static inline void settle_twiddles(cpx (&w2)[A], cpx (&w3)[B]) {
#pragma unroll
    for (int i = 0; i < A; ++i) w2[i] = pinned(w2[i]);
#pragma unroll
    for (int i = 0; i < B; ++i) w3[i] = pinned(w3[i]);
  }
  template <int R>
  __device__ static inline void apply_twiddle_powers(cpx (&v)[R], cpx w) {
    cpx wr = w;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = cmul(v[r], wr);
      wr = cmul(wr, w);
    }
  }

  // tid is the thread index; callers inside loops may pass an opaque copy so
  // that the per-stage LDS addresses are not hoisted and kept live.
  template <bool TABLE = false>
  __device__ static inline void run(cpx (&v1)[M1][R1], cpx (&v3)[M3][R3], cpx* lds, const cpx* __restrict__ tw,
                                    int tid = threadIdx.x) {
    run_hooked<TABLE, 1>(v1, v3, lds, tw, [] {}, tid);
  }

  // The stage-2 and stage-3 twiddles of this thread (one table entry each;
  // their powers are formed where they are applied).
  struct StageTw {
    cpx w2[M2], w3[M3];
  };
  __device__ static inline StageTw stage_twiddles_of(const cpx* __restrict__ tw, int tid) {
    StageTw t;
#pragma unroll
    for (int i = 0; i < M2; ++i) {
      const int b = tid + i * NT;
      t.w2[i] = (B2 % NT == 0 || b < B2) ? twid(tw, ((b / C) % R1) * (N / (R1 * R2))) : cpx{1.f, 0.f};
    }
#pragma unroll
    for (int i = 0; i < M3; ++i) {
      const int b = tid + i * NT;
      t.w3[i] = (B3 % NT == 0 || b < B3) ? twid(tw, b / C) : cpx{1.f, 0.f};
    }
    return t;
  }

  // As run(), calling hook() once stage AT (1 or 2) has written its outputs
  // to LDS, for callers that start the loads of their next transform there.
  // EARLY_TW is for hooks that start copies into LDS: the stage-2 and
  // stage-3 twiddles are read before stage 1 and settled before the hook, so
  // that no vector-memory wait after it waits on the copies too (vector-memory
  // loads complete in issue order), and the stage barriers after the hook do
  // not wait for them either.
  template <bool TABLE, int AT, bool EARLY_TW = false, class Hook>
  __device__ static inline void run_hooked(cpx (&v1)[M1][R1], cpx (&v3)[M3][R3], cpx* lds,
                                           const cpx* __restrict__ tw, Hook&& hook, int tid = threadIdx.x) {
    static_assert(!(EARLY_TW && TABLE), "early twiddles are single table entries");
    run_core<TABLE, AT, EARLY_TW ? 1 : 0>(v1, v3, lds, tw, hook, tid,
                                            EARLY_TW ? stage_twiddles_of(tw, tid) : StageTw{});
  }

  // As run(), with the stage twiddles read beforehand (stage_twiddles_of):
  // for transforms in a loop whose twiddles do not change, so that the loop
  // issues no vector-memory load that would wait on its earlier stores.
  __device__ static inline void run_with_twiddles(cpx (&v1)[M1][R1], cpx (&v3)[M3][R3], cpx* lds, const StageTw& t,
                                                  int tid) {
    run_core<false, 1, 2>(v1, v3, lds, nullptr, [] {}, tid, t);
  }

  // MODE 0: twiddles read in their stage; 1: read early, settled before the
  // hook, copy-tolerant stage barriers after it; 2: supplied by the caller.
  template <bool TABLE, int AT, int MODE, class Hook>
  __device__ static inline void run_core(cpx (&v1)[M1][R1], cpx (&v3)[M3][R3], cpx* lds, const cpx* __restrict__ tw,
                                         Hook&& hook, int tid, StageTw t) {
    static_assert(AT == 1 || AT == 2, "hook after stage 1 or 2");
    constexpr bool EARLY_TW = MODE == 1, GIVEN_TW = MODE >= 1;
    // stage 1 (Ns = 1): no twiddles; output q of butterfly j goes to j R1 + q
#pragma unroll
    for (int i = 0; i < M1; ++i) {
      const int b = tid + i * NT;
      if (B1 % NT == 0 || b < B1) {
        const int s = b % C, j = b / C;
        Dft<R1, INV>::run(v1[i]);
        if constexpr (PAD == 0) {
          const int p0 = j * R1 * C + s;
#pragma unroll
          for (int q = 0; q < R1; ++q) lds[p0 + q * C] = v1[i][q];
        } else if constexpr ((R1 * C) % (1 << PAD) == 0 && (1 << PAD) % C == 0) {
          // j R1 C is a multiple of the period and q C + s never crosses one past it
          const int p0 = lds_pad<PAD>(j * R1 * C) + s;
#pragma unroll
          for (int q = 0; q < R1; ++q) lds[p0 + q * C + ((q * C) >> PAD)] = v1[i][q];
        } else {
#pragma unroll
          for (int q = 0; q < R1; ++q) lds[lds_pad<PAD>((j * R1 + q) * C + s)] = v1[i][q];
        }
      }
    }
    lds_barrier();
    if constexpr (AT == 1) {
      if constexpr (EARLY_TW) settle_twiddles(t.w2, t.w3);
      hook();
    }
    // stage 2 (Ns = R1)
    cpx v2[M2][R2];
#pragma unroll
    for (int i = 0; i < M2; ++i) {
      const int b = tid + i * NT;
      if (B2 % NT == 0 || b < B2) {
        const int s = b % C, j = b / C, k = j % R1;
        const int p0 = lds_pad<PAD>(j * C + s);
#pragma unroll
        for (int r = 0; r < R2; ++r)
          v2[i][r] = lds[strided_pad<(N / R2) * C, PAD>(p0, j * C + s, r)];
        if constexpr (GIVEN_TW)
          apply_twiddle_powers(v2[i], pinned(t.w2[i]));
        else
          apply_twiddles<R2, TABLE>(v2[i], tw, k * (N / (R1 * R2)));
        Dft<R2, INV>::run(v2[i]);
      }
    }
    stage_barrier<EARLY_TW>();
#pragma unroll
    for (int i = 0; i < M2; ++i) {
      const int b = tid + i * NT;
      if (B2 % NT == 0 || b < B2) {
        const int s = b % C, j = b / C, k = j % R1;
        const int base = (j - k) * R2 + k;
        const int p0 = lds_pad<PAD>(base * C + s);
#pragma unroll
        for (int q = 0; q < R2; ++q) lds[strided_pad<R1 * C, PAD>(p0, base * C + s, q)] = v2[i][q];
      }
    }
    stage_barrier<EARLY_TW>();
    if constexpr (AT == 2) {
      if constexpr (EARLY_TW) settle_twiddles(t.w2, t.w3);
      hook();
    }
    // stage 3 (Ns = R1 R2 = N / R3): j < Ns, so k = j and outputs land at j + q N/R3
#pragma unroll
    for (int i = 0; i < M3; ++i) {
      const int b = tid + i * NT;
      if (B3 % NT == 0 || b < B3) {
        const int s = b % C, j = b / C;
        const int p0 = lds_pad<PAD>(j * C + s);
#pragma unroll
        for (int r = 0; r < R3; ++r) v3[i][r] = lds[strided_pad<(N / R3) * C, PAD>(p0, j * C + s, r)];
        if constexpr (GIVEN_TW)
          apply_twiddle_powers(v3[i], pinned(t.w3[i]));
        else
          apply_twiddles<R3, TABLE>(v3[i], tw, j);
        Dft<R3, INV>::run(v3[i]);
      }
    }
    stage_barrier<EARLY_TW>();   // LDS is free again for the caller
  }
};

}  // namespace chrf
